// Block Lanczos engine: allocation, the launch sequence of both passes, the
// job tables of a batch and the pass transitions.
#include "block.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace csvd {

// Chunks of stored bases that no solve is using, per device, kept for the
// next solve: freeing and re-allocating tens of GB per solve stalls the
// device while the driver clears the memory.  Idle chunks are freed when a
// new chunk would not leave kStoreReserve free, when any other device
// allocation runs out of memory (DevBuf::alloc), and by csvd_trim.  The
// pool lives until the process ends (never destroyed: it may hold device
// memory past the runtime's own teardown).
namespace {
struct ChunkPool {
  std::mutex mu;
  std::map<int, std::vector<std::unique_ptr<DevBuf>>> idle;  // device -> idle chunks
};
ChunkPool &chunk_pool() {
  static ChunkPool *p = new ChunkPool();
  return *p;
}
int current_device() {
  int d = 0;
  return hipGetDevice(&d) == hipSuccess ? d : 0;
}
}  // namespace

void release_idle_chunks() {
  ChunkPool &p = chunk_pool();
  std::lock_guard<std::mutex> g(p.mu);
  p.idle[current_device()].clear();
}

static int lp_bit(int Lp) { return Lp == 16 ? 1 : (Lp == 32 ? 2 : 4); }

hipError_t LongRows::build(const std::vector<int> &rowptr, hipStream_t st) {
  std::vector<int> b, e, r, ls(1, 0);
  nnz_long = 0;
  for (size_t i = 0; i + 1 < rowptr.size(); ++i) {
    const int s0 = rowptr[i], s1 = rowptr[i + 1];
    if (s1 - s0 <= kLongRow) continue;
    r.push_back((int)i);
    for (int p = s0; p < s1; p += kLongRow) {
      b.push_back(p);
      e.push_back(std::min(p + kLongRow, s1));
    }
    ls.push_back((int)b.size());
    nnz_long += s1 - s0;
  }
  nseg = (int)b.size();
  nlong = (int)r.size();
  hipError_t err;
  if ((err = sgb.alloc(sizeof(int) * std::max(nseg, 1))) != hipSuccess) return err;
  if ((err = sge.alloc(sizeof(int) * std::max(nseg, 1))) != hipSuccess) return err;
  if ((err = lrow.alloc(sizeof(int) * std::max(nlong, 1))) != hipSuccess) return err;
  if ((err = lseg.alloc(sizeof(int) * (nlong + 1))) != hipSuccess) return err;
  if (nseg > 0) {
    if ((err = hipMemcpyAsync(sgb.p, b.data(), sizeof(int) * nseg, hipMemcpyHostToDevice, st)) != hipSuccess) return err;
    if ((err = hipMemcpyAsync(sge.p, e.data(), sizeof(int) * nseg, hipMemcpyHostToDevice, st)) != hipSuccess) return err;
    if ((err = hipMemcpyAsync(lrow.p, r.data(), sizeof(int) * nlong, hipMemcpyHostToDevice, st)) != hipSuccess)
      return err;
  }
  if ((err = hipMemcpyAsync(lseg.p, ls.data(), sizeof(int) * (nlong + 1), hipMemcpyHostToDevice, st)) != hipSuccess)
    return err;
  return hipStreamSynchronize(st);  // the host vectors are temporaries
}

// Tiles of the block sparse products: rows with few nonzeros (G = 1) are
// handled four columns per lane, kThreads / (Lp / 4) rows per tile.
// The lane split G follows the mean length of the rows the tiles compute
// (rows longer than kLongRow are summed from segments); the tiles cover all
// rows.
static Tiling block_tiling(int64_t rows, int64_t nnz, int Lp, int64_t long_rows = 0, int64_t long_nnz = 0) {
  const int64_t sr = std::max<int64_t>(rows - long_rows, 1);
  Tiling t = tiling_for(rows, (nnz - long_nnz) * rows / sr, Lp);
  if (t.G == 1) {
    t.E = 1;
    t.rpt = kThreads * 4 / Lp;
    t.tiles = (int)((rows + t.rpt - 1) / t.rpt);
  }
  return t;
}

// Workgroups of the tall kernels (one per CU, each walking its share of the
// rows): the per-shift recurrences of the previous step (one workgroup per
// shift) run beside them on the side stream, and a tall workgroup cannot
// share a CU with one, so the tall kernels leave those CUs out.
static int tall_workgroups(int64_t n, int S) {
  const int64_t cap = std::max<int64_t>(kBlockMaxVB - S, kBlockMaxVB / 4);
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlockPanel - 1) / kBlockPanel, cap));
}

size_t BlockJob::bytes_needed(int64_t m, int64_t n, int64_t nnz, int Lp, int S, int Kcap, int L, int Kmom) {
  (void)nnz;
  const int64_t L2 = (int64_t)Lp * Lp;
  const int64_t nvb = tall_workgroups(n, S);
  size_t b = 0;
  b += 8 * (size_t)(m * Lp);                       // U
  b += 8 * (size_t)((kMomWindow + 2 + 2) * n * Lp);  // Q ring, W, Vpad
  b += 8 * (size_t)(nvb * 2 * L2);                 // partial Gram matrices
  b += 8 * (size_t)(7 * L2);                       // reduced Gram matrices, R1, R1^-1, T
  b += 8 * (size_t)(5 * (Kcap + 1) * L2);          // A, B, M, N, P histories
  b += 16 * (size_t)(2 * S * (Kcap + 1) * L2);     // Hinv, Z histories
  b += 16 * (size_t)(2 * S * L2);                  // complex scratch
  b += 8 * (size_t)(S * Lp) + 8 * Lp + 16 * 4;     // res, beta0, counters
  b += 8 * (size_t)((int64_t)Kcap * Kmom * L * Lp);  // moment coefficients
  b += 8 * (size_t)(2 * n * Lp + Lp + 2 * hh_blocked_ws_doubles(Lp));  // Householder QR of a block
  b += 256 * 40;
  return b;
}

hipError_t BlockJob::create(const int *rp, const int *ci, const double *va, const int *rpT, const int *ciT,
                            const double *vaT, int64_t m, int64_t n, int64_t nnz, int L, int Lp, int S, int Kcap_,
                            int Kmom, double tol, const std::vector<double> &sre, const std::vector<double> &sim,
                            const std::vector<double> &cre, const std::vector<double> &cim, int cstride,
                            hipStream_t st, const LongRows *lr) {
  Kcap = Kcap_;
  const int64_t L2 = (int64_t)Lp * Lp;
  hipError_t e = mem.alloc(bytes_needed(m, n, nnz, Lp, S, Kcap, L, Kmom));
  if (e != hipSuccess) return e;
  char *base = mem.as<char>();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    char *p = base + off;
    off += bytes;
    return (void *)p;
  };
  BJobDesc &J = h;
  std::memset(&J, 0, sizeof(J));
  J.rp = rp; J.ci = ci; J.va = va; J.rpT = rpT; J.ciT = ciT; J.vaT = vaT;
  J.m = (int)m; J.n = (int)n; J.Lp = Lp; J.lgLp = ilog2i(Lp); J.L = L; J.S = S;
  J.npad = (int)round_up(n, kRowPad);
  // the row tiles hold the rows up to kLongRow nonzeros; longer rows are
  // summed from segments (lr[0]: rows of A, lr[1]: rows of A^T)
  const Tiling t1 = block_tiling(m, nnz, Lp, lr ? lr[0].nlong : 0, lr ? lr[0].nnz_long : 0);
  const Tiling t2 = block_tiling(n, nnz, Lp, lr ? lr[1].nlong : 0, lr ? lr[1].nnz_long : 0);
  J.G1 = t1.G; J.lgG1 = t1.lgG; J.E1 = t1.E; J.rpt1 = t1.rpt; J.tiles1 = t1.tiles;
  J.G2 = t2.G; J.lgG2 = t2.lgG; J.E2 = t2.E; J.rpt2 = t2.rpt; J.tiles2 = t2.tiles;
  J.nchunk = (int)((n + kBlockPanel - 1) / kBlockPanel);
  J.nvb = tall_workgroups(n, S);
  J.Kcap = Kcap;
  J.Kmom = Kmom;
  J.cstride = cstride;
  J.tol = tol;
  J.U = (double *)take(8 * (size_t)(m * Lp));
  J.nring = kMomWindow + 2;
  J.Q = (double *)take(8 * (size_t)(J.nring * n * Lp));
  J.qC = J.nring;
  J.qT = 1;
  J.W = (double *)take(8 * (size_t)(n * Lp));
  J.Vpad = (double *)take(8 * (size_t)(n * Lp));
  J.gpart = (double *)take(8 * (size_t)(J.nvb * 2 * L2));
  J.red = (double *)take(8 * 4 * L2);
  J.scr = (double *)take(8 * 3 * L2);
  J.Ah = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Bh = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Mh = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Nh = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Ph = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Hinv = (double2 *)take(16 * (size_t)(S * (Kcap + 1) * L2));
  J.Zh = (double2 *)take(16 * (size_t)(S * (Kcap + 1) * L2));
  J.ctmp = (double2 *)take(16 * (size_t)(2 * S * L2));
  J.res = (double *)take(8 * (size_t)(S * Lp));
  J.beta0 = (double *)take(8 * (size_t)Lp);
  J.active = (int *)take(4 * 4);
  J.flags = (int *)take(4 * 4);
  J.F = (double *)take(8 * (size_t)((int64_t)Kcap * Kmom * L * Lp));
  orth_x = (double *)take(8 * (size_t)(n * Lp));
  orth_z = (double *)take(8 * (size_t)(n * Lp));
  orth_tau = (double *)take(8 * (size_t)Lp);
  orth_ws = (double *)take(8 * (size_t)hh_blocked_ws_doubles(Lp));
  orth_ws2 = (double *)take(8 * (size_t)hh_blocked_ws_doubles(Lp));
  if (off > mem.bytes) return hipErrorOutOfMemory;
  J.tlong = lr ? kLongRow : 0x7fffffff;  // without segment tables every row is tiled
  if (lr) {
    J.sgb1 = lr[0].sgb.as<int>(); J.sge1 = lr[0].sge.as<int>(); J.lrow1 = lr[0].lrow.as<int>();
    J.lseg1 = lr[0].lseg.as<int>(); J.nseg1 = lr[0].nseg; J.nlong1 = lr[0].nlong;
    J.sgb2 = lr[1].sgb.as<int>(); J.sge2 = lr[1].sge.as<int>(); J.lrow2 = lr[1].lrow.as<int>();
    J.lseg2 = lr[1].lseg.as<int>(); J.nseg2 = lr[1].nseg; J.nlong2 = lr[1].nlong;
  }
  if (J.nseg1 + J.nseg2 > 0) {
    e = seg_part.alloc(8 * (size_t)(J.nseg1 + J.nseg2) * Lp);
    if (e != hipSuccess) return e;
    J.sgp1 = seg_part.as<double>();
    J.sgp2 = J.sgp1 + (size_t)J.nseg1 * Lp;
  }
  // shifts and moment coefficients
  e = d_shift.alloc(sizeof(double2) * S);
  if (e != hipSuccess) return e;
  e = d_cmom.alloc(sizeof(double2) * cre.size());
  if (e != hipSuccess) return e;
  std::vector<double> sh(2 * S), cc(2 * cre.size());
  for (int s = 0; s < S; ++s) {
    sh[2 * s] = sre[s];
    sh[2 * s + 1] = sim[s];
  }
  for (size_t i = 0; i < cre.size(); ++i) {
    cc[2 * i] = cre[i];
    cc[2 * i + 1] = cim[i];
  }
  e = hipMemcpyAsync(d_shift.p, sh.data(), sizeof(double) * sh.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(d_cmom.p, cc.data(), sizeof(double) * cc.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  J.shift = d_shift.as<double2>();
  J.cmom = d_cmom.as<double2>();
  e = hipMemsetAsync(J.flags, 0, 16, st);
  if (e != hipSuccess) return e;
  // basis table: room for the stored basis of Kcap + 2 blocks; ring mode
  qtab.assign((size_t)(Kcap + 2 + kStoreChunk - 1) / kStoreChunk + 1, nullptr);
  e = d_qtab.alloc(sizeof(double *) * qtab.size());
  if (e != hipSuccess) return e;
  J.Qtab = d_qtab.as<double *>();
  q32tab.assign(qtab.size(), nullptr);
  e = d_q32tab.alloc(sizeof(float *) * q32tab.size());
  if (e != hipSuccess) return e;
  J.Q32tab = d_q32tab.as<float *>();
  J.store32 = 0;
  J.sL = L;
  J.soff = 0;
  if ((e = set_ring(st)) != hipSuccess) return e;
  // solo tables: one job
  e = d_desc.alloc(sizeof(BJobDesc));
  if (e != hipSuccess) return e;
  e = d_toff.alloc(sizeof(int) * 8);
  if (e != hipSuccess) return e;
  const int toff[8] = {0, J.tiles1, 0, J.tiles2, 0, J.nvb, 0, S};
  e = hipMemcpyAsync(d_toff.p, toff, sizeof(toff), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  int *dt = d_toff.as<int>();
  solo.jobs = d_desc.as<BJobDesc>();
  solo.njob = 1;
  solo.toff1 = dt;
  solo.toff2 = dt + 2;
  solo.toffr = dt + 4;
  solo.toffs = dt + 6;
  solo.total1 = J.tiles1;
  solo.total2 = J.tiles2;
  solo.totalr = J.nvb;
  solo.totals = S;
  solo.lpmask = lp_bit(Lp);
  return hipStreamSynchronize(st);  // host vectors are temporaries
}

hipError_t BlockJob::set_ring(hipStream_t st) {
  h.qC = h.nring;
  h.qT = 1;
  h.store32 = 0;
  std::fill(qtab.begin(), qtab.end(), nullptr);
  qtab[0] = h.Q;
  store = false;
  hipError_t e = hipMemcpyAsync(d_qtab.p, qtab.data(), sizeof(double *) * qtab.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

bool BlockJob::grow_store(int kneed, hipStream_t st) {
  if (store_cap > 0 && kneed >= store_cap) return false;  // blocks 0 .. kneed would pass the cap
  const size_t esz = mixed ? sizeof(float) : sizeof(double);
  const size_t bytes = esz * (size_t)kStoreChunk * h.n * h.Lp;
  bool changed = false;
  while ((int64_t)chunks.size() * kStoreChunk <= kneed) {
    if (chunks.size() + 1 >= qtab.size()) return false;
    std::unique_ptr<DevBuf> c;
    {
      ChunkPool &p = chunk_pool();
      std::lock_guard<std::mutex> g(p.mu);
      auto &idle = p.idle[current_device()];
      for (size_t i = idle.size(); i-- > 0;)
        if (idle[i]->bytes == bytes) {
          c = std::move(idle[i]);
          idle.erase(idle.begin() + (std::ptrdiff_t)i);
          break;
        }
      if (!c) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
        if (fr < bytes + kStoreReserve && !idle.empty()) {
          idle.clear();  // idle chunks of other widths make room
          if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
        }
        if (fr < bytes + kStoreReserve) return false;
        c.reset(new DevBuf());
        if (c->alloc(bytes, false) != hipSuccess) return false;  // the pool's lock is held
      }
    }
    if (mixed) q32tab[chunks.size()] = c->as<float>();
    else qtab[chunks.size()] = c->as<double>();
    chunks.push_back(std::move(c));
    changed = true;
  }
  if (changed) {
    const hipError_t ec = mixed ? hipMemcpyAsync(d_q32tab.p, q32tab.data(), sizeof(float *) * q32tab.size(),
                                                 hipMemcpyHostToDevice, st)
                                : hipMemcpyAsync(d_qtab.p, qtab.data(), sizeof(double *) * qtab.size(),
                                                 hipMemcpyHostToDevice, st);
    if (ec != hipSuccess) return false;
    if (hipStreamSynchronize(st) != hipSuccess) return false;
  }
  return true;
}

void BlockJob::free_store(bool keep) {
  if (keep && !chunks.empty()) {
    ChunkPool &p = chunk_pool();
    std::lock_guard<std::mutex> g(p.mu);
    auto &idle = p.idle[current_device()];
    for (auto &c : chunks) idle.push_back(std::move(c));
  }
  chunks.clear();
}

hipError_t BlockJob::sync_desc(hipStream_t st) {
  hipError_t e = hipMemcpyAsync(d_desc.p, &h, sizeof(BJobDesc), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);  // `h` may change before the copy runs otherwise
}

// ------------------------------------------------------------------ engine
hipError_t BEngine::init() {
  hipError_t e = hipStreamCreateWithFlags(&side_, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  {
    // step graphs are opt-in: replays measured slower than eager launches
    // (each step kernel then waits on a dependent load of the clock, and the
    // host already runs ahead of the device)
    const char *v = std::getenv("CSVD_STEP_GRAPH");
    graphs_ = (v && v[0] == '1');
  }
  if ((e = hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking)) != hipSuccess) return e;
  if ((e = clk_.alloc(sizeof(int64_t))) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&ev_, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&snap_main_, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&snap_side_, hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

BEngine::~BEngine() {
  if (side_) {
    (void)hipStreamSynchronize(side_);
    (void)hipStreamDestroy(side_);
  }
  (void)hipStreamSynchronize(st_);
  if (gexec_) (void)hipGraphExecDestroy(gexec_);
  if (cap_) (void)hipStreamDestroy(cap_);
  if (ev_) (void)hipEventDestroy(ev_);
  if (snap_main_) (void)hipEventDestroy(snap_main_);
  if (snap_side_) (void)hipEventDestroy(snap_side_);
  if (snap_host_) (void)hipHostFree(snap_host_);
}

// the shift recurrences of the current step on the side stream, after the
// main stream has produced B_{k+1} (init: the starting Z_0 = B_0)
hipError_t BEngine::launch_shift(const BBatch &b, int init) {
  hipError_t e = hipEventRecord(ev_, st_);
  if (e != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(side_, ev_, 0)) != hipSuccess) return e;
  return launch_b_shift(b, init, side_);
}

// Householder QR of Vpad gives Q_0 and R_0 = B_0; Z_0 = R_0 for every shift.
hipError_t BEngine::start(BlockJob *j) {
  BJobDesc &J = j->h;
  J.start_clock = (int)clock_;
  J.Kstop = j->Kcap;
  j->pass = 1;
  j->converged = false;
  j->K = 0;
  hipError_t e = hipMemsetAsync(J.Q, 0, 8 * (size_t)J.nring * J.n * J.Lp, st_);
  if (e != hipSuccess) return e;
  // store mode if the first chunks fit (blocks 0 .. kBlockPoll + 1 before the first poll)
  j->free_store(true);
  if ((e = j->set_ring(st_)) != hipSuccess) return e;
  if (j->want_store && j->mixed) {
    // FP32 copies of the blocks in the store, the FP64 recurrence in the ring
    std::fill(j->q32tab.begin(), j->q32tab.end(), nullptr);
    if (j->grow_store(std::min(kBlockPollSteps + 2, j->Kcap + 1), st_)) {
      j->store = true;
      J.store32 = 1;
    } else {
      j->free_store(false);
    }
  } else if (j->want_store) {
    J.qC = kStoreChunk;
    J.qT = (int)j->qtab.size();
    std::fill(j->qtab.begin(), j->qtab.end(), nullptr);
    if (j->grow_store(std::min(kBlockPollSteps + 2, j->Kcap + 1), st_)) {
      j->store = true;
    } else {
      j->free_store(false);
      if ((e = j->set_ring(st_)) != hipSuccess) return e;
    }
  }
  j->stored_last = false;
  e = hipMemsetAsync(J.active, 0, 16, st_);
  if (e != hipSuccess) return e;
  e = j->sync_desc(st_);
  if (e != hipSuccess) return e;
  // one-pass flag, counter and robust-step mark of this round start at zero
  if ((e = hipMemsetAsync(J.flags + 1, 0, 3 * sizeof(int), st_)) != hipSuccess) return e;
  if ((e = start_block(j, true)) != hipSuccess) return e;
  // A numerically rank-deficient starting block (a filtered block with fewer
  // values than columns, a starting guess close to an invariant subspace of
  // lower dimension) makes the first new blocks tiny and ill conditioned,
  // beyond what Cholesky QR resolves: its first steps orthonormalise by
  // Householder QR.  (Rounds after the first always do.)  The test reads the
  // diagonal of B_0 = R from the QR of the starting block.
  if (j->robust_steps == 0) {
    std::vector<double> r((size_t)J.Lp * J.Lp);
    if ((e = hipMemcpyAsync(r.data(), J.Bh, 8 * r.size(), hipMemcpyDeviceToHost, st_)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st_)) != hipSuccess) return e;
    double dmax = 0.0, dmin = HUGE_VAL;
    for (int i = 0; i < J.Lp; ++i) {
      const double d = std::fabs(r[(size_t)i * J.Lp + i]);
      dmax = std::max(dmax, d);
      dmin = std::min(dmin, d);
    }
    if (!(dmin > kRankTol * dmax)) j->robust_steps = kRobustSteps;
  }
  if ((e = launch_b_store32(J, 0, st_)) != hipSuccess) return e;
  BBatch b = j->solo;
  b.clock = clock_;
  if ((e = launch_shift(b, 1)) != hipSuccess) return e;
  p1_.push_back(j);
  dirty1_ = true;
  return hipSuccess;
}

// Householder QR of a row-major n x Lp block: stays orthonormal also when
// the block is numerically rank deficient (a Cholesky QR of such a block
// loses orthogonality).  Deterministic, so a second pass reproduces it bit
// for bit.
// The work buffers are the job's own (taken at create), so a Householder
// step allocates nothing while the engine steps.
hipError_t BEngine::orth_block(BlockJob *j, const double *src, double *dst, double *R, double *norms) {
  BJobDesc &J = j->h;
  const int64_t n = J.n;
  const int Lp = J.Lp;
  hipError_t e;
  double *x = j->orth_x, *z = j->orth_z;
  if ((e = launch_row_to_col((int)n, Lp, src, Lp, x, n, st_)) != hipSuccess) return e;
  if (norms && (e = launch_col_norms(x, n, (int)n, Lp, norms, st_)) != hipSuccess) return e;
  if ((e = hh_qr_blocked(x, n, (int)n, Lp, j->orth_tau, j->orth_ws, st_)) != hipSuccess) return e;
  if (R && (e = launch_b_r0(x, n, Lp, R, st_)) != hipSuccess) return e;
  if ((e = launch_b_eye(z, n, n, Lp, st_)) != hipSuccess) return e;
  if ((e = hh_apply_blocked(x, n, (int)n, Lp, j->orth_ws, z, n, Lp, j->orth_ws2, st_)) != hipSuccess) return e;
  if ((e = launch_col_to_row((int)n, Lp, z, n, dst, Lp, st_)) != hipSuccess) return e;
  return hipStreamSynchronize(st_);
}

// Q_0 (block 0 of the basis) and, on the first pass, B_0 and the column norms
// of the starting block, by Householder QR.
hipError_t BEngine::start_block(BlockJob *j, bool first) {
  BJobDesc &J = j->h;
  return orth_block(j, J.Vpad, j->block_ptr(0), first ? J.Bh : nullptr, first ? J.beta0 : nullptr);
}

// Step 0 of a round without Householder steps.  A starting block close to an
// invariant subspace (a good starting guess) gives new directions many orders
// smaller than the products they come from, and one that mixes invariant and
// other directions gives a first new block of widely different column
// sizes; Cholesky QR of such a block loses the accuracy the shifted solves
// need.  From the reduced Gram matrices of step 0: per column, ||w2_c||^2 =
// G2(c, c) against the squared norm before the projection, ||P(:, c)||^2 +
// G2(c, c) (below kInvTol^2: nearly invariant), and the pivots of the
// Cholesky factorisation of G2 - C^T C = W3^T W3 (smallest over largest
// below kInvTol^2: cond(W3) above 1 / kInvTol).  Either makes the job take
// Householder steps from step 0 on.
hipError_t BEngine::check_first_block(BlockJob *j) {
  const BJobDesc &J = j->h;
  const int Lp = J.Lp;
  const size_t L2 = (size_t)Lp * Lp;
  std::vector<double> red(3 * L2);
  hipError_t e = hipMemcpyAsync(red.data(), J.red, 8 * red.size(), hipMemcpyDeviceToHost, st_);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st_)) != hipSuccess) return e;
  const double *P = red.data(), *C = red.data() + L2, *G2 = red.data() + 2 * L2;
  // G2 holds its upper 16 x 16 tiles: entry (r, c) at (r, c) when the tile of
  // r is not below the tile of c, else at (c, r)
  auto g2 = [&](int r, int c) { return (r >> 4) <= (c >> 4) ? G2[(size_t)r * Lp + c] : G2[(size_t)c * Lp + r]; };
  double worst = HUGE_VAL;
  for (int c = 0; c < Lp; ++c) {
    double own = g2(c, c);
    for (int i = 0; i < Lp; ++i) own += P[(size_t)i * Lp + c] * P[(size_t)i * Lp + c];
    if (own > 0.0) worst = std::min(worst, g2(c, c) / own);
  }
  std::vector<double> M(L2);
  for (int r = 0; r < Lp; ++r)
    for (int c = 0; c < Lp; ++c) {
      double v = g2(r, c);
      for (int i = 0; i < Lp; ++i) v -= C[(size_t)i * Lp + r] * C[(size_t)i * Lp + c];
      M[(size_t)r * Lp + c] = v;
    }
  double pmin = HUGE_VAL, pmax = 0.0;
  for (int c = 0; c < Lp; ++c) {  // right-looking Cholesky, pivots only
    const double d = M[(size_t)c * Lp + c];
    pmin = std::min(pmin, d);
    pmax = std::max(pmax, d);
    if (!(d > 0.0)) break;
    for (int r = c + 1; r < Lp; ++r)
      for (int q = c + 1; q < Lp; ++q) M[(size_t)r * Lp + q] -= M[(size_t)r * Lp + c] * M[(size_t)c * Lp + q] / d;
  }
  if (worst < kInvTol * kInvTol || !(pmin > kInvTol * kInvTol * pmax)) j->robust_steps = kRobustSteps;
  return hipSuccess;
}

// After gamma wrote W3 = W2 - Q_k C into block k + 1 of a robust step:
// Q_{k+1} and (first pass) B_{k+1} = R by Householder QR.
hipError_t BEngine::robust_finish(std::vector<BlockJob *> &v, bool first_pass) {
  for (BlockJob *j : v) {
    const int k = (int)(clock_ - j->h.start_clock);
    if (k >= j->robust_steps || k >= j->h.Kstop) continue;
    double *blk = j->block_ptr(k + 1);
    const size_t L2 = (size_t)j->h.Lp * j->h.Lp;
    hipError_t e = orth_block(j, blk, blk, first_pass ? j->h.Bh + (size_t)(k + 1) * L2 : nullptr, nullptr);
    if (e != hipSuccess) return e;
    if ((e = launch_b_store32(j->h, k + 1, st_)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// zero the job's columns of Sout (all of it, or the Kmom column ranges of a
// column group)
hipError_t BEngine::clear_moments(const BJobDesc &J) {
  if (J.sL == J.L && J.soff == 0)
    return hipMemsetAsync(J.Sout, 0, 8 * (size_t)J.npad * J.Kmom * J.L, st_);
  for (int k = 0; k < J.Kmom; ++k) {
    hipError_t e = hipMemsetAsync(J.Sout + ((size_t)k * J.sL + J.soff) * J.npad, 0, 8 * (size_t)J.npad * J.L, st_);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Store mode: the basis is complete in memory; solve the projected systems
// backwards, form the coefficients and accumulate the moments from the stored
// blocks in the same windows as the second pass would (same bits).
hipError_t BEngine::finish_stored(BlockJob *j) {
  BJobDesc &J = j->h;
  hipError_t e = launch_b_backsolve(J, j->K, st_);
  if (e != hipSuccess) return e;
  if ((e = launch_b_fcoef(J, j->K, st_)) != hipSuccess) return e;
  if ((e = clear_moments(J)) != hipSuccess) return e;
  for (int k0 = 0; k0 < j->K; k0 += kMomWindow) {
    const int T = std::min(kMomWindow, j->K - k0);
    const bool timed = timer_ && T == kMomWindow;
    if (timed && (e = timer_->begin(3, st_)) != hipSuccess) return e;
    if ((e = launch_b_moments(J, k0, T, st_)) != hipSuccess) return e;
    if (timed && (e = timer_->end(st_)) != hipSuccess) return e;
  }
  if ((e = hipStreamSynchronize(st_)) != hipSuccess) return e;
  j->free_store(true);
  j->store = false;
  j->stored_last = true;
  j->pass = 3;
  return j->set_ring(st_);
}

hipError_t BEngine::enter_pass2(BlockJob *j, bool coefficients) {
  BJobDesc &J = j->h;
  hipError_t e;
  if (coefficients) {
    if ((e = launch_b_backsolve(J, j->K, st_)) != hipSuccess) return e;
    if ((e = launch_b_fcoef(J, j->K, st_)) != hipSuccess) return e;
  }
  if ((e = clear_moments(J)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(J.Q, 0, 8 * (size_t)J.nring * J.n * J.Lp, st_)) != hipSuccess) return e;
  J.start_clock = (int)clock_;
  J.Kstop = j->K;
  j->pass = 2;
  j->mflushed = 0;
  if ((e = j->sync_desc(st_)) != hipSuccess) return e;
  if ((e = start_block(j, false)) != hipSuccess) return e;
  p2_.push_back(j);
  dirty2_ = true;
  return hipSuccess;
}

hipError_t BEngine::rebuild(std::vector<BlockJob *> &jobs, DevBuf &dj, DevBuf &dt, BBatch &b) {
  // the side stream may still read the old tables
  hipError_t es = hipStreamSynchronize(side_);
  if (es != hipSuccess) return es;
  if (&b == &b1_ && gexec_) {  // the step graph holds the old tables
    if ((es = hipStreamSynchronize(st_)) != hipSuccess) return es;
    (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
  }
  const int nj = (int)jobs.size();
  std::vector<BJobDesc> descs(nj);
  std::vector<int> toff(4 * (nj + 1), 0);
  int *t1 = &toff[0], *t2 = &toff[nj + 1], *tr = &toff[2 * (nj + 1)], *ts = &toff[3 * (nj + 1)];
  for (int i = 0; i < nj; ++i) {
    descs[i] = jobs[i]->h;
    t1[i + 1] = t1[i] + descs[i].tiles1;
    t2[i + 1] = t2[i] + descs[i].tiles2;
    tr[i + 1] = tr[i] + descs[i].nvb;
    ts[i + 1] = ts[i] + descs[i].S;
  }
  if (dj.bytes < sizeof(BJobDesc) * std::max(nj, 1)) {
    hipError_t e = dj.alloc(sizeof(BJobDesc) * std::max(nj, 1) * 2);
    if (e != hipSuccess) return e;
  }
  if (dt.bytes < sizeof(int) * toff.size()) {
    hipError_t e = dt.alloc(sizeof(int) * toff.size() * 2);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipMemcpyAsync(dj.p, descs.data(), sizeof(BJobDesc) * nj, hipMemcpyHostToDevice, st_);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(dt.p, toff.data(), sizeof(int) * toff.size(), hipMemcpyHostToDevice, st_);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return e;
  int *d = dt.as<int>();
  b.jobs = dj.as<BJobDesc>();
  b.njob = nj;
  b.toff1 = d;
  b.toff2 = d + (nj + 1);
  b.toffr = d + 2 * (nj + 1);
  b.toffs = d + 3 * (nj + 1);
  b.total1 = t1[nj];
  b.total2 = t2[nj];
  b.totalr = tr[nj];
  b.totals = ts[nj];
  b.lpmask = 0;
  for (int i = 0; i < nj; ++i) b.lpmask |= lp_bit(descs[i].Lp);
  return hipSuccess;
}

hipError_t BEngine::step(KernelTimer *timer, bool sample) {
  timer_ = timer;
  hipError_t e;
  if (!p1_.empty()) {
    if (dirty1_) {
      if ((e = flush_shifts()) != hipSuccess) return e;  // with the tables of their steps
      if ((e = rebuild(p1_, dj1_, dt1_, b1_)) != hipSuccess) return e;
      dirty1_ = false;
    }
    b1_.clock = clock_;
    b1_.clkp = nullptr;
    const BBatch &b = b1_;
    if (!(timer && sample) && graph_step_ok()) {
      if (!gexec_ && (e = capture_step()) != hipSuccess) return e;
      if (!clk_synced_ && (e = launch_b_setclock(clk_.as<int64_t>(), clock_, st_)) != hipSuccess) return e;
      if ((e = hipGraphLaunch(gexec_, st_)) != hipSuccess) return e;  // ends with clk_ = clock_ + 1
      clk_synced_ = true;
      ++graph_steps_;
    } else {
      clk_synced_ = false;
      ++eager_steps_;
      if (timer && sample) timer->begin(0, st_);
      if ((e = launch_b_spmm_a(b, st_)) != hipSuccess) return e;
      if ((e = long_rows(p1_, 1)) != hipSuccess) return e;
      if (timer && sample) timer->end(st_);
      if (timer && sample) timer->begin(1, st_);
      if ((e = launch_b_spmm_at(b, st_)) != hipSuccess) return e;
      if ((e = long_rows(p1_, 2)) != hipSuccess) return e;
      if (timer && sample) timer->end(st_);
      if (timer && sample) timer->begin(2, st_);
      if ((e = launch_bs_tall(b, 0, 1, st_)) != hipSuccess) return e;   // W', P
      if ((e = launch_bs_reduce(b, 0, 1, 0, 0, st_)) != hipSuccess) return e;
      if ((e = launch_bs_tall(b, 1, 1, st_)) != hipSuccess) return e;   // C, G2
      if ((e = launch_bs_reduce(b, 0, 2, 1, 0, st_)) != hipSuccess) return e;
      for (BlockJob *j : p1_) {  // mark the robust steps for small1
        const int k = (int)(clock_ - j->h.start_clock);
        if (k == 0 && j->robust_steps == 0 && (e = check_first_block(j)) != hipSuccess) return e;
        if (j->robust_steps > 0 && (k == 0 || k == j->robust_steps) &&
            (e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(j->h.flags + 3), k == 0 ? 1 : 0, 1, st_)) !=
                hipSuccess)
          return e;
      }
      if ((e = launch_bs_small1(b, st_)) != hipSuccess) return e;
      if ((e = launch_bs_tall(b, 2, 1, st_)) != hipSuccess) return e;   // G3
      if ((e = launch_bs_reduce(b, 1, 1, 3, 1, st_)) != hipSuccess) return e;
      if ((e = launch_bs_small2(b, st_)) != hipSuccess) return e;
      if ((e = launch_bs_gamma(b, st_)) != hipSuccess) return e;
      if ((e = robust_finish(p1_, true)) != hipSuccess) return e;
      if (timer && sample) timer->end(st_);
    }
    ++npend_;  // its shift recurrences run at the next poll
  }
  if (!p2_.empty()) {
    if (dirty2_) {
      if ((e = rebuild(p2_, dj2_, dt2_, b2_)) != hipSuccess) return e;
      dirty2_ = false;
    }
    b2_.clock = clock_;
    const BBatch &b = b2_;
    // moments of the last window: S += sum Q_k F_k over kMomWindow steps,
    // before the ring slots of that window are reused
    for (BlockJob *j : p2_) {
      const int k = (int)(clock_ - j->h.start_clock);
      if (k <= j->K && k - j->mflushed == kMomWindow) {
        if ((e = launch_b_moments(j->h, j->mflushed, kMomWindow, st_)) != hipSuccess) return e;
        j->mflushed = k;
      }
    }
    if ((e = launch_b_spmm_a(b, st_)) != hipSuccess) return e;
    if ((e = long_rows(p2_, 1)) != hipSuccess) return e;
    if ((e = launch_b_spmm_at(b, st_)) != hipSuccess) return e;
    if ((e = long_rows(p2_, 2)) != hipSuccess) return e;
    if ((e = launch_bs_tall(b, 0, 0, st_)) != hipSuccess) return e;  // W2 = W - Q_{k-1} B_k^T - Q_k P_k
    if ((e = launch_bs_gamma(b, st_)) != hipSuccess) return e;
    if ((e = robust_finish(p2_, false)) != hipSuccess) return e;
  }
  if (p1_.empty() && p2_.empty()) return hipSuccess;
  ++clock_;
  for (BlockJob *j : p1_) j->steps_total++;
  for (BlockJob *j : p2_) j->steps_total++;
  return hipSuccess;
}

// A pass-1 step is replayed from the graph when no second-pass job shares
// the engine and no job needs host-side work in it: no robust step (their
// marks and Householder QR), no long-row segments (launched per job).
bool BEngine::graph_step_ok() const {
  if (!graphs_ || !p2_.empty()) return false;
  for (const BlockJob *j : p1_) {
    const int k = (int)(clock_ - j->h.start_clock);
    if (k == 0) return false;  // the first step of a pass reads its Gram matrices on the host
    if (j->robust_steps > 0 && k <= j->robust_steps) return false;
    if (j->h.nseg1 + j->h.nseg2 > 0) return false;
  }
  return true;
}

// The step kernels of the batch b (the eager sequence of a plain step, the
// clock read from b.clkp) and the tick, captured on the private stream.
hipError_t BEngine::capture_step() {
  BBatch b = b1_;
  b.clkp = clk_.as<int64_t>();
  hipError_t e = hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t el = step_kernels(b, cap_);
  if (el == hipSuccess) el = launch_b_tick(clk_.as<int64_t>(), cap_);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cap_, &g);
  if (el != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return el;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

hipError_t BEngine::step_kernels(const BBatch &b, hipStream_t st) {
  hipError_t e;
  if ((e = launch_b_spmm_a(b, st)) != hipSuccess) return e;
  if ((e = launch_b_spmm_at(b, st)) != hipSuccess) return e;
  if ((e = launch_bs_tall(b, 0, 1, st)) != hipSuccess) return e;   // W', P
  if ((e = launch_bs_reduce(b, 0, 1, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_bs_tall(b, 1, 1, st)) != hipSuccess) return e;   // C, G2
  if ((e = launch_bs_reduce(b, 0, 2, 1, 0, st)) != hipSuccess) return e;
  if ((e = launch_bs_small1(b, st)) != hipSuccess) return e;
  if ((e = launch_bs_tall(b, 2, 1, st)) != hipSuccess) return e;   // G3
  if ((e = launch_bs_reduce(b, 1, 1, 3, 1, st)) != hipSuccess) return e;
  if ((e = launch_bs_small2(b, st)) != hipSuccess) return e;
  return launch_bs_gamma(b, st);
}

hipError_t BEngine::long_rows(const std::vector<BlockJob *> &v, int side) {
  for (BlockJob *j : v) {
    const BJobDesc &J = j->h;
    const int k = (int)(clock_ - J.start_clock);
    if (k >= J.Kstop || (side == 1 ? J.nseg1 : J.nseg2) == 0) continue;
    hipError_t e = launch_b_spmm_long(J, side, k, st_);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t BEngine::flush_shifts() {
  if (npend_ == 0) return hipSuccess;
  hipError_t e = hipEventRecord(ev_, st_);
  if (e != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(side_, ev_, 0)) != hipSuccess) return e;
  BBatch b = b1_;
  for (int i = npend_; i > 0; --i) {
    b.clock = clock_ - i;
    if ((e = launch_b_shift(b, 0, side_)) != hipSuccess) return e;
  }
  npend_ = 0;
  return hipSuccess;
}

hipError_t BEngine::take_snapshot() {
  snap_.clear();
  if (p1_.empty()) return hipSuccess;
  hipError_t e;
  if (dirty1_) {  // the batch tables list the jobs in the order of p1_
    if ((e = rebuild(p1_, dj1_, dt1_, b1_)) != hipSuccess) return e;
    dirty1_ = false;
  }
  if (p1_.size() > snap_cap_) {
    // nothing writes to the old buffer any more: the events of its last
    // snapshot were waited for
    if (snap_host_) (void)hipHostFree(snap_host_);
    snap_host_ = nullptr;
    snap_cap_ = 0;
    const size_t cap = std::max<size_t>(16, 2 * p1_.size());
    if ((e = hipHostMalloc((void **)&snap_host_, 4 * sizeof(int) * cap, hipHostMallocDefault)) != hipSuccess)
      return e;
    snap_cap_ = cap;
  }
  b1_.clock = clock_;
  if ((e = launch_b_snap(b1_, 0, snap_host_, side_)) != hipSuccess) return e;
  if ((e = launch_b_snap(b1_, 1, snap_host_, st_)) != hipSuccess) return e;
  if ((e = hipEventRecord(snap_main_, st_)) != hipSuccess) return e;
  if ((e = hipEventRecord(snap_side_, side_)) != hipSuccess) return e;
  for (BlockJob *j : p1_) {
    const int steps = (int)(clock_ - j->h.start_clock);
    snap_.push_back({steps > 0 ? j : nullptr, steps});
  }
  return hipSuccess;
}

hipError_t BEngine::poll(std::vector<BlockJob *> *finished) {
  hipError_t e;
  if ((e = flush_shifts()) != hipSuccess) return e;
  // pass-1 jobs that were unconverged after their last step at the previous poll
  std::vector<BlockJob *> ending;
  if (!snap_.empty()) {
    if ((e = hipEventSynchronize(snap_main_)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(snap_side_)) != hipSuccess) return e;
    for (size_t i = 0; i < snap_.size(); ++i) {
      BlockJob *j = snap_[i].j;
      if (!j || j->pass != 1) continue;
      const int *h = snap_host_ + 4 * i;
      const int steps = snap_[i].steps;
      if (h[0] == 0 || steps >= j->Kcap) {
        j->K = std::min(steps, j->Kcap);
        j->steps_last = j->K;
        j->converged = (h[0] == 0);
        j->deflated_last = h[1];
        j->one_pass_last = h[3];
        ending.push_back(j);
      }
    }
    snap_.clear();
  }
  // the next snapshot, of the jobs that go on
  if ((e = take_snapshot()) != hipSuccess) return e;
  for (Snap &x : snap_)
    if (std::find(ending.begin(), ending.end(), x.j) != ending.end()) x.j = nullptr;
  // the shift recurrences of the steps past K may still run on the side
  // stream: they end before the backward solution and a new round's set-up
  if (!ending.empty() && (e = hipStreamSynchronize(side_)) != hipSuccess) return e;
  std::vector<BlockJob *> keep1;
  for (BlockJob *j : p1_) {
    const int steps = (int)(clock_ - j->h.start_clock);
    if (std::find(ending.begin(), ending.end(), j) != ending.end()) {
      dirty1_ = true;
      if (j->store) {
        if ((e = finish_stored(j)) != hipSuccess) return e;
        finished->push_back(j);
      } else if ((e = enter_pass2(j)) != hipSuccess) {
        return e;
      }
    } else {
      // blocks up to Q_{steps + kBlockPoll + 1} exist before the next poll (none past Q_Kcap)
      if (j->store && !j->grow_store(std::min(steps + kBlockPollSteps + 2, j->Kcap + 1), st_)) {
        // out of memory for the stored basis: continue with the ring (blocks
        // Q_{k-1} and Q_k move there; a mixed-precision job has them there
        // already) and regenerate the basis in pass 2
        BJobDesc &J = j->h;
        const size_t blk = sizeof(double) * (size_t)J.n * J.Lp;
        for (int kk = std::max(steps - 1, 0); !j->mixed && kk <= steps; ++kk) {
          const double *src = j->qtab[kk / kStoreChunk] + (size_t)(kk % kStoreChunk) * J.n * J.Lp;
          double *dst = J.Q + (size_t)(kk % J.nring) * J.n * J.Lp;
          if ((e = hipMemcpyAsync(dst, src, blk, hipMemcpyDeviceToDevice, st_)) != hipSuccess) return e;
        }
        if ((e = hipStreamSynchronize(st_)) != hipSuccess) return e;
        j->free_store(false);
        if ((e = j->set_ring(st_)) != hipSuccess) return e;
        if ((e = j->sync_desc(st_)) != hipSuccess) return e;
        dirty1_ = true;
      }
      keep1.push_back(j);
    }
  }
  p1_.swap(keep1);
  std::vector<BlockJob *> keep2;
  for (BlockJob *j : p2_) {
    const int steps = (int)(clock_ - j->h.start_clock);
    if (steps >= j->K) {
      // the rest of the last window (steps past K did no work, so the ring
      // still holds it)
      if (j->mflushed < j->K &&
          (e = launch_b_moments(j->h, j->mflushed, j->K - j->mflushed, st_)) != hipSuccess)
        return e;
      j->mflushed = j->K;
      j->pass = 3;
      finished->push_back(j);
      dirty2_ = true;
    } else {
      keep2.push_back(j);
    }
  }
  p2_.swap(keep2);
  return hipSuccess;
}

void BEngine::remove(BlockJob *j) {
  // the caller frees the job next: no launch may still use it
  (void)flush_shifts();
  (void)hipStreamSynchronize(side_);
  (void)hipStreamSynchronize(st_);
  auto r = [&](std::vector<BlockJob *> &v, bool &dirty) {
    auto it = std::find(v.begin(), v.end(), j);
    if (it != v.end()) {
      v.erase(it);
      dirty = true;
    }
  };
  r(p1_, dirty1_);
  r(p2_, dirty2_);
  for (Snap &x : snap_)
    if (x.j == j) x.j = nullptr;
}

}  // namespace csvd
