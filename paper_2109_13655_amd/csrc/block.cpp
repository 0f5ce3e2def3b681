// Block Lanczos engine: allocation, the launch sequence of both passes, the
// job tables of a batch and the pass transitions.
#include "block.h"

#include <algorithm>
#include <cstring>

namespace csvd {

size_t BlockJob::bytes_needed(int64_t m, int64_t n, int64_t nnz, int Lp, int S, int Kcap, int L, int Kmom) {
  (void)nnz;
  const int64_t L2 = (int64_t)Lp * Lp;
  const int64_t rchunks = (n + kChunk - 1) / kChunk;
  size_t b = 0;
  b += 8 * (size_t)(m * Lp);                       // U
  b += 8 * (size_t)(6 * n * Lp);                   // Q ring, W, W2, Vpad
  b += 8 * (size_t)(rchunks * L2);                 // partial Gram matrices
  b += 8 * (size_t)(3 * L2);                       // G, R1, R1inv
  b += 8 * (size_t)(4 * (Kcap + 1) * L2);          // A, C, B, M histories
  b += 16 * (size_t)(2 * S * (Kcap + 1) * L2);     // Hinv, Z histories
  b += 16 * (size_t)(2 * S * L2);                  // complex scratch
  b += 8 * (size_t)(S * Lp) + 8 * Lp + 16 * 4;     // res, beta0, counters
  b += 8 * (size_t)((int64_t)Kcap * Kmom * L * Lp);  // moment coefficients
  b += 256 * 32;
  return b;
}

hipError_t BlockJob::create(const int *rp, const int *ci, const double *va, const int *rpT, const int *ciT,
                            const double *vaT, int64_t m, int64_t n, int64_t nnz, int L, int Lp, int S, int Kcap_,
                            int Kmom, double tol, const std::vector<double> &sre, const std::vector<double> &sim,
                            const std::vector<double> &cre, const std::vector<double> &cim, int cstride,
                            hipStream_t st) {
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
  const Tiling t1 = tiling_for(m, nnz, Lp), t2 = tiling_for(n, nnz, Lp);
  J.G1 = t1.G; J.lgG1 = t1.lgG; J.E1 = t1.E; J.rpt1 = t1.rpt; J.tiles1 = t1.tiles;
  J.G2 = t2.G; J.lgG2 = t2.lgG; J.E2 = t2.E; J.rpt2 = t2.rpt; J.tiles2 = t2.tiles;
  J.rchunks = (int)((n + kChunk - 1) / kChunk);
  J.Kcap = Kcap;
  J.Kmom = Kmom;
  J.cstride = cstride;
  J.tol = tol;
  J.U = (double *)take(8 * (size_t)(m * Lp));
  J.Q = (double *)take(8 * (size_t)(3 * n * Lp));
  J.W = (double *)take(8 * (size_t)(n * Lp));
  J.W2 = (double *)take(8 * (size_t)(n * Lp));
  J.Vpad = (double *)take(8 * (size_t)(n * Lp));
  J.gpart = (double *)take(8 * (size_t)(J.rchunks * L2));
  J.G = (double *)take(8 * L2);
  J.R1 = (double *)take(8 * L2);
  J.R1inv = (double *)take(8 * L2);
  J.Ah = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Ch = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Bh = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Mh = (double *)take(8 * (size_t)((Kcap + 1) * L2));
  J.Hinv = (double2 *)take(16 * (size_t)(S * (Kcap + 1) * L2));
  J.Zh = (double2 *)take(16 * (size_t)(S * (Kcap + 1) * L2));
  J.ctmp = (double2 *)take(16 * (size_t)(2 * S * L2));
  J.res = (double *)take(8 * (size_t)(S * Lp));
  J.beta0 = (double *)take(8 * (size_t)Lp);
  J.active = (int *)take(4 * 4);
  J.flags = (int *)take(4 * 4);
  J.F = (double *)take(8 * (size_t)((int64_t)Kcap * Kmom * L * Lp));
  if (off > mem.bytes) return hipErrorOutOfMemory;
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
  // solo tables: one job
  e = d_desc.alloc(sizeof(BJobDesc));
  if (e != hipSuccess) return e;
  e = d_toff.alloc(sizeof(int) * 8);
  if (e != hipSuccess) return e;
  const int toff[8] = {0, J.tiles1, 0, J.tiles2, 0, J.rchunks, 0, S};
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
  solo.totalr = J.rchunks;
  solo.totals = S;
  return hipStreamSynchronize(st);  // host vectors are temporaries
}

hipError_t BlockJob::sync_desc(hipStream_t st) {
  hipError_t e = hipMemcpyAsync(d_desc.p, &h, sizeof(BJobDesc), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);  // `h` may change before the copy runs otherwise
}

// ------------------------------------------------------------------ engine
hipError_t BEngine::init() {
  hipError_t e = d_clock_.alloc(sizeof(int64_t));
  if (e != hipSuccess) return e;
  return hipMemsetAsync(d_clock_.p, 0, sizeof(int64_t), st_);
}

// CholeskyQR2 of Vpad gives Q_0 and R_0 = B_0; Z_0 = R_0 for every shift.
hipError_t BEngine::start(BlockJob *j) {
  BJobDesc &J = j->h;
  J.start_clock = (int)clock_;
  J.Kstop = j->Kcap;
  j->pass = 1;
  j->converged = false;
  j->K = 0;
  hipError_t e = hipMemsetAsync(J.Q, 0, 8 * (size_t)3 * J.n * J.Lp, st_);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(J.active, 0, 16, st_);
  if (e != hipSuccess) return e;
  e = j->sync_desc(st_);
  if (e != hipSuccess) return e;
  BBatch b = j->solo;
  b.clock = d_clock_.as<int64_t>();
  if ((e = launch_b_gram(b, BVPAD, BVPAD, 2, st_)) != hipSuccess) return e;
  if ((e = launch_b_chol(b, 1, 1, st_)) != hipSuccess) return e;
  if ((e = launch_b_rowmm(b, BVPAD, BNONE, BW, BM_R1INV, st_)) != hipSuccess) return e;
  if ((e = launch_b_gram(b, BW, BW, 2, st_)) != hipSuccess) return e;
  if ((e = launch_b_chol(b, 2, 1, st_)) != hipSuccess) return e;
  if ((e = launch_b_rowmm(b, BVPAD, BNONE, BQ_CUR, BM_MINIT, st_)) != hipSuccess) return e;
  if ((e = launch_b_shift(b, 1, st_)) != hipSuccess) return e;
  p1_.push_back(j);
  dirty1_ = true;
  return hipSuccess;
}

hipError_t BEngine::enter_pass2(BlockJob *j) {
  BJobDesc &J = j->h;
  hipError_t e = launch_b_backsolve(J, j->K, st_);
  if (e != hipSuccess) return e;
  if ((e = launch_b_fcoef(J, j->K, st_)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(J.Sout, 0, 8 * (size_t)J.npad * J.Kmom * J.L, st_)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(J.Q, 0, 8 * (size_t)3 * J.n * J.Lp, st_)) != hipSuccess) return e;
  J.start_clock = (int)clock_;
  J.Kstop = j->K;
  j->pass = 2;
  if ((e = j->sync_desc(st_)) != hipSuccess) return e;
  BBatch b = j->solo;
  b.clock = d_clock_.as<int64_t>();
  if ((e = launch_b_rowmm(b, BVPAD, BNONE, BQ_CUR, BM_MINIT, st_)) != hipSuccess) return e;
  p2_.push_back(j);
  dirty2_ = true;
  return hipSuccess;
}

hipError_t BEngine::rebuild(std::vector<BlockJob *> &jobs, DevBuf &dj, DevBuf &dt, BBatch &b) {
  const int nj = (int)jobs.size();
  std::vector<BJobDesc> descs(nj);
  std::vector<int> toff(4 * (nj + 1), 0);
  int *t1 = &toff[0], *t2 = &toff[nj + 1], *tr = &toff[2 * (nj + 1)], *ts = &toff[3 * (nj + 1)];
  for (int i = 0; i < nj; ++i) {
    descs[i] = jobs[i]->h;
    t1[i + 1] = t1[i] + descs[i].tiles1;
    t2[i + 1] = t2[i] + descs[i].tiles2;
    tr[i + 1] = tr[i] + descs[i].rchunks;
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
  b.clock = d_clock_.as<int64_t>();
  return hipSuccess;
}

hipError_t BEngine::step(KernelTimer *timer, bool sample) {
  hipError_t e;
  if (!p1_.empty()) {
    if (dirty1_) {
      if ((e = rebuild(p1_, dj1_, dt1_, b1_)) != hipSuccess) return e;
      dirty1_ = false;
    }
    const BBatch &b = b1_;
    if (timer && sample) timer->begin(0, st_);
    if ((e = launch_b_spmm_a(b, st_)) != hipSuccess) return e;
    if (timer && sample) timer->end(st_);
    if (timer && sample) timer->begin(1, st_);
    if ((e = launch_b_spmm_at(b, st_)) != hipSuccess) return e;
    if (timer && sample) timer->end(st_);
    if (timer && sample) timer->begin(2, st_);
    if ((e = launch_b_rowmm(b, BQ_PREV, BW, BW, BM_BK_T, st_)) != hipSuccess) return e;
    if ((e = launch_b_gram(b, BQ_CUR, BW, 0, st_)) != hipSuccess) return e;
    if ((e = launch_b_rowmm(b, BQ_CUR, BW, BW2, BM_AK, st_)) != hipSuccess) return e;
    if ((e = launch_b_gram(b, BQ_CUR, BW2, 1, st_)) != hipSuccess) return e;
    if ((e = launch_b_rowmm(b, BQ_CUR, BW, BW2, BM_AK_CK, st_)) != hipSuccess) return e;
    if ((e = launch_b_gram(b, BW2, BW2, 2, st_)) != hipSuccess) return e;
    if ((e = launch_b_chol(b, 1, 0, st_)) != hipSuccess) return e;
    if ((e = launch_b_rowmm(b, BW2, BNONE, BW, BM_R1INV, st_)) != hipSuccess) return e;
    if ((e = launch_b_gram(b, BW, BW, 2, st_)) != hipSuccess) return e;
    if ((e = launch_b_chol(b, 2, 0, st_)) != hipSuccess) return e;
    if ((e = launch_b_rowmm(b, BW2, BNONE, BQ_NEXT, BM_MK, st_)) != hipSuccess) return e;
    if ((e = launch_b_shift(b, 0, st_)) != hipSuccess) return e;
    if (timer && sample) timer->end(st_);
  }
  if (!p2_.empty()) {
    if (dirty2_) {
      if ((e = rebuild(p2_, dj2_, dt2_, b2_)) != hipSuccess) return e;
      dirty2_ = false;
    }
    const BBatch &b = b2_;
    // moments first: Sout += Q_k F_k uses Q_k before the slot is reused
    for (BlockJob *j : p2_) {
      const BJobDesc &J = j->h;
      const int k = (int)(clock_ - J.start_clock);
      if (k >= j->K) continue;
      const int64_t nL = (int64_t)J.n * J.Lp;
      const int KL = J.Kmom * J.L;
      if ((e = launch_gemm_ta(J.n, KL, J.Lp, 1.0, J.Q + (int64_t)(k % 3) * nL, J.Lp,
                              J.F + (int64_t)k * KL * J.Lp, J.Lp, 1.0, J.Sout, J.npad, st_)) != hipSuccess)
        return e;
    }
    if ((e = launch_b_spmm_a(b, st_)) != hipSuccess) return e;
    if ((e = launch_b_spmm_at(b, st_)) != hipSuccess) return e;
    if ((e = launch_b_rowmm(b, BQ_PREV, BW, BW, BM_BK_T, st_)) != hipSuccess) return e;
    if ((e = launch_b_rowmm(b, BQ_CUR, BW, BW2, BM_AK_CK, st_)) != hipSuccess) return e;
    if ((e = launch_b_rowmm(b, BW2, BNONE, BQ_NEXT, BM_MK, st_)) != hipSuccess) return e;
  }
  if (p1_.empty() && p2_.empty()) return hipSuccess;
  if ((e = launch_b_tick(d_clock_.as<int64_t>(), st_)) != hipSuccess) return e;
  ++clock_;
  for (BlockJob *j : p1_) j->steps_total++;
  for (BlockJob *j : p2_) j->steps_total++;
  return hipSuccess;
}

hipError_t BEngine::poll(std::vector<BlockJob *> *finished) {
  hipError_t e;
  // pass-1 jobs: unconverged pairs after their last step
  const int n1 = (int)p1_.size();
  std::vector<int> act(n1, 1);
  for (int i = 0; i < n1; ++i) {
    const BJobDesc &J = p1_[i]->h;
    const int klast = (int)(clock_ - 1 - J.start_clock);
    if (klast < 0) continue;
    e = hipMemcpyAsync(&act[i], J.active + (klast & 1), sizeof(int), hipMemcpyDeviceToHost, st_);
    if (e != hipSuccess) return e;
  }
  if ((e = hipStreamSynchronize(st_)) != hipSuccess) return e;
  std::vector<BlockJob *> keep1;
  for (int i = 0; i < n1; ++i) {
    BlockJob *j = p1_[i];
    const int steps = (int)(clock_ - j->h.start_clock);
    if (steps > 0 && (act[i] == 0 || steps >= j->Kcap)) {
      j->K = std::min(steps, j->Kcap);
      j->steps_last = j->K;
      j->converged = (act[i] == 0);
      dirty1_ = true;
      if ((e = enter_pass2(j)) != hipSuccess) return e;
    } else {
      keep1.push_back(j);
    }
  }
  p1_.swap(keep1);
  std::vector<BlockJob *> keep2;
  for (BlockJob *j : p2_) {
    const int steps = (int)(clock_ - j->h.start_clock);
    if (steps >= j->K) {
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
  auto r = [&](std::vector<BlockJob *> &v, bool &dirty) {
    auto it = std::find(v.begin(), v.end(), j);
    if (it != v.end()) {
      v.erase(it);
      dirty = true;
    }
  };
  r(p1_, dirty1_);
  r(p2_, dirty2_);
}

}  // namespace csvd
