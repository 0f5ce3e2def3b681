// Batched Lanczos engine: allocation of job state, the job table and the
// per-window launch sequence shared by solo, batched and served solves.
#include "engine.h"

#include <algorithm>
#include <cstring>

namespace csvd {

static int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

size_t Job::bytes_needed(int64_t m, int64_t n, int64_t nnz, int Lp, int S, int W, bool mixed) {
  const int64_t npad = round_up(n, kRowPad);
  const int64_t nL = n * Lp;
  size_t b = 0;
  b += sizeof(double) * (size_t)(m * Lp);                       // u
  b += sizeof(double) * 3 * (size_t)nL;                         // ring
  b += (mixed ? sizeof(float) : sizeof(double)) * (size_t)W * Lp * npad;   // window
  b += (mixed ? sizeof(float2) : sizeof(double2)) * 2 * (size_t)S * Lp * npad;  // X, P
  b += sizeof(double) * (size_t)Lp * (tiling_for(m, nnz, Lp).tiles + tiling_for(n, nnz, Lp).tiles);  // partials
  b += sizeof(double) * 6 * Lp + sizeof(double) * 2 * kHist;
  b += (sizeof(double2) * 2 + sizeof(int) * 3 + sizeof(double)) * (size_t)S * Lp;
  b += sizeof(double2) * 2 * (size_t)W * S * Lp + sizeof(double) * W * Lp;
  b += sizeof(double2) * (2 + 2 * (size_t)W) * S * Lp + 2 * sizeof(int);
  b += 256 * 48;  // alignment slack of the sub-allocations
  return b;
}

hipError_t Job::create(const int *rp, const int *ci, const double *va, const int *rpT, const int *ciT,
                       const double *vaT, int64_t m, int64_t n, int64_t nnz, int L, int Lp, int S, int W, bool mixed,
                       double tol,
                       const std::vector<double> &sre, const std::vector<double> &sim, hipStream_t st) {
  const int64_t npad = round_up(n, kRowPad);
  const Tiling t1 = tiling_for(m, nnz, Lp), t2 = tiling_for(n, nnz, Lp);
  const int tiles1 = t1.tiles, tiles2 = t2.tiles;
  hipError_t e = mem.alloc(bytes_needed(m, n, nnz, Lp, S, W, mixed));
  if (e != hipSuccess) return e;
  char *base = mem.as<char>();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    char *p = base + off;
    off += bytes;
    return (void *)p;
  };
  JobDesc &J = h;
  std::memset(&J, 0, sizeof(J));
  J.rp = rp; J.ci = ci; J.va = va;
  J.rpT = rpT; J.ciT = ciT; J.vaT = vaT;
  J.m = (int)m; J.n = (int)n; J.Lp = Lp; J.lgLp = ilog2(Lp); J.L = L; J.S = S; J.W = W; J.npad = (int)npad;
  J.tiles1 = tiles1; J.tiles2 = tiles2;
  J.G1 = t1.G; J.lgG1 = t1.lgG; J.E1 = t1.E; J.rpt1 = t1.rpt;
  J.G2 = t2.G; J.lgG2 = t2.lgG; J.E2 = t2.E; J.rpt2 = t2.rpt;
  {
    const int rtiles = (int)((n + kThreads - 1) / kThreads);
    int nsg = (int)std::min<int64_t>(S, std::max<int64_t>(1, 4096 / std::max<int64_t>(1, (int64_t)L * rtiles)));
    J.Sg = (S + nsg - 1) / nsg;
    J.Sg = std::min(J.Sg, std::max(1, 1024 / W));  // LDS staging limit of the window kernel
    J.nsg = (S + J.Sg - 1) / J.Sg;
  }
  J.tol = tol;
  J.u = (double *)take(sizeof(double) * m * Lp);
  J.wring = (double *)take(sizeof(double) * 3 * n * Lp);
  if (mixed) {
    J.winf = (float *)take(sizeof(float) * (size_t)W * Lp * npad);
    J.Xf = (float2 *)take(sizeof(float2) * (size_t)S * Lp * npad);
    J.Pf = (float2 *)take(sizeof(float2) * (size_t)S * Lp * npad);
  } else {
    J.win = (double *)take(sizeof(double) * (size_t)W * Lp * npad);
    J.X = (double2 *)take(sizeof(double2) * (size_t)S * Lp * npad);
    J.P = (double2 *)take(sizeof(double2) * (size_t)S * Lp * npad);
  }
  J.part1 = (double *)take(sizeof(double) * (size_t)Lp * tiles1);
  J.part2 = (double *)take(sizeof(double) * (size_t)Lp * tiles2);
  J.beta0 = (double *)take(sizeof(double) * Lp);
  J.alpha = (double *)take(sizeof(double) * Lp);
  J.coup = (double *)take(sizeof(double) * Lp);
  J.inv_cur = (double *)take(sizeof(double) * Lp);
  J.inv_prev = (double *)take(sizeof(double) * Lp);
  J.nrm_hist = (double *)take(sizeof(double) * 2 * kHist);
  J.eta = (double2 *)take(sizeof(double2) * S * Lp);
  J.zeta = (double2 *)take(sizeof(double2) * S * Lp);
  J.done = (int *)take(sizeof(int) * S * Lp);
  J.conv_iter = (int *)take(sizeof(int) * S * Lp);
  J.res = (double *)take(sizeof(double) * S * Lp);
  J.w_eta = (double2 *)take(sizeof(double2) * (size_t)W * S * Lp);
  J.w_zeta = (double2 *)take(sizeof(double2) * (size_t)W * S * Lp);
  J.w_e = (double *)take(sizeof(double) * (size_t)W * Lp);
  J.skip_pair = (int *)take(sizeof(int) * S * Lp);
  J.cA = (double2 *)take(sizeof(double2) * S * Lp);
  J.cC = (double2 *)take(sizeof(double2) * S * Lp);
  J.cE = (double2 *)take(sizeof(double2) * (size_t)W * S * Lp);
  J.cD = (double2 *)take(sizeof(double2) * (size_t)W * S * Lp);
  J.active = (int *)take(sizeof(int) * 2);
  if (off > mem.bytes) return hipErrorOutOfMemory;
  e = d_shift.alloc(sizeof(double2) * S);
  if (e != hipSuccess) return e;
  std::vector<double> sh(2 * S);
  for (int s = 0; s < S; ++s) {
    sh[2 * s] = sre[s];
    sh[2 * s + 1] = sim[s];
  }
  e = hipMemcpyAsync(d_shift.p, sh.data(), sizeof(double2) * S, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  J.shift = d_shift.as<double2>();
  e = hipMemsetAsync(J.active, 0, 2 * sizeof(int), st);
  if (e != hipSuccess) return e;
  // synchronous: the host vector `sh` goes out of scope
  return hipStreamSynchronize(st);
}

// ------------------------------------------------------------- KernelTimer
KernelTimer::~KernelTimer() {
  for (auto &e : ev) (void)hipEventDestroy(e);
}

hipError_t KernelTimer::begin(int k, hipStream_t st) {
  if (used + 2 > ev.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
  }
  kind.push_back(k);
  return hipEventRecord(ev[used++], st);
}

hipError_t KernelTimer::end(hipStream_t st) { return hipEventRecord(ev[used++], st); }

void KernelTimer::summarize(double out[kKinds], int64_t cnt[kKinds]) {
  for (int i = 0; i < kKinds; ++i) {
    out[i] = 0;
    cnt[i] = 0;
  }
  for (size_t i = 0; i + 1 < used && i / 2 < kind.size(); i += 2) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) {
      out[kind[i / 2]] += ms;
      cnt[kind[i / 2]] += 1;
    }
  }
  for (int i = 0; i < kKinds; ++i)
    if (cnt[i]) out[i] /= (double)cnt[i];
}

// ------------------------------------------------------------------ Engine
Engine::~Engine() {}

hipError_t Engine::init() {
  hipError_t e = d_clock_.alloc(sizeof(int64_t));
  if (e != hipSuccess) return e;
  e = d_ticket_.alloc(sizeof(int));
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(d_clock_.p, 0, sizeof(int64_t), st_);
  if (e != hipSuccess) return e;
  return hipMemsetAsync(d_ticket_.p, 0, sizeof(int), st_);
}

hipError_t Engine::add(Job *j) {
  j->h.start_clock = (int)clock_;
  jobs_.push_back(j);
  dirty_ = true;
  return hipSuccess;
}

void Engine::remove(Job *j) {
  auto it = std::find(jobs_.begin(), jobs_.end(), j);
  if (it != jobs_.end()) {
    jobs_.erase(it);
    dirty_ = true;
  }
}

hipError_t Engine::rebuild() {
  const int nj = (int)jobs_.size();
  std::vector<JobDesc> descs(nj);
  // 5 prefix tables of nj + 1 ints
  std::vector<int> toff(5 * (nj + 1), 0);
  int *t1 = &toff[0], *t2 = &toff[nj + 1], *tw = &toff[2 * (nj + 1)], *tc = &toff[3 * (nj + 1)],
      *tp = &toff[4 * (nj + 1)];
  for (int i = 0; i < nj; ++i) {
    descs[i] = jobs_[i]->h;
    const JobDesc &J = descs[i];
    t1[i + 1] = t1[i] + J.tiles1;
    t2[i + 1] = t2[i] + J.tiles2;
    tw[i + 1] = tw[i] + J.L * ((J.n + kThreads - 1) / kThreads) * J.nsg;
    tc[i + 1] = tc[i] + J.Lp;
    tp[i + 1] = tp[i] + J.S * J.L;
  }
  const size_t need = sizeof(JobDesc) * std::max(nj, 1);
  if (d_jobs_.bytes < need) {
    hipError_t e = d_jobs_.alloc(need * 2);
    if (e != hipSuccess) return e;
  }
  if (d_toff_.bytes < sizeof(int) * toff.size()) {
    hipError_t e = d_toff_.alloc(sizeof(int) * toff.size() * 2);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipMemcpyAsync(d_jobs_.p, descs.data(), sizeof(JobDesc) * nj, hipMemcpyHostToDevice, st_);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(d_toff_.p, toff.data(), sizeof(int) * toff.size(), hipMemcpyHostToDevice, st_);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st_);  // host vectors are temporaries
  if (e != hipSuccess) return e;
  int *dt = d_toff_.as<int>();
  bl_.jobs = d_jobs_.as<JobDesc>();
  bl_.njob = nj;
  bl_.toff1 = dt;
  bl_.toff2 = dt + (nj + 1);
  bl_.toffw = dt + 2 * (nj + 1);
  bl_.toffc = dt + 3 * (nj + 1);
  bl_.toffp = dt + 4 * (nj + 1);
  bl_.total1 = t1[nj];
  bl_.total2 = t2[nj];
  bl_.totalw = tw[nj];
  bl_.totalc = tc[nj];
  bl_.totalp = tp[nj];
  bl_.clock = d_clock_.as<int64_t>();
  bl_.clock_mut = d_clock_.as<int64_t>();
  bl_.ticket = d_ticket_.as<int>();
  bl_.Wmax = W_;
  bl_.mixed = mixed_ ? 1 : 0;
  dirty_ = false;
  return hipSuccess;
}

hipError_t Engine::run_window(KernelTimer *timer, int sample_every) {
  if (jobs_.empty()) return hipSuccess;
  hipError_t e;
  if (dirty_) {
    e = rebuild();
    if (e != hipSuccess) return e;
  }
  for (int q = 0; q < W_; ++q) {
    const bool sample = timer && sample_every > 0 && (step_count_ % sample_every) == 0;
    if (sample) timer->begin(0, st_);
    e = launch_k1_spmm_alpha(bl_, st_);
    if (e != hipSuccess) return e;
    if (sample) timer->end(st_);
    e = launch_r1_alpha(bl_, st_);
    if (e != hipSuccess) return e;
    if (sample) timer->begin(1, st_);
    e = launch_k2_spmm_lanczos(bl_, st_);
    if (e != hipSuccess) return e;
    if (sample) timer->end(st_);
    e = launch_s2_step(bl_, st_);
    if (e != hipSuccess) return e;
    ++clock_;
    ++step_count_;
  }
  for (Job *j : jobs_) j->iters += W_;
  parity_ ^= 1;
  for (Job *j : jobs_) {
    e = hipMemsetAsync(j->h.active + parity_, 0, sizeof(int), st_);
    if (e != hipSuccess) return e;
  }
  e = launch_window_coef(bl_, W_, parity_, st_);
  if (e != hipSuccess) return e;
  const bool samplew = timer && sample_every > 0 && ((step_count_ / W_) % 4) == 1;
  if (samplew) timer->begin(2, st_);
  e = launch_window_apply(bl_, W_, st_);
  if (e != hipSuccess) return e;
  if (samplew) timer->end(st_);
  return hipSuccess;
}

hipError_t Engine::collect(std::vector<Job *> *finished_jobs) {
  const int nj = (int)jobs_.size();
  std::vector<int> act(nj, 0);
  for (int i = 0; i < nj; ++i) {
    hipError_t e = hipMemcpyAsync(&act[i], jobs_[i]->h.active + parity_, sizeof(int), hipMemcpyDeviceToHost, st_);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return e;
  std::vector<Job *> keep;
  for (int i = 0; i < nj; ++i) {
    Job *j = jobs_[i];
    if (act[i] == 0 || j->iters >= j->max_iters) {
      j->finished = true;
      j->converged = (act[i] == 0);
      finished_jobs->push_back(j);
      dirty_ = true;
    } else {
      keep.push_back(j);
    }
  }
  jobs_.swap(keep);
  return hipSuccess;
}

}  // namespace csvd
