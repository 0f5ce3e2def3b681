// C ABI of the interior singular triplet solver: argument checking, the
// quadrature rule, the round structure of Algorithms 1/2 (eq. iter1/iter2)
// around the batched Lanczos engine, and the dense steps 3-5.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "block.h"
#include "engine.h"

using namespace csvd;

namespace {

// ------------------------------------------------------------------ errors
int set_err(csvd_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_code(hipError_t e) { return e == hipErrorOutOfMemory ? CSVD_ENOMEM : CSVD_EDEVICE; }

#define HIPCHK(ctx, expr)                                                                              \
  do {                                                                                                 \
    hipError_t _e = (expr);                                                                            \
    if (_e != hipSuccess)                                                                              \
      return set_err((ctx), hip_code(_e), std::string("HIP error '") + hipGetErrorString(_e) + "' in " \
                                              + #expr);                                                \
  } while (0)

// Column blocks between a device array with leading dimension ld and a
// contiguous host array (rows x cols, column-major).  Strided transfers go
// through a packed device copy and a plain 1-D transfer.
// Host transfers of column blocks with a leading dimension go through a
// staging buffer kept in the context (a fresh buffer per call would free
// device memory, and hipFree waits for the whole device, in the middle of
// other contexts' work on a batch).
constexpr int kStagingSlot = 31;

static int d2h_cols(csvd_ctx *ctx, double *host, const double *dev, int64_t ld, int64_t rows, int cols,
                    hipStream_t st) {
  if (rows <= 0 || cols <= 0) return CSVD_OK;
  const size_t bytes = sizeof(double) * (size_t)rows * cols;
  if (ld == rows) {
    HIPCHK(ctx, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    return CSVD_OK;
  }
  DevBuf &tmp = ctx->ws[kStagingSlot];
  if (!tmp.p || tmp.bytes < bytes) HIPCHK(ctx, tmp.alloc(bytes));
  HIPCHK(ctx, launch_copy_block(dev, ld, tmp.as<double>(), rows, rows, cols, st));
  HIPCHK(ctx, hipMemcpyAsync(host, tmp.p, bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return CSVD_OK;
}

static int h2d_cols(csvd_ctx *ctx, double *dev, int64_t ld, const double *host, int64_t rows, int cols,
                    hipStream_t st) {
  if (rows <= 0 || cols <= 0) return CSVD_OK;
  const size_t bytes = sizeof(double) * (size_t)rows * cols;
  DevBuf &tmp = ctx->ws[kStagingSlot];
  if (!tmp.p || tmp.bytes < bytes) HIPCHK(ctx, tmp.alloc(bytes));
  HIPCHK(ctx, hipMemcpyAsync(tmp.p, host, bytes, hipMemcpyHostToDevice, st));
  HIPCHK(ctx, launch_copy_block(tmp.as<double>(), rows, dev, ld, rows, cols, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  return CSVD_OK;
}

#define XFER(expr)           \
  do {                       \
    const int _rc = (expr);  \
    if (_rc) return _rc;     \
  } while (0)

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// --------------------------------------------------------------- quadrature
// Sec. 4: theta_j = 2 pi (j - 1/2) / N; point t_j = gamma + rho (cos + i alpha sin);
// plain: shift z_j = t_j, weight omega_j = rho/N (alpha cos + i sin);
// exp:   shift exp(t_j), weight psi_j = rho/N exp(t_j) (alpha cos + i sin).
// Only j = 1..N/2 are kept (the other half are conjugates, Sec. 3.1).
void quadrature(double a, double b, int N, int M, double alpha, int transform, SolveSpec *out) {
  const int S = N / 2;
  double gamma, rho;
  if (transform == CSVD_PLAIN) {
    gamma = 0.5 * (a * a + b * b);
    rho = 0.5 * (b * b - a * a);
  } else {
    gamma = std::log(a) + std::log(b);
    rho = std::log(b) - std::log(a);
  }
  out->S = S;
  out->shift_re.assign(S, 0.0);
  out->shift_im.assign(S, 0.0);
  out->c_re.assign((size_t)S * (M + 1), 0.0);
  out->c_im.assign((size_t)S * (M + 1), 0.0);
  for (int j = 0; j < S; ++j) {
    const double th = 2.0 * M_PI / N * (j + 0.5);
    const double ct = std::cos(th), st = std::sin(th);
    const double tr = gamma + rho * ct, ti = rho * alpha * st;  // point t_j
    double dr = rho / N * alpha * ct, di = rho / N * st;        // rho/N (alpha cos + i sin)
    double sr = tr, si = ti;
    if (transform == CSVD_EXP) {
      const double ex = std::exp(tr);
      sr = ex * std::cos(ti);
      si = ex * std::sin(ti);
      const double wr = dr * sr - di * si, wi = dr * si + di * sr;  // times exp(t_j)
      dr = wr;
      di = wi;
    }
    out->shift_re[j] = sr;
    out->shift_im[j] = si;
    double pr = 1.0, pi = 0.0;  // t_j^k
    for (int k = 0; k <= M; ++k) {
      out->c_re[(size_t)j * (M + 1) + k] = dr * pr - di * pi;
      out->c_im[(size_t)j * (M + 1) + k] = dr * pi + di * pr;
      const double nr = pr * tr - pi * ti, ni = pr * ti + pi * tr;
      pr = nr;
      pi = ni;
    }
  }
}

// ---------------------------------------------------------------- V_in RNG
// Counter-based N(0,1): SplitMix64 (Steele, Lea, Flood 2014) output k of the
// stream seeded with s is mix(s + (k+1) * 0x9E3779B97F4A7C15); entry e of
// the column-major n x L block uses outputs 2e and 2e+1 as u1, u2 (top 53
// bits / 2^53) and the Box-Muller value sqrt(-2 ln(1-u1)) cos(2 pi u2).
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void gaussian_block(uint64_t seed, int64_t count, double *out) {
  const uint64_t g = 0x9E3779B97F4A7C15ULL;
  for (int64_t e = 0; e < count; ++e) {
    const uint64_t k1 = 2 * (uint64_t)e, k2 = k1 + 1;
    const double u1 = (double)(mix64(seed + (k1 + 1) * g) >> 11) * 0x1.0p-53;
    const double u2 = (double)(mix64(seed + (k2 + 1) * g) >> 11) * 0x1.0p-53;
    out[e] = std::sqrt(-2.0 * std::log1p(-u1)) * std::cos(2.0 * M_PI * u2);
  }
}

// --------------------------------------------------------- small host math
// largest eigenvalue of a symmetric tridiagonal (diag d, off e) by bisection
double tridiag_max_eig(const std::vector<double> &d, const std::vector<double> &e) {
  const int k = (int)d.size();
  if (k == 0) return 0.0;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {  // Sturm count of eigenvalues < x
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < k; ++i) {
      if (q == 0.0) q = 1e-300;
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= k) hi = mid; else lo = mid;
  }
  return hi;
}

int pad_L(int L);

int check_params(csvd_ctx *ctx, double a, double b, const csvd_params *p) {
  if (!p) return set_err(ctx, CSVD_EINVAL, "params is NULL");
  if (!(std::isfinite(a) && std::isfinite(b)) || !(0.0 <= a && a < b))
    return set_err(ctx, CSVD_EINVAL, "need 0 <= a < b (finite)");
  if (p->N < 2 || p->N % 2 || p->N / 2 > kMaxShifts)
    return set_err(ctx, CSVD_EINVAL, "N must be even, 2 <= N <= 128");
  if (p->L < 1 || p->L > kMaxLp) return set_err(ctx, CSVD_EINVAL, "L must be in 1..256");
  if (p->M < 1) return set_err(ctx, CSVD_EINVAL, "M must be >= 1");
  if ((int64_t)p->L * p->M > ctx->n) return set_err(ctx, CSVD_EINVAL, "L*M must not exceed n");
  if (p->ell < 1) return set_err(ctx, CSVD_EINVAL, "ell must be >= 1");
  if (p->transform != CSVD_PLAIN && p->transform != CSVD_EXP)
    return set_err(ctx, CSVD_EINVAL, "transform must be CSVD_PLAIN or CSVD_EXP");
  if (p->transform == CSVD_EXP && !(a > 0.0))
    return set_err(ctx, CSVD_EINVAL, "the exp transform needs a > 0");
  if (p->precision != CSVD_FP64 && p->precision != CSVD_MIXED)
    return set_err(ctx, CSVD_EINVAL, "precision must be CSVD_FP64 or CSVD_MIXED");
  if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return set_err(ctx, CSVD_EINVAL, "alpha must be > 0");
  if (!(p->delta >= 0.0) || !(p->solve_rtol > 0.0) || !(p->spurious_eps >= 0.0))
    return set_err(ctx, CSVD_EINVAL, "delta, spurious_eps must be >= 0 and solve_rtol > 0");
  if (p->max_iters < 1) return set_err(ctx, CSVD_EINVAL, "max_iters must be >= 1");
  if (p->window < 0 || p->window > kMaxWindow) return set_err(ctx, CSVD_EINVAL, "window must be 0..64");
  if (!(p->norm_a >= 0.0)) return set_err(ctx, CSVD_EINVAL, "norm_a must be >= 0");
  if (p->solver != CSVD_SOLVER_AUTO && p->solver != CSVD_SOLVER_BLOCK && p->solver != CSVD_SOLVER_SINGLE)
    return set_err(ctx, CSVD_EINVAL, "solver must be CSVD_SOLVER_AUTO, CSVD_SOLVER_BLOCK or CSVD_SOLVER_SINGLE");
  if (p->keep_basis < 0) return set_err(ctx, CSVD_EINVAL, "keep_basis must be >= 0");
  if (p->cholqr_passes != 0 && p->cholqr_passes != 2)
    return set_err(ctx, CSVD_EINVAL, "cholqr_passes must be 0 or 2");
  if (!(p->resid_target >= 0.0)) return set_err(ctx, CSVD_EINVAL, "resid_target must be >= 0");
  if (p->ell_adaptive != 0 && p->ell_adaptive != 1) return set_err(ctx, CSVD_EINVAL, "ell_adaptive must be 0 or 1");
  if (p->ell_adaptive && !(p->resid_target > 0.0))
    return set_err(ctx, CSVD_EINVAL, "ell_adaptive needs resid_target > 0");
  return CSVD_OK;
}

int pick_window(const csvd_params *p) {
  int w = p->window > 0 ? p->window : 32;
  return w;
}

int pad_L(int L) {
  int lp = 1;
  while (lp < L) lp <<= 1;
  return lp;
}

// the block solver needs the padded width within its LDS-staged kernels
constexpr int kBlockPoll = kBlockPollSteps;

// Automatic choice: the block basis only when the matrix has at least
// kBlockMinRatio columns per basis column.  Below that a few block steps
// exhaust the whole space, the new blocks are rounding noise that local
// orthogonalization cannot separate from the old ones, and no deflation
// threshold suits both well and badly conditioned spectra; the per-column
// bases degrade gracefully there instead.
constexpr int kBlockMinRatio = 64;

// residual target of CSVD_MIXED (relative triplet residual)
constexpr double kMixedResidTarget = 1e-6;

// the block basis is at least one MFMA tile wide
int block_Lp(int L) { return std::max(kBlockMinLp, pad_L(L)); }

// groups_ok: L > kBlockMaxLp may run as column groups (solo solves only)
bool use_block(const csvd_params *p, int64_t n, bool groups_ok = false) {
  if (p->solver == CSVD_SOLVER_SINGLE) return false;
  const bool fits = pad_L(p->L) <= kBlockMaxLp || groups_ok;
  if (p->solver == CSVD_SOLVER_BLOCK) return fits;
  return fits && n >= (int64_t)kBlockMinRatio * block_Lp(std::min(p->L, kBlockMaxLp));
}

}  // namespace

// ============================================================================
// Solve state machine shared by the solo, batched and served paths.
namespace csvd {

struct SolveRun {
  csvd_ctx *ctx = nullptr;
  SolveSpec spec;
  int round = 0;
  DevBuf d_rhs;           // current right-hand side block, column-major
  int64_t rhs_ld = 0;
  DevBuf d_coef;          // S x (M+1) moment coefficients (double2)
  std::unique_ptr<Job> job;        // single-vector solver
  bool block = false;
  std::unique_ptr<BlockJob> bjob;  // block solver (first column group)
  // further column groups of the block solver: L > kBlockMaxLp columns run as
  // independent block jobs of at most kBlockMaxLp columns each, in one engine
  std::vector<std::unique_ptr<BlockJob>> bextra;
  std::vector<std::vector<double>> pad_cols;  // per group: seeded padding columns (n x (Lp - Lg), column-major)
  int gdone = 0;                   // groups whose current round has finished
  DevBuf d_Stmp;                   // S_0 of the intermediate rounds (block solver)
  int64_t iters_total = 0;
  int64_t iters_last = 0;
  bool all_converged = true;
  double max_res_est = 0.0;
  int status = CSVD_OK;
  double t_start = 0, t_solve_end = 0;
  std::vector<double> hist;  // column-0 Lanczos scalars of the first round
  std::vector<BlockJob *> groups() const {
    std::vector<BlockJob *> g;
    if (bjob) g.push_back(bjob.get());
    for (auto &x : bextra) g.push_back(x.get());
    return g;
  }
};

// ||A||_2 by power iteration on A^T A (60 products with one column); used to
// make residuals relative when the caller gives no norm.  Cached per matrix.
static int estimate_norm(csvd_ctx *ctx, double *out) {
  if (ctx->norm_est > 0) {
    *out = ctx->norm_est;
    return CSVD_OK;
  }
  const int64_t n = ctx->n, m = ctx->m;
  std::vector<double> x(n), y(n);
  gaussian_block(0x6e6f726dULL, n, x.data());
  DevBuf dx, du, dy;
  HIPCHK(ctx, dx.alloc(8 * n));
  HIPCHK(ctx, du.alloc(8 * m));
  HIPCHK(ctx, dy.alloc(8 * n));
  double lam = 0.0;
  for (int it = 0; it < 60; ++it) {
    double nx = 0;
    for (double v : x) nx += v * v;
    nx = std::sqrt(nx);
    if (!(nx > 0)) break;
    for (double &v : x) v /= nx;
    HIPCHK(ctx, hipMemcpyAsync(dx.p, x.data(), 8 * n, hipMemcpyHostToDevice, ctx->st));
    HIPCHK(ctx, launch_spmm_rowmajor((int)m, 1, ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(),
                                     dx.as<double>(), du.as<double>(), ctx->st));
    HIPCHK(ctx, launch_spmm_rowmajor((int)n, 1, ctx->rpT.as<int>(), ctx->ciT.as<int>(), ctx->vaT.as<double>(),
                                     du.as<double>(), dy.as<double>(), ctx->st));
    HIPCHK(ctx, hipMemcpyAsync(y.data(), dy.p, 8 * n, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(ctx, hipStreamSynchronize(ctx->st));
    double r = 0;
    for (int64_t i = 0; i < n; ++i) r += x[i] * y[i];
    lam = std::max(lam, r);
    x.swap(y);
  }
  ctx->norm_est = std::sqrt(std::max(lam, 0.0));
  *out = ctx->norm_est;
  return CSVD_OK;
}

// Uploads the padded starting block of every column group: its columns
// soff .. soff + Lg - 1 of V (column-major, leading dimension ldv, host),
// padding columns from pad_cols.
static int upload_vpad(SolveRun &R, const double *V, int64_t ldv, hipStream_t st = nullptr) {
  csvd_ctx *ctx = R.ctx;
  if (!st) st = ctx->st;
  const int64_t n = ctx->n;
  const std::vector<BlockJob *> gs = R.groups();
  for (size_t g = 0; g < gs.size(); ++g) {
    BlockJob &B = *gs[g];
    const int L = B.h.L, Lp = B.h.Lp, l0 = B.h.soff;
    std::vector<double> Vp((size_t)n * Lp);
    for (int64_t i = 0; i < n; ++i) {
      for (int l = 0; l < L; ++l) Vp[(size_t)i * Lp + l] = V[(size_t)(l0 + l) * ldv + i];
      for (int l = L; l < Lp; ++l) Vp[(size_t)i * Lp + l] = R.pad_cols[g][(size_t)(l - L) * n + i];
    }
    HIPCHK(ctx, hipMemcpyAsync(B.h.Vpad, Vp.data(), 8 * Vp.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
  }
  return CSVD_OK;
}

int run_begin(SolveRun &R, csvd_ctx *ctx, double a, double b, const csvd_params *p, const double *V_host,
              int W, bool mixed, bool groups_ok = false) {
  R.ctx = ctx;
  int rc = check_params(ctx, a, b, p);
  if (rc) return rc;
  R.t_start = now_ms();
  R.spec = SolveSpec();
  R.spec.a = a;
  R.spec.b = b;
  R.spec.p = *p;
  quadrature(a, b, p->N, p->M, p->alpha, p->transform, &R.spec);
  R.spec.Lp = use_block(p, ctx->n, groups_ok) ? block_Lp(std::min(p->L, kBlockMaxLp)) : pad_L(p->L);
  R.spec.W = W;
  const int S = R.spec.S, M = p->M, L = p->L;
  const int64_t n = ctx->n;
  // host V_in (column-major n x L)
  std::vector<double> V((size_t)n * L);
  if (V_host) {
    std::memcpy(V.data(), V_host, sizeof(double) * V.size());
    for (double x : V)
      if (!std::isfinite(x)) return set_err(ctx, CSVD_ENUMERIC, "V_in has a non-finite entry");
  } else {
    gaussian_block(p->seed, (int64_t)V.size(), V.data());
  }
  HIPCHK(ctx, R.d_rhs.alloc(sizeof(double) * V.size()));
  HIPCHK(ctx, hipMemcpyAsync(R.d_rhs.p, V.data(), sizeof(double) * V.size(), hipMemcpyHostToDevice, ctx->st));
  R.rhs_ld = n;
  std::vector<double> cc(2 * (size_t)S * (M + 1));
  for (size_t i = 0; i < (size_t)S * (M + 1); ++i) {
    cc[2 * i] = R.spec.c_re[i];
    cc[2 * i + 1] = R.spec.c_im[i];
  }
  HIPCHK(ctx, R.d_coef.alloc(sizeof(double) * cc.size()));
  HIPCHK(ctx, hipMemcpyAsync(R.d_coef.p, cc.data(), sizeof(double) * cc.size(), hipMemcpyHostToDevice, ctx->st));
  R.block = use_block(p, ctx->n, groups_ok);
  if (R.block) {
    // a round that may be the last accumulates every moment; the others only
    // S_0, the next round's right-hand side (eq. iter1)
    const bool all_moments = (p->ell == 1) || p->ell_adaptive;
    const int Kmom = all_moments ? M + 1 : 1;
    // the deflation test of the basis is relative to ||A^T A||
    double na = p->norm_a;
    if (!(na > 0)) {
      int rc1 = estimate_norm(ctx, &na);
      if (rc1) return rc1;
    }
    const int64_t npad = round_up(n, kRowPad);
    HIPCHK(ctx, ctx->d_S.alloc(sizeof(double) * npad * (size_t)(M + 1) * L));
    if (!all_moments) HIPCHK(ctx, R.d_Stmp.alloc(sizeof(double) * npad * (size_t)L));
    // column groups of at most kBlockMaxLp columns (one group when L fits)
    const int ng = (L + kBlockMaxLp - 1) / kBlockMaxLp;
    R.bextra.clear();
    R.pad_cols.assign(ng, std::vector<double>());
    for (int g = 0; g < ng; ++g) {
      const int l0 = g * kBlockMaxLp, Lg = std::min(kBlockMaxLp, L - l0), Lp = block_Lp(Lg);
      const int64_t kc = std::min<int64_t>(p->max_iters, (int64_t)std::ceil(3.5 * (double)n / Lp) + 32);
      std::unique_ptr<BlockJob> B(new BlockJob());
      HIPCHK(ctx, B->create(ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(), ctx->rpT.as<int>(),
                            ctx->ciT.as<int>(), ctx->vaT.as<double>(), ctx->m, n, ctx->nnz, Lg, Lp, S, (int)kc,
                            M + 1, p->solve_rtol, R.spec.shift_re, R.spec.shift_im, R.spec.c_re, R.spec.c_im,
                            M + 1, ctx->st, ctx->lr));
      B->h.Kmom = Kmom;
      B->want_store = (p->keep_basis != 0);
      B->mixed = (p->precision == CSVD_MIXED);
      B->store_cap = (p->keep_basis >= 2) ? p->keep_basis : 0;
      B->h.onepass_rho = (p->cholqr_passes == 2) ? 0.0 : kOnePassRho;
      B->h.dscale = na * na;
      B->h.sL = L;
      B->h.soff = l0;
      B->h.Sout = all_moments ? ctx->d_S.as<double>() : R.d_Stmp.as<double>();
      R.pad_cols[g].assign((size_t)n * (Lp - Lg), 0.0);
      if (Lp > Lg)
        gaussian_block(p->seed ^ (0xA5A5F00DCAFEULL + (uint64_t)g * 0x9E3779B97F4A7C15ULL),
                       (int64_t)R.pad_cols[g].size(), R.pad_cols[g].data());
      if (g == 0) R.bjob = std::move(B);
      else R.bextra.push_back(std::move(B));
    }
    R.gdone = 0;
    int rc2 = upload_vpad(R, V.data(), n);
    if (rc2) return rc2;
    R.round = 0;
    R.iters_total = 0;
    R.all_converged = true;
    R.max_res_est = 0;
    return CSVD_OK;
  }
  R.job.reset(new Job());
  HIPCHK(ctx, R.job->create(ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(), ctx->rpT.as<int>(),
                            ctx->ciT.as<int>(), ctx->vaT.as<double>(), ctx->m, n, ctx->nnz, L, R.spec.Lp, S, W, mixed,
                            p->solve_rtol, R.spec.shift_re, R.spec.shift_im, ctx->st));
  R.job->max_iters = p->max_iters;
  HIPCHK(ctx, launch_job_init(R.job->h, R.d_rhs.as<double>(), R.rhs_ld, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));  // host V goes out of scope
  R.round = 0;
  R.iters_total = 0;
  R.all_converged = true;
  R.max_res_est = 0;
  return CSVD_OK;
}

// Reads the exit state of the finished job (residual estimates, history).
static int harvest_job(SolveRun &R) {
  csvd_ctx *ctx = R.ctx;
  Job &J = *R.job;
  const int S = J.h.S, Lp = J.h.Lp, L = J.h.L;
  std::vector<double> res((size_t)S * Lp);
  HIPCHK(ctx, hipMemcpyAsync(res.data(), J.h.res, sizeof(double) * res.size(), hipMemcpyDeviceToHost, ctx->st));
  std::vector<double> hist(2 * kHist);
  HIPCHK(ctx, hipMemcpyAsync(hist.data(), J.h.nrm_hist, sizeof(double) * hist.size(), hipMemcpyDeviceToHost,
                             ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  double mx = 0;
  for (int s = 0; s < S; ++s)
    for (int l = 0; l < L; ++l) mx = std::max(mx, res[(size_t)s * Lp + l]);
  R.max_res_est = std::max(R.max_res_est, mx);
  R.iters_total += J.iters;
  if (!J.converged) R.all_converged = false;
  if (R.round == 0) {
    const int64_t k = std::min<int64_t>(J.iters, kHist);
    R.hist.assign(hist.begin(), hist.begin() + 2 * k);
  }
  return CSVD_OK;
}

// Called when the job of the current round has finished.  Returns 1 in *more
// when another round was started (the caller must re-add the job).
static int run_after_round_block(SolveRun &R, bool *more) {
  csvd_ctx *ctx = R.ctx;
  const std::vector<BlockJob *> gs = R.groups();
  int kmax = 0;
  for (BlockJob *Bp : gs) {
    BlockJob &B = *Bp;
    const int S = B.h.S, Lp = B.h.Lp, L = B.h.L;
    std::vector<double> res((size_t)S * Lp);
    HIPCHK(ctx, hipMemcpyAsync(res.data(), B.h.res, sizeof(double) * res.size(), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(ctx, hipStreamSynchronize(ctx->st));
    double mx = 0;
    for (int s = 0; s < S; ++s)
      for (int l = 0; l < L; ++l) mx = std::max(mx, res[(size_t)s * Lp + l]);
    R.max_res_est = std::max(R.max_res_est, mx);
    kmax = std::max(kmax, B.K);  // the groups step together: the round takes the longest
    if (!B.converged) R.all_converged = false;
  }
  R.iters_total += kmax;
  R.iters_last = kmax;
  R.gdone = 0;
  *more = false;
  const csvd_params &p = R.spec.p;
  if (R.round + 1 < p.ell && !p.ell_adaptive) {
    // eq. iter1: S_0^(nu) becomes the next right-hand side
    const int L = p.L;
    const int64_t n = ctx->n, npad = R.bjob->h.npad;
    std::vector<double> S0((size_t)npad * L);
    HIPCHK(ctx, hipMemcpyAsync(S0.data(), R.d_Stmp.p, sizeof(double) * S0.size(), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(ctx, hipStreamSynchronize(ctx->st));
    int rc = upload_vpad(R, S0.data(), npad);
    if (rc) return rc;
    // keep V for the solve check: the last round's right-hand side
    std::vector<double> Vc((size_t)n * L);
    for (int l = 0; l < L; ++l)
      for (int64_t i = 0; i < n; ++i) Vc[(size_t)l * n + i] = S0[(size_t)l * npad + i];
    HIPCHK(ctx, hipMemcpyAsync(R.d_rhs.p, Vc.data(), 8 * Vc.size(), hipMemcpyHostToDevice, ctx->st));
    HIPCHK(ctx, hipStreamSynchronize(ctx->st));
    R.round += 1;
    for (BlockJob *Bp : gs) {
      BlockJob &B = *Bp;
      B.robust_steps = kRobustSteps;  // the filtered block: first Krylov blocks by Householder QR
      if (R.round + 1 == p.ell) {
        B.h.Kmom = p.M + 1;
        B.h.Sout = ctx->d_S.as<double>();
      }
    }
    *more = true;
  }
  return CSVD_OK;
}

int run_after_round(SolveRun &R, bool *more) {
  if (R.block) return run_after_round_block(R, more);
  csvd_ctx *ctx = R.ctx;
  int rc = harvest_job(R);
  if (rc) return rc;
  *more = false;
  const csvd_params &p = R.spec.p;
  if (R.round + 1 < p.ell && !p.ell_adaptive) {
    // eq. iter1: S_0^(nu) = 2 sum_j Re(w_j Y_j) becomes the next right-hand side
    const int64_t npad = R.job->h.npad;
    DevBuf nr;
    HIPCHK(ctx, nr.alloc(sizeof(double) * npad * p.L));
    // the k = 0 coefficients are the first entries of each shift's row: gather
    std::vector<double> c0(2 * (size_t)R.spec.S);
    for (int s = 0; s < R.spec.S; ++s) {
      c0[2 * s] = R.spec.c_re[(size_t)s * (p.M + 1)];
      c0[2 * s + 1] = R.spec.c_im[(size_t)s * (p.M + 1)];
    }
    DevBuf dc0;
    HIPCHK(ctx, dc0.alloc(sizeof(double) * c0.size()));
    HIPCHK(ctx, hipMemcpyAsync(dc0.p, c0.data(), sizeof(double) * c0.size(), hipMemcpyHostToDevice, ctx->st));
    HIPCHK(ctx, launch_moments(R.job->h, dc0.as<double2>(), 1, nr.as<double>(), ctx->st));
    HIPCHK(ctx, hipStreamSynchronize(ctx->st));
    std::swap(R.d_rhs.p, nr.p);
    std::swap(R.d_rhs.bytes, nr.bytes);
    R.rhs_ld = npad;
    R.round += 1;
    R.job->iters = 0;
    R.job->finished = false;
    R.job->converged = false;
    HIPCHK(ctx, launch_job_init(R.job->h, R.d_rhs.as<double>(), R.rhs_ld, ctx->st));
    *more = true;
  }
  return CSVD_OK;
}

// ell_adaptive: called after steps 3-5 of a round.  When a triplet missed
// resid_target (largest residual before drops) and rounds remain, the next
// round of eq. iter1 starts from this round's S_0 (the first L columns of
// the moments) and *more is set; the caller restarts the round's jobs.
// Host copies go through `stream` (default: the context's stream).
static int run_next_round(SolveRun &R, bool *more, hipStream_t stream = nullptr) {
  csvd_ctx *ctx = R.ctx;
  hipStream_t st = stream ? stream : ctx->st;
  const csvd_params &p = R.spec.p;
  *more = false;
  if (!p.ell_adaptive || R.round + 1 >= p.ell || !(ctx->resid_all_max > p.resid_target)) return CSVD_OK;
  const int L = p.L;
  const int64_t n = ctx->n, npad = round_up(n, kRowPad);
  if (R.block) {
    std::vector<double> S0((size_t)npad * L);
    HIPCHK(ctx, hipMemcpyAsync(S0.data(), ctx->d_S.p, sizeof(double) * S0.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    int rc = upload_vpad(R, S0.data(), npad, st);
    if (rc) return rc;
    for (BlockJob *B : R.groups()) B->robust_steps = kRobustSteps;  // see run_after_round_block
  } else {
    DevBuf nr;
    HIPCHK(ctx, nr.alloc(sizeof(double) * npad * L));
    HIPCHK(ctx, hipMemcpyAsync(nr.p, ctx->d_S.p, sizeof(double) * npad * L, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    std::swap(R.d_rhs.p, nr.p);
    std::swap(R.d_rhs.bytes, nr.bytes);
    R.rhs_ld = npad;
    R.job->iters = 0;
    R.job->finished = false;
    R.job->converged = false;
    HIPCHK(ctx, launch_job_init(R.job->h, R.d_rhs.as<double>(), R.rhs_ld, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
  }
  R.round += 1;
  *more = true;
  return CSVD_OK;
}

// Epilogue buffers live in the context's workspace slots and are only
// reallocated when a solve needs more room than the last one (hipFree would
// wait for the device; csvd_trim and csvd_destroy free them).
static hipError_t ws_grow(DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.p && b.bytes >= bytes) return hipSuccess;
  return b.alloc(bytes);
}

// Steps 1-2 (moments) and 3-5 (dense) after the last round, on `stream`
// (default: the context's stream).
int run_finalize(SolveRun &R, hipStream_t stream = nullptr) {
  csvd_ctx *ctx = R.ctx;
  hipStream_t st = stream ? stream : ctx->st;
  const csvd_params &p = R.spec.p;
  const int L = p.L, M = p.M, S = R.spec.S;
  const int64_t m = ctx->m, n = ctx->n;
  const int64_t npad = round_up(n, kRowPad), mpad = round_up(m, kRowPad);
  ctx->L = L;
  ctx->M = M;
  ctx->N = p.N;
  ctx->S = S;
  ctx->npad = npad;
  ctx->mpad = mpad;
  csvd_info &info = ctx->info;
  std::memset(&info, 0, sizeof(info));
  // ---- moments S_k, k = 0..M (step 2 and the extra moment of Sec. 3.4.1);
  // the block solver's second pass has already accumulated them
  if (!R.block) {
    HIPCHK(ctx, ctx->d_S.alloc(sizeof(double) * npad * (size_t)(M + 1) * L));
    HIPCHK(ctx, hipMemsetAsync(ctx->d_S.p, 0, ctx->d_S.bytes, st));
    HIPCHK(ctx, launch_moments(R.job->h, R.d_coef.as<double2>(), M + 1, ctx->d_S.as<double>(), st));
  }
  HIPCHK(ctx, hipStreamSynchronize(st));
  R.t_solve_end = now_ms();
  double t0 = R.t_solve_end;
  const int LM = L * M;
  // ---- step 3: QR of S-hat (Householder), SVD of R by one-sided Jacobi on R^T
  DevBuf &Xq = ctx->ws[0]; DevBuf &tau1 = ctx->ws[1];
  HIPCHK(ctx, ws_grow(Xq, sizeof(double) * npad * LM));
  HIPCHK(ctx, ws_grow(tau1, sizeof(double) * LM));
  HIPCHK(ctx, hipMemcpyAsync(Xq.p, ctx->d_S.p, sizeof(double) * npad * LM, hipMemcpyDeviceToDevice, st));
  DevBuf &ws1 = ctx->ws[2];
  HIPCHK(ctx, ws_grow(ws1, sizeof(double) * hh_blocked_ws_doubles(LM)));
  HIPCHK(ctx, hh_qr_blocked(Xq.as<double>(), npad, (int)n, LM, tau1.as<double>(), ws1.as<double>(), st));
  // R (LM x LM upper) to the host, R^T back as a column-major LMe x LMe block
  const int LMe = jacobi_padded_cols(LM);  // zero columns to a whole number of Jacobi block pairs
  std::vector<double> Rh((size_t)LM * LM);
  XFER(d2h_cols(ctx, Rh.data(), Xq.as<double>(), npad, LM, LM, st));
  std::vector<double> Rt((size_t)LMe * LMe, 0.0), Jm((size_t)LMe * LMe, 0.0);
  for (int c = 0; c < LM; ++c)
    for (int r = 0; r <= c; ++r) Rt[(size_t)r * LMe + c] = Rh[(size_t)c * LM + r];  // Rt[c, r] = R[r, c]
  for (int i = 0; i < LMe; ++i) Jm[(size_t)i * LMe + i] = 1.0;
  DevBuf &dRt = ctx->ws[3]; DevBuf &dJ = ctx->ws[4]; DevBuf &dcnt = ctx->ws[5]; DevBuf &dnorm = ctx->ws[6];
  HIPCHK(ctx, ws_grow(dRt, sizeof(double) * Rt.size()));
  HIPCHK(ctx, ws_grow(dJ, sizeof(double) * Jm.size()));
  HIPCHK(ctx, ws_grow(dcnt, sizeof(int)));
  HIPCHK(ctx, ws_grow(dnorm, sizeof(double) * (LMe + 1)));
  HIPCHK(ctx, hipMemcpyAsync(dRt.p, Rt.data(), sizeof(double) * Rt.size(), hipMemcpyHostToDevice, st));
  HIPCHK(ctx, hipMemcpyAsync(dJ.p, Jm.data(), sizeof(double) * Jm.size(), hipMemcpyHostToDevice, st));
  // one-sided Jacobi; a pair is rotated while |a_p^T a_q| > sqrt(rows) eps
  // ||a_p|| ||a_q|| (the rounding level of the dot product itself, as in
  // LAPACK's one-sided Jacobi): below it a rotation only moves noise.  Columns
  // with ||a_p|| <= eps^2 ||A||_F (fro2 = ||A||_F^2, from the host copy) are
  // not rotated: they lie far under the rank cut delta s_1 of every useful
  // delta and can only lose norm, while a rank-deficient S-hat leaves columns
  // whose squared norms are denormal, on which rotations need not converge.
  // Square A and V of jacobi_padded_cols columns: pairs of column blocks in
  // LDS where the size allows, else one launch per column pairing.
  bool sweeps_exhausted = false;
  auto jacobi = [&](double *A, int rows, int ncol_even, double *V, int vrows, double fro2) -> int {
    constexpr double eps = 2.220446049250313e-16;
    const double tol = std::sqrt((double)rows) * eps;
    const double floor2 = eps * eps * eps * eps * fro2;
    const int w = jacobi_block_width(ncol_even);
    const int nsteps = w ? ncol_even / w - 1 : ncol_even - 1;
    for (int sweep = 0; sweep < 60; ++sweep) {
      HIPCHK(ctx, hipMemsetAsync(dcnt.p, 0, sizeof(int), st));
      for (int s2 = 0; s2 < nsteps; ++s2) {
        if (w)
          HIPCHK(ctx, launch_jacobi_blk(A, ncol_even, rows, ncol_even, V, ncol_even, vrows, s2, tol, floor2,
                                        dcnt.as<int>(), st));
        else
          HIPCHK(ctx, launch_jacobi_step(A, ncol_even, rows, ncol_even, V, ncol_even, vrows, s2, tol, floor2,
                                         dcnt.as<int>(), st));
      }
      int cnt = 0;
      HIPCHK(ctx, hipMemcpyAsync(&cnt, dcnt.p, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
      if (cnt == 0) return CSVD_OK;
    }
    sweeps_exhausted = true;  // reported in csvd_info and by the solve's status
    return CSVD_OK;
  };
  double fro2R = 0.0;
  for (double x : Rt) fro2R += x * x;
  int rc = jacobi(dRt.as<double>(), LMe, LMe, dJ.as<double>(), LMe, fro2R);
  if (rc) return rc;
  std::vector<double> sS(LMe);
  HIPCHK(ctx, launch_col_norms(dRt.as<double>(), LMe, LMe, LMe, dnorm.as<double>(), st));
  HIPCHK(ctx, hipMemcpyAsync(sS.data(), dnorm.p, sizeof(double) * LMe, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipMemcpyAsync(Jm.data(), dJ.p, sizeof(double) * Jm.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  std::vector<int> perm(LMe);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return sS[x] > sS[y]; });
  const double s1 = sS[perm[0]];
  int r = 0;
  if (s1 > 0)
    for (int i = 0; i < LM; ++i)
      if (sS[perm[i]] > p.delta * s1) ++r;
  info.sigma_s1 = s1;
  info.rank = r;
  // V~ = Q [U_R(:, perm[0:r]); 0]
  DevBuf &Vt = ctx->ws[7];
  HIPCHK(ctx, ws_grow(Vt, sizeof(double) * npad * std::max(r, 1)));
  HIPCHK(ctx, hipMemsetAsync(Vt.p, 0, sizeof(double) * npad * std::max(r, 1), st));
  if (r > 0) {
    std::vector<double> Z((size_t)LM * r);
    for (int c = 0; c < r; ++c)
      for (int i = 0; i < LM; ++i) Z[(size_t)c * LM + i] = Jm[(size_t)perm[c] * LMe + i];
    XFER(h2d_cols(ctx, Vt.as<double>(), npad, Z.data(), LM, r, st));
    DevBuf &wsr = ctx->ws[8];
    HIPCHK(ctx, ws_grow(wsr, sizeof(double) * hh_blocked_ws_doubles(r)));
    HIPCHK(ctx, hh_apply_blocked(Xq.as<double>(), npad, (int)n, LM, ws1.as<double>(), Vt.as<double>(), npad, r,
                                 wsr.as<double>(), st));
    HIPCHK(ctx, hipStreamSynchronize(st));
  }
  double t1 = now_ms();
  // ---- step 4: X = A V~, [U~, B] = qr(X)
  const int re = jacobi_padded_cols(r);
  DevBuf &Vrow = ctx->ws[9]; DevBuf &Xrow = ctx->ws[10]; DevBuf &Xa = ctx->ws[11]; DevBuf &tau2 = ctx->ws[12]; DevBuf &ws2 = ctx->ws[13];
  std::vector<double> Bh;
  if (r > 0) {
    HIPCHK(ctx, ws_grow(Vrow, sizeof(double) * n * r));
    HIPCHK(ctx, ws_grow(Xrow, sizeof(double) * m * r));
    HIPCHK(ctx, ws_grow(Xa, sizeof(double) * mpad * r));
    HIPCHK(ctx, ws_grow(tau2, sizeof(double) * r));
    HIPCHK(ctx, hipMemsetAsync(Xa.p, 0, sizeof(double) * mpad * r, st));
    HIPCHK(ctx, launch_col_to_row((int)n, r, Vt.as<double>(), npad, Vrow.as<double>(), r, st));
    HIPCHK(ctx, launch_spmm_rowmajor((int)m, r, ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(),
                                     Vrow.as<double>(), Xrow.as<double>(), st));
    HIPCHK(ctx, launch_row_to_col((int)m, r, Xrow.as<double>(), r, Xa.as<double>(), mpad, st));
    HIPCHK(ctx, ws_grow(ws2, sizeof(double) * hh_blocked_ws_doubles(r)));
    HIPCHK(ctx, hh_qr_blocked(Xa.as<double>(), mpad, (int)m, r, tau2.as<double>(), ws2.as<double>(), st));
    Bh.assign((size_t)r * r, 0.0);
    std::vector<double> Rb((size_t)r * r);
    XFER(d2h_cols(ctx, Rb.data(), Xa.as<double>(), mpad, r, r, st));
    for (int c = 0; c < r; ++c)
      for (int i = 0; i <= c; ++i) Bh[(size_t)c * r + i] = Rb[(size_t)c * r + i];
  }
  double t2 = now_ms();
  // ---- step 5: SVD of B = P Phi Q^T by one-sided Jacobi (B J = P Phi, Q = J)
  std::vector<int> sel;
  std::vector<double> phi, tauv;
  std::vector<double> Bj, Jb;
  if (r > 0) {
    std::vector<double> Be((size_t)re * re, 0.0), Ie((size_t)re * re, 0.0);
    for (int c = 0; c < r; ++c)
      for (int i = 0; i < r; ++i) Be[(size_t)c * re + i] = Bh[(size_t)c * r + i];
    for (int i = 0; i < re; ++i) Ie[(size_t)i * re + i] = 1.0;
    DevBuf &dB = ctx->ws[14]; DevBuf &dQ = ctx->ws[15];
    HIPCHK(ctx, ws_grow(dB, sizeof(double) * Be.size()));
    HIPCHK(ctx, ws_grow(dQ, sizeof(double) * Ie.size()));
    HIPCHK(ctx, hipMemcpyAsync(dB.p, Be.data(), sizeof(double) * Be.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(dQ.p, Ie.data(), sizeof(double) * Ie.size(), hipMemcpyHostToDevice, st));
    double fro2B = 0.0;
    for (double x : Be) fro2B += x * x;
    rc = jacobi(dB.as<double>(), re, re, dQ.as<double>(), re, fro2B);
    if (rc) return rc;
    phi.assign(re, 0.0);
    HIPCHK(ctx, launch_col_norms(dB.as<double>(), re, re, re, dnorm.as<double>(), st));
    HIPCHK(ctx, hipMemcpyAsync(phi.data(), dnorm.p, sizeof(double) * re, hipMemcpyDeviceToHost, st));
    Bj.assign((size_t)re * re, 0.0);
    Jb.assign((size_t)re * re, 0.0);
    HIPCHK(ctx, hipMemcpyAsync(Bj.data(), dB.p, sizeof(double) * Bj.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(Jb.data(), dQ.p, sizeof(double) * Jb.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    // spurious index tau_i = q^T q / q^T Sigma_S1^{-1} q  (Sec. 3.4.2), q = Q(:, i)
    tauv.assign(re, 0.0);
    for (int i = 0; i < re; ++i) {
      double num = 0, den = 0;
      for (int j = 0; j < r; ++j) {
        const double q = Jb[(size_t)i * re + j];
        num += q * q;
        den += q * q / sS[perm[j]];
      }
      tauv[i] = den > 0 ? num / den : 0.0;
    }
    for (int i = 0; i < re; ++i) {
      if (phi[i] >= R.spec.a && phi[i] <= R.spec.b && tauv[i] >= p.spurious_eps * s1 && phi[i] > 0.0) sel.push_back(i);
    }
    std::stable_sort(sel.begin(), sel.end(), [&](int x, int y) { return phi[x] < phi[y]; });
  }
  const int t = (int)sel.size();
  ctx->sigma.assign(t, 0.0);
  ctx->resid.assign(t, 0.0);
  ctx->resid_est.assign(t, 0.0);
  // triplet vectors (column stride mpad / npad); kept between solves
  HIPCHK(ctx, ws_grow(ctx->d_U, sizeof(double) * mpad * std::max(t, 1)));
  HIPCHK(ctx, ws_grow(ctx->d_V, sizeof(double) * npad * std::max(t, 1)));
  double normA = p.norm_a;
  if (!(normA > 0) && !R.block) {
    std::vector<double> d, e;
    for (size_t k = 0; k + 1 < R.hist.size(); k += 2) d.push_back(R.hist[k]);
    for (size_t k = 0; k + 1 < R.hist.size() && e.size() + 1 < d.size(); k += 2) e.push_back(R.hist[k + 1]);
    normA = std::sqrt(std::max(tridiag_max_eig(d, e), 0.0));
  }
  if (!(normA > 0)) {
    rc = estimate_norm(ctx, &normA);
    if (rc) return rc;
  }
  info.norm_a = normA;
  if (t > 0) {
    std::vector<double> Qs((size_t)r * t), Ps((size_t)r * t);
    for (int c = 0; c < t; ++c) {
      const int i = sel[c];
      ctx->sigma[c] = phi[i];
      for (int j = 0; j < r; ++j) {
        Qs[(size_t)c * r + j] = Jb[(size_t)i * re + j];
        Ps[(size_t)c * r + j] = Bj[(size_t)i * re + j] / phi[i];
      }
    }
    DevBuf &dQs = ctx->ws[16]; DevBuf &dPs = ctx->ws[17]; DevBuf &dsig = ctx->ws[18];
    HIPCHK(ctx, ws_grow(dQs, sizeof(double) * Qs.size()));
    HIPCHK(ctx, ws_grow(dsig, sizeof(double) * t));
    HIPCHK(ctx, hipMemcpyAsync(dQs.p, Qs.data(), sizeof(double) * Qs.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(dsig.p, ctx->sigma.data(), sizeof(double) * t, hipMemcpyHostToDevice, st));
    // V-hat = V~ Q_sel (MFMA GEMM);  U-hat = Q_X [P_sel; 0]
    HIPCHK(ctx, hipMemsetAsync(ctx->d_V.p, 0, ctx->d_V.bytes, st));
    HIPCHK(ctx, launch_gemm((int)npad, t, r, 1.0, Vt.as<double>(), npad, dQs.as<double>(), r, 0.0,
                            ctx->d_V.as<double>(), npad, st));
    HIPCHK(ctx, hipMemsetAsync(ctx->d_U.p, 0, ctx->d_U.bytes, st));
    XFER(h2d_cols(ctx, ctx->d_U.as<double>(), mpad, Ps.data(), r, t, st));
    DevBuf &wsu = ctx->ws[19];
    HIPCHK(ctx, ws_grow(wsu, sizeof(double) * hh_blocked_ws_doubles(t)));
    HIPCHK(ctx, hh_apply_blocked(Xa.as<double>(), mpad, (int)m, r, ws2.as<double>(), ctx->d_U.as<double>(), mpad, t,
                                 wsu.as<double>(), st));
    HIPCHK(ctx, launch_sign_fix(ctx->d_U.as<double>(), mpad, (int)m, ctx->d_V.as<double>(), npad, (int)n, t, st));
    // residuals: ||A v - s u|| and ||A^T u - s v||
    DevBuf &vr = ctx->ws[20]; DevBuf &ur = ctx->ws[21]; DevBuf &av = ctx->ws[22]; DevBuf &atu = ctx->ws[23]; DevBuf &o1 = ctx->ws[24]; DevBuf &o2 = ctx->ws[25];
    HIPCHK(ctx, ws_grow(vr, sizeof(double) * n * t));
    HIPCHK(ctx, ws_grow(ur, sizeof(double) * m * t));
    HIPCHK(ctx, ws_grow(av, sizeof(double) * m * t));
    HIPCHK(ctx, ws_grow(atu, sizeof(double) * n * t));
    HIPCHK(ctx, ws_grow(o1, sizeof(double) * t));
    HIPCHK(ctx, ws_grow(o2, sizeof(double) * t));
    HIPCHK(ctx, launch_col_to_row((int)n, t, ctx->d_V.as<double>(), npad, vr.as<double>(), t, st));
    HIPCHK(ctx, launch_col_to_row((int)m, t, ctx->d_U.as<double>(), mpad, ur.as<double>(), t, st));
    HIPCHK(ctx, launch_spmm_rowmajor((int)m, t, ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(),
                                     vr.as<double>(), av.as<double>(), st));
    HIPCHK(ctx, launch_spmm_rowmajor((int)n, t, ctx->rpT.as<int>(), ctx->ciT.as<int>(), ctx->vaT.as<double>(),
                                     ur.as<double>(), atu.as<double>(), st));
    HIPCHK(ctx, launch_resid_cols(av.as<double>(), ctx->d_U.as<double>(), mpad, dsig.as<double>(), (int)m, t,
                                  o1.as<double>(), st));
    HIPCHK(ctx, launch_resid_cols(atu.as<double>(), ctx->d_V.as<double>(), npad, dsig.as<double>(), (int)n, t,
                                  o2.as<double>(), st));
    std::vector<double> h1(t), h2(t);
    HIPCHK(ctx, hipMemcpyAsync(h1.data(), o1.p, sizeof(double) * t, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(h2.data(), o2.p, sizeof(double) * t, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    for (int c = 0; c < t; ++c) {
      ctx->resid[c] = std::sqrt(std::max(h1[c], h2[c])) / (normA > 0 ? normA : 1.0);
      info.max_triplet_resid = std::max(info.max_triplet_resid, ctx->resid[c]);
    }
    // Sec. 3.4.1: the residual ||A^T u_i - s_i v_i|| estimated from the
    // moments alone.  With S-hat = Q_S R and R^T J = B (one-sided Jacobi),
    // R = J Sigma W^T, so U_S1 = Q_S J(:, 1:r), W_S1 Sigma_S1^-1 =
    // B(:, 1:r) Sigma_S1^-2, and v_i = U_S1 q_i.  eq. residual (plain):
    // ||S_+ W_S1 Sigma_S1^-1 q_i - s_i^2 U_S1 q_i|| / s_i, S_+ = [S_1 .. S_M];
    // exp transform: the same with log(s_i^2) in place of s_i^2, scaled by mu
    // of eq. res_nonlinear from one computed residual (the largest).
    {
      const int LMe2 = LMe;
      std::vector<double> Bm((size_t)LMe2 * LMe2);
      HIPCHK(ctx, hipMemcpyAsync(Bm.data(), dRt.p, sizeof(double) * Bm.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
      const bool nt = (p.transform == CSVD_EXP);
      std::vector<double> Z((size_t)LM * t, 0.0), Qg((size_t)r * t);
      for (int c = 0; c < t; ++c) {
        const int i = sel[c];
        const double s2 = ctx->sigma[c] * ctx->sigma[c];
        const double g = nt ? std::log(s2) : s2;  // g^-1(s^2)
        for (int j = 0; j < r; ++j) {
          const double q = Jb[(size_t)i * re + j];
          const double w = q / (sS[perm[j]] * sS[perm[j]]);
          const double *bcol = Bm.data() + (size_t)perm[j] * LMe2;
          for (int a = 0; a < LM; ++a) Z[(size_t)c * LM + a] += bcol[a] * w;
          Qg[(size_t)c * r + j] = g * q;
        }
      }
      DevBuf &dZ = ctx->ws[26]; DevBuf &dQg = ctx->ws[27]; DevBuf &dE = ctx->ws[28]; DevBuf &dn = ctx->ws[29];
      HIPCHK(ctx, ws_grow(dZ, sizeof(double) * Z.size()));
      HIPCHK(ctx, ws_grow(dQg, sizeof(double) * Qg.size()));
      HIPCHK(ctx, ws_grow(dE, sizeof(double) * npad * t));
      HIPCHK(ctx, ws_grow(dn, sizeof(double) * t));
      HIPCHK(ctx, hipMemcpyAsync(dZ.p, Z.data(), sizeof(double) * Z.size(), hipMemcpyHostToDevice, st));
      HIPCHK(ctx, hipMemcpyAsync(dQg.p, Qg.data(), sizeof(double) * Qg.size(), hipMemcpyHostToDevice, st));
      // E = S_+ Z - V~ (g Q_sel) on the matrix cores, then column norms
      HIPCHK(ctx, launch_gemm((int)npad, t, LM, 1.0, ctx->d_S.as<double>() + (size_t)L * npad, npad,
                              dZ.as<double>(), LM, 0.0, dE.as<double>(), npad, st));
      HIPCHK(ctx, launch_gemm((int)npad, t, r, -1.0, Vt.as<double>(), npad, dQg.as<double>(), r, 1.0,
                              dE.as<double>(), npad, st));
      HIPCHK(ctx, launch_col_norms(dE.as<double>(), npad, (int)n, t, dn.as<double>(), st));
      std::vector<double> en(t);
      HIPCHK(ctx, hipMemcpyAsync(en.data(), dn.p, sizeof(double) * t, hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
      double mu = 1.0;
      if (nt) {  // eq. res_nonlinear: mu from the triplet with the largest computed residual
        int ip = 0;
        for (int c = 1; c < t; ++c)
          if (h2[c] > h2[ip]) ip = c;
        const double rt = en[ip] / ctx->sigma[ip];
        mu = rt > 0 ? std::sqrt(h2[ip]) / rt : 0.0;
      }
      ctx->resid_est.assign(t, 0.0);
      for (int c = 0; c < t; ++c) ctx->resid_est[c] = mu * en[c] / ctx->sigma[c] / (normA > 0 ? normA : 1.0);
    }
  }
  // resid_target > 0: triplets whose computed residual exceeds it are not
  // returned (their columns of U and V are closed up, order kept); the
  // count goes to csvd_info.dropped and the solve's status says so
  int t_out = t;
  ctx->resid_all_max = info.max_triplet_resid;
  if (p.resid_target > 0 && t > 0) {
    int w = 0;
    for (int c = 0; c < t; ++c) {
      if (!(ctx->resid[c] <= p.resid_target)) continue;
      if (w != c) {
        ctx->sigma[w] = ctx->sigma[c];
        ctx->resid[w] = ctx->resid[c];
        ctx->resid_est[w] = ctx->resid_est[c];
        HIPCHK(ctx, hipMemcpyAsync(ctx->d_U.as<double>() + (size_t)w * mpad, ctx->d_U.as<double>() + (size_t)c * mpad,
                                   sizeof(double) * mpad, hipMemcpyDeviceToDevice, st));
        HIPCHK(ctx, hipMemcpyAsync(ctx->d_V.as<double>() + (size_t)w * npad, ctx->d_V.as<double>() + (size_t)c * npad,
                                   sizeof(double) * npad, hipMemcpyDeviceToDevice, st));
      }
      ++w;
    }
    HIPCHK(ctx, hipStreamSynchronize(st));
    t_out = w;
    ctx->sigma.resize(w);
    ctx->resid.resize(w);
    ctx->resid_est.resize(w);
    info.max_triplet_resid = 0.0;
    for (int c = 0; c < w; ++c) info.max_triplet_resid = std::max(info.max_triplet_resid, ctx->resid[c]);
  }
  info.dropped = t - t_out;
  double t3 = now_ms();
  info.svd_sweeps_exhausted = sweeps_exhausted ? 1 : 0;
  info.rounds = R.round + 1;
  info.iterations = R.block ? R.iters_last : R.job->iters;
  info.iterations_total = R.iters_total;
  info.t_hat = t_out;
  info.converged = R.all_converged ? 1 : 0;
  info.n_shift = S;
  info.max_solve_resid_est = R.max_res_est;
  info.t_solve_ms = R.t_solve_end - R.t_start;
  info.t_lowrank_ms = t1 - t0;
  info.t_qr_ms = t2 - t1;
  info.t_extract_ms = t3 - t2;
  info.t_total_ms = t3 - R.t_start;
  info.window = R.block ? 0 : R.job->h.W;
  info.L_padded = R.spec.Lp;
  info.solver = R.block ? CSVD_SOLVER_BLOCK : CSVD_SOLVER_SINGLE;
  const double Lp = R.spec.Lp;
  int64_t nnz = ctx->nnz;
  if (R.block) {
    // one A product launch: per column group A, x gather (n x Lp), y write
    // (m x Lp); one A^T product launch: per group A^T, u gather (m x Lp), w
    // write (n x Lp)
    info.spmm_a_bytes = info.spmm_at_bytes = 0.0;
    info.basis_stored = 1;
    for (BlockJob *B : R.groups()) {
      const double lp = B->h.Lp;
      info.spmm_a_bytes += nnz * 12.0 + 4.0 * (m + 1) + 8.0 * lp * (n + m);
      info.spmm_at_bytes += nnz * 12.0 + 4.0 * (n + 1) + 8.0 * lp * (m + n);
      info.deflated += B->deflated_last;
      if (!B->stored_last) info.basis_stored = 0;
    }
    info.one_pass_steps = R.bjob->one_pass_last;
    info.column_groups = (int32_t)R.groups().size();
  } else {
    info.spmm_a_bytes = nnz * 12.0 + 4.0 * (m + 1) + 8.0 * Lp * (n + m);
    info.spmm_at_bytes = nnz * 12.0 + 4.0 * (n + 1) + 8.0 * Lp * (m + 4.0 * n);
    info.window_bytes = 8.0 * R.job->h.W * L * n + 64.0 * S * L * n;
  }
  ctx->solved = true;
  return CSVD_OK;
}

// Optional: true FP64 residual of every shifted solve, max over (shift, column)
// of ||V - (z I - A^T A) Y|| / ||V||.
int check_solves(SolveRun &R) {
  csvd_ctx *ctx = R.ctx;
  hipStream_t st = ctx->st;
  if (R.block) {  // the block solver keeps no per-shift solution vectors
    ctx->info.max_solve_resid_true = std::nan("");
    return CSVD_OK;
  }
  Job &J = *R.job;
  const int L = J.h.L, S = J.h.S;
  const int64_t n = ctx->n, m = ctx->m;
  DevBuf re, im, rowb, ub, gb;
  HIPCHK(ctx, re.alloc(sizeof(double) * n * L));
  HIPCHK(ctx, im.alloc(sizeof(double) * n * L));
  HIPCHK(ctx, rowb.alloc(sizeof(double) * n * 2 * L));
  HIPCHK(ctx, ub.alloc(sizeof(double) * m * 2 * L));
  HIPCHK(ctx, gb.alloc(sizeof(double) * n * 2 * L));
  std::vector<double> V((size_t)n * L), G((size_t)n * 2 * L), Yr((size_t)n * L), Yi((size_t)n * L);
  XFER(d2h_cols(ctx, V.data(), R.d_rhs.as<double>(), R.rhs_ld, n, L, st));
  double worst = 0;
  for (int s = 0; s < S; ++s) {
    HIPCHK(ctx, launch_get_solution(J.h, s, re.as<double>(), im.as<double>(), st));
    // [Re | Im] as one row-major n x 2L block, formed on the host
    HIPCHK(ctx, hipMemcpyAsync(Yr.data(), re.p, sizeof(double) * Yr.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(Yi.data(), im.p, sizeof(double) * Yi.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    std::vector<double> Yrow((size_t)n * 2 * L);
    for (int64_t i = 0; i < n; ++i)
      for (int l = 0; l < L; ++l) {
        Yrow[(size_t)i * 2 * L + l] = Yr[(size_t)l * n + i];
        Yrow[(size_t)i * 2 * L + L + l] = Yi[(size_t)l * n + i];
      }
    HIPCHK(ctx, hipMemcpyAsync(rowb.p, Yrow.data(), sizeof(double) * Yrow.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, launch_spmm_rowmajor((int)m, 2 * L, ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(),
                                     rowb.as<double>(), ub.as<double>(), st));
    HIPCHK(ctx, launch_spmm_rowmajor((int)n, 2 * L, ctx->rpT.as<int>(), ctx->ciT.as<int>(), ctx->vaT.as<double>(),
                                     ub.as<double>(), gb.as<double>(), st));
    HIPCHK(ctx, hipMemcpyAsync(G.data(), gb.p, sizeof(double) * G.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    const double zr = R.spec.shift_re[s], zi = R.spec.shift_im[s];
    for (int l = 0; l < L; ++l) {
      double rn = 0, vn = 0;
      for (int64_t i = 0; i < n; ++i) {
        const double yr = Yr[(size_t)l * n + i], yi = Yi[(size_t)l * n + i];
        const double gr = G[(size_t)i * 2 * L + l], gi = G[(size_t)i * 2 * L + L + l];
        const double v = V[(size_t)l * n + i];
        const double rr = v - (zr * yr - zi * yi - gr);
        const double ri = -(zr * yi + zi * yr - gi);
        rn += rr * rr + ri * ri;
        vn += v * v;
      }
      if (vn > 0) worst = std::max(worst, std::sqrt(rn / vn));
    }
  }
  ctx->info.max_solve_resid_true = worst;
  return CSVD_OK;
}

// Status of a finished solve: CSVD_ENOTCONV when a shifted solve stopped at
// max_iters or a dense SVD stopped at its sweep limit (triplets are still
// readable), CSVD_OK otherwise.
int finish_status(csvd_ctx *ctx) {
  if (!ctx->info.converged) {
    ctx->last_status = CSVD_ENOTCONV;
    ctx->err = "shifted solves reached max_iters before solve_rtol";
  } else if (ctx->info.svd_sweeps_exhausted) {
    ctx->last_status = CSVD_ENOTCONV;
    ctx->err = "a one-sided Jacobi SVD of step 3 or 5 reached its sweep limit";
  } else if (ctx->info.dropped > 0) {
    ctx->last_status = CSVD_ENOTCONV;
    ctx->err = std::to_string(ctx->info.dropped) + " triplet(s) above resid_target were not returned";
  } else {
    ctx->last_status = CSVD_OK;
  }
  return ctx->last_status;
}

}  // namespace csvd

// ============================================================================
// ABI
extern "C" {

int csvd_params_default(csvd_params *p) {
  if (!p) return CSVD_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->L = 16;
  p->M = 8;
  p->N = 32;
  p->ell = 1;
  p->delta = 1e-20;
  p->alpha = 0.1;
  p->transform = CSVD_PLAIN;
  p->precision = CSVD_FP64;
  p->solve_rtol = 1e-10;
  p->max_iters = 1000000;
  p->spurious_eps = 1e-12;
  p->seed = 2109;
  p->norm_a = 0.0;
  p->window = 0;
  p->check_solves = 0;
  p->solver = CSVD_SOLVER_AUTO;
  p->keep_basis = 1;
  p->cholqr_passes = 0;
  p->resid_target = 0.0;
  p->ell_adaptive = 0;
  return CSVD_OK;
}

int csvd_create(csvd_ctx **out, int64_t m, int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                const double *vals, int32_t on_device, void *hip_stream) {
  if (!out) return CSVD_EINVAL;
  *out = nullptr;
  std::unique_ptr<csvd_ctx> ctx(new csvd_ctx());
  csvd_ctx *c = ctx.get();
  if (n < 1 || m < n) return CSVD_EINVAL;
  if (nnz < 0 || nnz >= (int64_t)1 << 31 || m >= (int64_t)1 << 31) return CSVD_EINVAL;
  if (!rowptr || (nnz > 0 && (!colidx || !vals))) return CSVD_EINVAL;
  c->m = m;
  c->n = n;
  c->nnz = nnz;
  c->st = (hipStream_t)hip_stream;
  if (!on_device) {
    // every row pointer in [0, nnz] and non-decreasing before any entry is read
    if (rowptr[0] != 0 || rowptr[m] != nnz) return CSVD_EINVAL;
    for (int64_t i = 0; i < m; ++i)
      if (rowptr[i + 1] < rowptr[i] || rowptr[i + 1] > nnz) return CSVD_EINVAL;
    for (int64_t i = 0; i < m; ++i) {
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        if (colidx[k] < 0 || colidx[k] >= n) return CSVD_EINVAL;
        if (k > rowptr[i] && colidx[k] <= colidx[k - 1]) return CSVD_EINVAL;
        if (!std::isfinite(vals[k])) return CSVD_ENUMERIC;
      }
    }
  }
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (c->rp.alloc(sizeof(int) * (m + 1)) || c->ci.alloc(sizeof(int) * std::max<int64_t>(nnz, 1)) ||
      c->va.alloc(sizeof(double) * std::max<int64_t>(nnz, 1)) || c->rpT.alloc(sizeof(int) * (n + 1)) ||
      c->ciT.alloc(sizeof(int) * std::max<int64_t>(nnz, 1)) || c->vaT.alloc(sizeof(double) * std::max<int64_t>(nnz, 1)) ||
      c->work.alloc(sizeof(int) * (n + 8)))
    return CSVD_ENOMEM;
  if (hipMemcpyAsync(c->rp.p, rowptr, sizeof(int) * (m + 1), kind, c->st) != hipSuccess) return CSVD_EDEVICE;
  if (nnz > 0) {
    if (hipMemcpyAsync(c->ci.p, colidx, sizeof(int) * nnz, kind, c->st) != hipSuccess) return CSVD_EDEVICE;
    if (hipMemcpyAsync(c->va.p, vals, sizeof(double) * nnz, kind, c->st) != hipSuccess) return CSVD_EDEVICE;
  }
  if (on_device) {
    if (launch_check_csr((int)m, (int)n, c->rp.as<int>(), c->ci.as<int>(), c->va.as<double>(), (int)nnz,
                         c->work.as<int>(), c->st) != hipSuccess)
      return CSVD_EDEVICE;
    int flags[3] = {0, 0, 0};
    if (hipMemcpyAsync(flags, c->work.p, sizeof(flags), hipMemcpyDeviceToHost, c->st) != hipSuccess) return CSVD_EDEVICE;
    if (hipStreamSynchronize(c->st) != hipSuccess) return CSVD_EDEVICE;
    if (flags[0] || flags[1]) return CSVD_EINVAL;
    if (flags[2]) return CSVD_ENUMERIC;
  }
  if (launch_csr_transpose((int)m, (int)n, (int)nnz, c->rp.as<int>(), c->ci.as<int>(), c->va.as<double>(),
                           c->rpT.as<int>(), c->ciT.as<int>(), c->vaT.as<double>(), c->work.as<int>(),
                           c->st) != hipSuccess)
    return CSVD_EDEVICE;
  if (hipStreamSynchronize(c->st) != hipSuccess) return CSVD_EDEVICE;
  // long rows of A and of A^T for the block products (segment tables)
  {
    std::vector<int> rph((size_t)m + 1), rpth((size_t)n + 1);
    if (hipMemcpy(rph.data(), c->rp.p, sizeof(int) * (m + 1), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(rpth.data(), c->rpT.p, sizeof(int) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess)
      return CSVD_EDEVICE;
    const hipError_t e0 = c->lr[0].build(rph, c->st);
    if (e0 != hipSuccess) return hip_code(e0);
    const hipError_t e1 = c->lr[1].build(rpth, c->st);
    if (e1 != hipSuccess) return hip_code(e1);
  }
  *out = ctx.release();
  return CSVD_OK;
}

void csvd_destroy(csvd_ctx *ctx) { delete ctx; }

int csvd_trim(csvd_ctx *ctx) {
  if (!ctx) return CSVD_EINVAL;
  ctx->err.clear();
  if (hipStreamSynchronize(ctx->st) != hipSuccess) return set_err(ctx, CSVD_EDEVICE, "stream synchronize failed");
  csvd::release_idle_chunks();
  for (csvd::DevBuf &b : ctx->ws) b.release();
  return CSVD_OK;
}

const char *csvd_last_error(const csvd_ctx *ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int csvd_solve_interval(csvd_ctx *ctx, double a, double b, const csvd_params *p, const double *V_in) {
  if (!ctx) return CSVD_EINVAL;
  if (ctx->busy) return set_err(ctx, CSVD_ESTATE, "the context is held by a live server request");
  ctx->err.clear();
  ctx->solved = false;
  std::unique_ptr<SolveRun> R(new SolveRun());
  const bool mixed = p && p->precision == CSVD_MIXED;
  const int W = p ? pick_window(p) : 32;
  int rc = run_begin(*R, ctx, a, b, p, V_in, W, mixed, true);
  if (rc) return rc;
  KernelTimer timer;
  std::unique_ptr<BEngine> beng;
  std::unique_ptr<Engine> seng;
  if (R->block) {
    // every column group is one job of the engine; a round ends when all have
    beng.reset(new BEngine(ctx->st));
    HIPCHK(ctx, beng->init());
    for (BlockJob *B : R->groups()) HIPCHK(ctx, beng->start(B));
  } else {
    seng.reset(new Engine(ctx->st, W, mixed));
    HIPCHK(ctx, seng->init());
    HIPCHK(ctx, seng->add(R->job.get()));
  }
  // rounds of eq. iter1/iter2, then steps 3-5; with ell_adaptive steps 3-5
  // follow every round and decide whether another one runs
  while (true) {
    if (R->block) {
      BEngine &eng = *beng;
      const std::vector<BlockJob *> gs = R->groups();
      int64_t step = 0;
      while (true) {
        for (int q = 0; q < kBlockPoll; ++q, ++step) HIPCHK(ctx, eng.step(&timer, (step % 8) == 3));
        std::vector<BlockJob *> fin;
        HIPCHK(ctx, eng.poll(&fin));
        R->gdone += (int)fin.size();
        if (R->gdone == (int)gs.size()) {
          bool more = false;
          rc = run_after_round(*R, &more);
          if (rc) return rc;
          if (more) {
            for (BlockJob *B : gs) HIPCHK(ctx, eng.start(B));
            continue;
          }
          break;
        }
      }
    } else {
      Engine &eng = *seng;
      while (true) {
        HIPCHK(ctx, eng.run_window(&timer, 64));
        std::vector<Job *> fin;
        HIPCHK(ctx, eng.collect(&fin));
        if (!fin.empty()) {
          bool more = false;
          rc = run_after_round(*R, &more);
          if (rc) return rc;
          if (more) {
            HIPCHK(ctx, eng.add(R->job.get()));
            continue;
          }
          break;
        }
      }
    }
    rc = run_finalize(*R);
    if (rc) return rc;
    const bool mixed_stored = R->block && R->bjob->mixed && R->bjob->stored_last;
    const double resid_fp32 = ctx->resid_all_max;  // before any resid_target drop
    if (mixed_stored && !(resid_fp32 <= kMixedResidTarget)) {
      // FP64 refinement of a mixed-precision solve whose triplets miss the
      // mixed target: the moments are accumulated again from the basis
      // regenerated in FP64 (the histories and coefficients of the last round
      // are kept), then steps 3-5 run again
      int pending = 0;
      for (BlockJob *B : R->groups())
        if (B->stored_last) {
          HIPCHK(ctx, beng->regenerate(B));
          ++pending;
        }
      while (pending > 0) {
        for (int q = 0; q < kBlockPoll; ++q) HIPCHK(ctx, beng->step(&timer, false));
        std::vector<BlockJob *> fin;
        HIPCHK(ctx, beng->poll(&fin));
        pending -= (int)fin.size();
      }
      rc = run_finalize(*R);
      if (rc) return rc;
      ctx->info.mixed_refined = 1;
    }
    if (mixed_stored) ctx->info.mixed_resid_fp32 = resid_fp32;
    bool again = false;
    rc = run_next_round(*R, &again);
    if (rc) return rc;
    if (!again) break;
    R->gdone = 0;
    if (R->block)
      for (BlockJob *B : R->groups()) HIPCHK(ctx, beng->start(B));
    else
      HIPCHK(ctx, seng->add(R->job.get()));
  }
  if (p->check_solves) {
    rc = check_solves(*R);
    if (rc) return rc;
  }
  double avg[KernelTimer::kKinds];
  int64_t cnt[KernelTimer::kKinds];
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  timer.summarize(avg, cnt);
  ctx->info.moments_ms = avg[3];
  ctx->info.spmm_a_ms = avg[0];
  ctx->info.spmm_at_ms = avg[1];
  if (R->block) ctx->info.rest_ms = avg[2];
  else ctx->info.window_ms = avg[2];
  ctx->info.spmm_samples = cnt[0];
  ctx->job = std::move(R->job);
  ctx->spec = R->spec;
  return finish_status(ctx);
}

int csvd_get_triplets(csvd_ctx *ctx, int64_t *t_hat, int64_t capacity, double *sigma, double *U, double *V,
                      double *resid) {
  if (!ctx || !t_hat) return CSVD_EINVAL;
  if (ctx->busy) return set_err(ctx, CSVD_ESTATE, "the context is held by a live server request");
  if (!ctx->solved) return set_err(ctx, CSVD_ESTATE, "no solve has completed on this context");
  const int64_t t = (int64_t)ctx->sigma.size();
  *t_hat = t;
  if (capacity == 0) return CSVD_OK;
  if (capacity < t) return set_err(ctx, CSVD_EINVAL, "capacity smaller than t_hat");
  if (sigma) std::memcpy(sigma, ctx->sigma.data(), sizeof(double) * t);
  if (resid) std::memcpy(resid, ctx->resid.data(), sizeof(double) * t);
  if (t > 0 && U) XFER(d2h_cols(ctx, U, ctx->d_U.as<double>(), ctx->mpad, ctx->m, t, ctx->st));
  if (t > 0 && V) XFER(d2h_cols(ctx, V, ctx->d_V.as<double>(), ctx->npad, ctx->n, t, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return CSVD_OK;
}

int csvd_get_residual_estimates(csvd_ctx *ctx, int64_t capacity, double *est) {
  if (!ctx || (capacity > 0 && !est)) return CSVD_EINVAL;
  if (ctx->busy) return set_err(ctx, CSVD_ESTATE, "the context is held by a live server request");
  if (!ctx->solved) return set_err(ctx, CSVD_ESTATE, "no solve has completed on this context");
  const int64_t t = (int64_t)ctx->resid_est.size();
  if (capacity < t) return set_err(ctx, CSVD_EINVAL, "capacity smaller than t_hat");
  if (t > 0) std::memcpy(est, ctx->resid_est.data(), sizeof(double) * t);
  return CSVD_OK;
}

int csvd_get_info(csvd_ctx *ctx, csvd_info *info) {
  if (!ctx || !info) return CSVD_EINVAL;
  if (ctx->busy) return set_err(ctx, CSVD_ESTATE, "the context is held by a live server request");
  if (!ctx->solved) return set_err(ctx, CSVD_ESTATE, "no solve has completed on this context");
  *info = ctx->info;
  return CSVD_OK;
}

int csvd_get_moment(csvd_ctx *ctx, int32_t k, double *S_k) {
  if (!ctx || !S_k) return CSVD_EINVAL;
  if (ctx->busy) return set_err(ctx, CSVD_ESTATE, "the context is held by a live server request");
  if (!ctx->solved) return set_err(ctx, CSVD_ESTATE, "no solve has completed on this context");
  if (k < 0 || k > ctx->M) return set_err(ctx, CSVD_EINVAL, "moment index out of range");
  const double *src = ctx->d_S.as<double>() + (size_t)k * ctx->L * ctx->npad;
  XFER(d2h_cols(ctx, S_k, src, ctx->npad, ctx->n, ctx->L, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return CSVD_OK;
}

int csvd_get_solution(csvd_ctx *ctx, int32_t j, double *Y_re, double *Y_im) {
  if (!ctx || !Y_re || !Y_im) return CSVD_EINVAL;
  if (ctx->busy) return set_err(ctx, CSVD_ESTATE, "the context is held by a live server request");
  if (!ctx->solved || !ctx->job) return set_err(ctx, CSVD_ESTATE, "no solve has completed on this context");
  if (j < 0 || j >= ctx->S) return set_err(ctx, CSVD_EINVAL, "shift index out of range");
  DevBuf re, im;
  HIPCHK(ctx, re.alloc(sizeof(double) * ctx->n * ctx->L));
  HIPCHK(ctx, im.alloc(sizeof(double) * ctx->n * ctx->L));
  HIPCHK(ctx, launch_get_solution(ctx->job->h, j, re.as<double>(), im.as<double>(), ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(Y_re, re.p, sizeof(double) * ctx->n * ctx->L, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(Y_im, im.p, sizeof(double) * ctx->n * ctx->L, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return CSVD_OK;
}

int csvd_quadrature(double a, double b, const csvd_params *p, double *shift_re, double *shift_im, double *w_re,
                    double *w_im, double *c_re, double *c_im) {
  if (!p) return CSVD_EINVAL;
  if (!(0.0 <= a && a < b) || p->N < 2 || p->N % 2 || p->M < 0 || !(p->alpha > 0)) return CSVD_EINVAL;
  if (p->transform == CSVD_EXP && !(a > 0)) return CSVD_EINVAL;
  SolveSpec s;
  quadrature(a, b, p->N, p->M, p->alpha, p->transform, &s);
  for (int j = 0; j < s.S; ++j) {
    if (shift_re) shift_re[j] = s.shift_re[j];
    if (shift_im) shift_im[j] = s.shift_im[j];
    if (w_re) w_re[j] = s.c_re[(size_t)j * (p->M + 1)];
    if (w_im) w_im[j] = s.c_im[(size_t)j * (p->M + 1)];
  }
  for (size_t i = 0; i < s.c_re.size(); ++i) {
    if (c_re) c_re[i] = s.c_re[i];
    if (c_im) c_im[i] = s.c_im[i];
  }
  return CSVD_OK;
}

int csvd_spmm(csvd_ctx *ctx, int32_t transpose, int64_t k, const double *X, double *Y) {
  if (!ctx || !X || !Y || k < 1) return CSVD_EINVAL;
  const int64_t rows_out = transpose ? ctx->n : ctx->m;
  const int64_t rows_in = transpose ? ctx->m : ctx->n;
  DevBuf xc, xr, yr, yc;
  HIPCHK(ctx, xc.alloc(sizeof(double) * rows_in * k));
  HIPCHK(ctx, xr.alloc(sizeof(double) * rows_in * k));
  HIPCHK(ctx, yr.alloc(sizeof(double) * rows_out * k));
  HIPCHK(ctx, yc.alloc(sizeof(double) * rows_out * k));
  HIPCHK(ctx, hipMemcpyAsync(xc.p, X, sizeof(double) * rows_in * k, hipMemcpyHostToDevice, ctx->st));
  HIPCHK(ctx, launch_col_to_row((int)rows_in, (int)k, xc.as<double>(), rows_in, xr.as<double>(), k, ctx->st));
  if (transpose)
    HIPCHK(ctx, launch_spmm_rowmajor((int)ctx->n, k, ctx->rpT.as<int>(), ctx->ciT.as<int>(), ctx->vaT.as<double>(),
                                     xr.as<double>(), yr.as<double>(), ctx->st));
  else
    HIPCHK(ctx, launch_spmm_rowmajor((int)ctx->m, k, ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(),
                                     xr.as<double>(), yr.as<double>(), ctx->st));
  HIPCHK(ctx, launch_row_to_col((int)rows_out, (int)k, yr.as<double>(), k, yc.as<double>(), rows_out, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(Y, yc.p, sizeof(double) * rows_out * k, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return CSVD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free sparse product.  The four staging blocks of csvd_spmm (X
// and Y, each column-major and row-major) live in one file-scope device
// array instead of fresh allocations.  Every GPU the library runs on holds
// its own copy of the array until the process ends.  Host code never hands
// the array's name to a kernel or a copy (in host code it is only a
// stand-in symbol): the device address is taken once per device with
// hipGetSymbolAddress and that pointer is used everywhere.
constexpr int64_t kNoAllocDoubles = (int64_t)4 << 20;  // 32 MiB of staging per device
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call per device)
int scratch_on_current_device(csvd_ctx *ctx, double **out) {
  int dev = 0;
  HIPCHK(ctx, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_err(ctx, CSVD_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_err(ctx, CSVD_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return CSVD_OK;
}
}  // namespace

extern "C" {

int csvd_spmm_noalloc(csvd_ctx *ctx, int32_t transpose, int64_t k, const double *X, double *Y) {
  if (!ctx || !X || !Y || k < 1) return CSVD_EINVAL;
  const int64_t rows_out = transpose ? ctx->n : ctx->m;
  const int64_t rows_in = transpose ? ctx->m : ctx->n;
  if (k > kNoAllocDoubles || 2 * k * (rows_in + rows_out) > kNoAllocDoubles)
    return set_err(ctx, CSVD_EINVAL,
                   "csvd_spmm_noalloc: 2 k (rows of X + rows of Y) = " + std::to_string(2 * k * (rows_in + rows_out)) +
                       " doubles exceeds its staging limit of " + std::to_string(kNoAllocDoubles));
  double *s = nullptr;
  XFER(scratch_on_current_device(ctx, &s));
  double *xc = s, *xr = xc + rows_in * k, *yr = xr + rows_in * k, *yc = yr + rows_out * k;
  HIPCHK(ctx, hipMemcpyAsync(xc, X, sizeof(double) * rows_in * k, hipMemcpyHostToDevice, ctx->st));
  HIPCHK(ctx, launch_col_to_row((int)rows_in, (int)k, xc, rows_in, xr, k, ctx->st));
  if (transpose)
    HIPCHK(ctx, launch_spmm_rowmajor((int)ctx->n, k, ctx->rpT.as<int>(), ctx->ciT.as<int>(), ctx->vaT.as<double>(), xr,
                                     yr, ctx->st));
  else
    HIPCHK(ctx, launch_spmm_rowmajor((int)ctx->m, k, ctx->rp.as<int>(), ctx->ci.as<int>(), ctx->va.as<double>(), xr,
                                     yr, ctx->st));
  HIPCHK(ctx, launch_row_to_col((int)rows_out, (int)k, yr, k, yc, rows_out, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(Y, yc, sizeof(double) * rows_out * k, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return CSVD_OK;
}

int csvd_dense_gemm(int64_t R, int64_t N, int64_t K, const double *A, const double *B, double *Cm) {
  if (R < 1 || N < 1 || K < 1 || !A || !B || !Cm) return CSVD_EINVAL;
  DevBuf a, b, c;
  if (a.alloc(sizeof(double) * R * K) || b.alloc(sizeof(double) * K * N) || c.alloc(sizeof(double) * R * N))
    return CSVD_ENOMEM;
  if (hipMemcpy(a.p, A, sizeof(double) * R * K, hipMemcpyHostToDevice) != hipSuccess) return CSVD_EDEVICE;
  if (hipMemcpy(b.p, B, sizeof(double) * K * N, hipMemcpyHostToDevice) != hipSuccess) return CSVD_EDEVICE;
  if (launch_gemm((int)R, (int)N, (int)K, 1.0, a.as<double>(), R, b.as<double>(), K, 0.0, c.as<double>(), R,
                  nullptr) != hipSuccess)
    return CSVD_EDEVICE;
  if (hipMemcpy(Cm, c.p, sizeof(double) * R * N, hipMemcpyDeviceToHost) != hipSuccess) return CSVD_EDEVICE;
  return CSVD_OK;
}

int csvd_get_transpose(csvd_ctx *ctx, int32_t *rowptr, int32_t *colidx, double *vals) {
  if (!ctx || !rowptr) return CSVD_EINVAL;
  HIPCHK(ctx, hipMemcpyAsync(rowptr, ctx->rpT.p, sizeof(int) * (ctx->n + 1), hipMemcpyDeviceToHost, ctx->st));
  if (ctx->nnz > 0 && colidx)
    HIPCHK(ctx, hipMemcpyAsync(colidx, ctx->ciT.p, sizeof(int) * ctx->nnz, hipMemcpyDeviceToHost, ctx->st));
  if (ctx->nnz > 0 && vals)
    HIPCHK(ctx, hipMemcpyAsync(vals, ctx->vaT.p, sizeof(double) * ctx->nnz, hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return CSVD_OK;
}

}  // extern "C"

// ============================================================================
// Batched solves and the serving loop.
extern "C" {

// Worker threads, each with its own stream, that run the epilogues (steps
// 3-5) of finished batch jobs while the calling thread keeps stepping the
// others.  An epilogue touches only its own context, and its kernels reduce
// in a fixed order, so the results do not depend on the stream or thread.
class FinishPool {
 public:
  using Fn = std::function<void(int, hipStream_t)>;
  FinishPool(int nthreads, Fn fn) : fn_(std::move(fn)) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (int i = 0; i < nthreads; ++i) th_.emplace_back([this, dev] { run(dev); });
  }
  ~FinishPool() { finish(); }
  FinishPool(const FinishPool &) = delete;
  FinishPool &operator=(const FinishPool &) = delete;
  void push(int i) {
    {
      std::lock_guard<std::mutex> g(mu_);
      q_.push_back(i);
    }
    cv_.notify_one();
  }
  // runs what is queued, then ends the threads
  void finish() {
    {
      std::lock_guard<std::mutex> g(mu_);
      done_ = true;
    }
    cv_.notify_all();
    for (std::thread &t : th_)
      if (t.joinable()) t.join();
  }

 private:
  void run(int dev) {
    (void)hipSetDevice(dev);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    for (;;) {
      int i;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return done_ || !q_.empty(); });
        if (q_.empty()) break;
        i = q_.front();
        q_.pop_front();
      }
      fn_(i, st);
    }
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  }
  Fn fn_;
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<int> q_;
  bool done_ = false;
};
constexpr int kFinishThreads = 8;

int csvd_solve_batch(int32_t count, csvd_ctx *const *ctxs, const double *a, const double *b,
                     const csvd_params *params, const double *const *V_in, int32_t *status) {
  if (count < 1 || !ctxs || !a || !b || !params || !status) return CSVD_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return CSVD_EINVAL;
    // each problem owns its context's results: a context listed twice would
    // have two solves writing its moments and triplets at once
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return set_err(ctxs[i], CSVD_EINVAL, "a context is listed twice in the batch");
    if (ctxs[i]->busy) return set_err(ctxs[i], CSVD_ESTATE, "the context is held by a live server request");
  }
  hipStream_t st = ctxs[0]->st;
  const int W = pick_window(&params[0]);
  const bool mixed = params[0].precision == CSVD_MIXED;
  if (use_block(&params[0], ctxs[0]->n)) {
    std::vector<std::unique_ptr<SolveRun>> runs(count);
    std::map<BlockJob *, int> owner;
    // epilogues in flight on the workers, and problems whose epilogue started
    // another round (ell_adaptive): only the loop below touches the engine
    std::mutex rq_mu;
    std::condition_variable rq_cv;
    std::vector<int> requeue;
    int in_epilogue = 0;
    auto finish_job = [&](int i, hipStream_t fst) {
      SolveRun &R = *runs[i];
      csvd_ctx *ctx = ctxs[i];
      int rc;
      bool again = false;
      try {
        rc = run_finalize(R, fst);
        if (!rc) rc = run_next_round(R, &again, fst);
      } catch (...) {
        rc = set_err(ctx, CSVD_ENOMEM, "host allocation failed in the epilogue");
      }
      if (!rc && again) {
        std::lock_guard<std::mutex> g(rq_mu);
        requeue.push_back(i);
        --in_epilogue;
        rq_cv.notify_all();
        return;
      }
      if (rc) {
        status[i] = rc;
      } else {
        ctx->spec = R.spec;
        status[i] = finish_status(ctx);
      }
      R.bjob.reset();  // free the basis histories
      std::lock_guard<std::mutex> g(rq_mu);
      --in_epilogue;
      rq_cv.notify_all();
    };
    FinishPool pool(std::min<int>(count, kFinishThreads), finish_job);
    BEngine eng(st);
    if (eng.init() != hipSuccess) return CSVD_EDEVICE;
    for (int i = 0; i < count; ++i) {
      status[i] = CSVD_OK;
      ctxs[i]->err.clear();
      ctxs[i]->solved = false;
      if (ctxs[i]->st != st || !use_block(&params[i], ctxs[i]->n) ||
          (params[i].solver == CSVD_SOLVER_BLOCK && pad_L(params[i].L) > kBlockMaxLp)) {
        status[i] = set_err(ctxs[i], CSVD_EINVAL, "batched problems must share the stream and the solver");
        continue;
      }
      runs[i].reset(new SolveRun());
      int rc = run_begin(*runs[i], ctxs[i], a[i], b[i], &params[i], V_in ? V_in[i] : nullptr, W, false);
      if (rc) {
        status[i] = rc;
        runs[i].reset();
        continue;
      }
      // a batch keeps FP64 stored bases: the FP64 refinement of a mixed
      // solve needs the engine after the epilogue, which a batch runs on
      // worker threads
      runs[i]->bjob->mixed = false;
      owner[runs[i]->bjob.get()] = i;
      if (eng.start(runs[i]->bjob.get()) != hipSuccess) return CSVD_EDEVICE;
    }
    while (true) {
      std::vector<int> restart;
      {
        std::unique_lock<std::mutex> g(rq_mu);
        if (eng.active() == 0) {  // nothing to step: wait for the epilogues
          rq_cv.wait(g, [&] { return in_epilogue == 0 || !requeue.empty(); });
          if (requeue.empty()) break;
        }
        restart.swap(requeue);
      }
      for (int i : restart)
        if (eng.start(runs[i]->bjob.get()) != hipSuccess) return CSVD_EDEVICE;
      for (int q = 0; q < kBlockPoll; ++q)
        if (eng.step(nullptr, false) != hipSuccess) return CSVD_EDEVICE;
      std::vector<BlockJob *> fin;
      if (eng.poll(&fin) != hipSuccess) return CSVD_EDEVICE;
      for (BlockJob *j : fin) {
        const int i = owner[j];
        SolveRun &R = *runs[i];
        bool more = false;
        int rc = run_after_round(R, &more);
        if (rc) {
          status[i] = rc;
          continue;
        }
        if (more) {
          if (eng.start(j) != hipSuccess) return CSVD_EDEVICE;
          continue;
        }
        {
          std::lock_guard<std::mutex> g(rq_mu);
          ++in_epilogue;
        }
        pool.push(i);  // steps 3-5 on a worker while the others go on
      }
    }
    pool.finish();
    return CSVD_OK;
  }
  std::vector<std::unique_ptr<SolveRun>> runs(count);
  std::map<Job *, int> owner;
  Engine eng(st, W, mixed);
  if (eng.init() != hipSuccess) return CSVD_EDEVICE;
  for (int i = 0; i < count; ++i) {
    status[i] = CSVD_OK;
    ctxs[i]->err.clear();
    ctxs[i]->solved = false;
    if (ctxs[i]->st != st || (params[i].precision == CSVD_MIXED) != mixed || pick_window(&params[i]) != W) {
      status[i] = set_err(ctxs[i], CSVD_EINVAL, "batched problems must share stream, precision and window");
      continue;
    }
    runs[i].reset(new SolveRun());
    int rc = run_begin(*runs[i], ctxs[i], a[i], b[i], &params[i], V_in ? V_in[i] : nullptr, W, mixed);
    if (rc) {
      status[i] = rc;
      runs[i].reset();
      continue;
    }
    owner[runs[i]->job.get()] = i;
    if (eng.add(runs[i]->job.get()) != hipSuccess) return CSVD_EDEVICE;
  }
  while (eng.active() > 0) {
    if (eng.run_window(nullptr, 0) != hipSuccess) return CSVD_EDEVICE;
    std::vector<Job *> fin;
    if (eng.collect(&fin) != hipSuccess) return CSVD_EDEVICE;
    for (Job *j : fin) {
      const int i = owner[j];
      SolveRun &R = *runs[i];
      bool more = false;
      int rc = run_after_round(R, &more);
      if (rc) {
        status[i] = rc;
        continue;
      }
      if (more) {
        if (eng.add(j) != hipSuccess) return CSVD_EDEVICE;
        continue;
      }
      rc = run_finalize(R);
      if (!rc && R.spec.p.check_solves) rc = check_solves(R);
      if (rc) {
        status[i] = rc;
        continue;
      }
      csvd_ctx *ctx = ctxs[i];
      ctx->job = std::move(R.job);
      ctx->spec = R.spec;
      status[i] = finish_status(ctx);
    }
  }
  return CSVD_OK;
}

}  // extern "C"

struct csvd_server {
  hipStream_t st = nullptr;
  int64_t budget = 0;
  int32_t max_batch = 0;
  int64_t used = 0;
  std::string err;
  std::unique_ptr<Engine> eng[2];  // single-vector solver: FP64, MIXED
  std::unique_ptr<BEngine> beng;   // block solver
  std::map<BlockJob *, int64_t> bowner;
  struct Req {
    csvd_ctx *ctx = nullptr;
    double a = 0, b = 0;
    csvd_params p{};
    std::vector<double> V;
    bool hasV = false;
    int state = 0;  // 0 queued, 1 running, 2 done, 3 cancelled
    int status = CSVD_OK;
    int64_t bytes = 0;
    std::unique_ptr<SolveRun> run;
  };
  std::map<int64_t, Req> reqs;
  std::deque<int64_t> queue;
  std::map<Job *, int64_t> owner;
  int64_t next_id = 0;
};

static int64_t request_bytes(const csvd_ctx *ctx, const csvd_params *p) {
  const int Lp = pad_L(p->L), S = p->N / 2, W = pick_window(p);
  const int64_t npad = round_up(ctx->n, kRowPad), mpad = round_up(ctx->m, kRowPad);
  const int64_t LM = (int64_t)p->L * p->M;
  int64_t b;
  if (use_block(p, ctx->n)) {
    const int bLp = block_Lp(p->L);
    const int64_t kc = std::min<int64_t>(p->max_iters, (int64_t)std::ceil(3.5 * (double)ctx->n / bLp) + 32);
    b = (int64_t)BlockJob::bytes_needed(ctx->m, ctx->n, ctx->nnz, bLp, S, (int)kc, p->L, p->M + 1);
  } else {
    b = (int64_t)Job::bytes_needed(ctx->m, ctx->n, ctx->nnz, Lp, S, W, p->precision == CSVD_MIXED);
  }
  // moments + QR copy + V~ + A V~ (row and column) + triplet vectors
  b += 8 * npad * (p->M + 1) * (int64_t)p->L + 8 * npad * LM * 2 + 8 * (mpad + ctx->m) * LM + 8 * ctx->n * LM;
  b += 8 * (mpad + npad) * LM;
  return b;
}

static int srv_err(csvd_server *s, int code, const std::string &m) {
  if (s) s->err = m;
  return code;
}

constexpr int64_t kSrvFreeReserve = 2LL << 30;  // device memory left free when admitting beside others

static int srv_admit(csvd_server *s) {
  int running = 0;
  for (auto &kv : s->reqs)
    if (kv.second.state == 1) ++running;
  while (!s->queue.empty() && running < s->max_batch) {
    const int64_t id = s->queue.front();
    auto &R = s->reqs[id];
    if (s->used + R.bytes > s->budget) break;  // FIFO: wait for memory
    // the budget counts live requests only: results that finished requests
    // keep in their contexts (and other users of the device) take memory
    // outside it.  While others run, a request that would not fit what is
    // really free waits; with none running it is tried (run_begin then
    // fails it alone with CSVD_ENOMEM if it does not fit)
    if (running > 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess && (int64_t)fr < R.bytes + kSrvFreeReserve) {
        release_idle_chunks();
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && (int64_t)fr < R.bytes + kSrvFreeReserve) break;
      }
    }
    s->queue.pop_front();
    const bool mixed = R.p.precision == CSVD_MIXED;
    Engine *e = s->eng[mixed ? 1 : 0].get();
    R.run.reset(new SolveRun());
    int rc = run_begin(*R.run, R.ctx, R.a, R.b, &R.p, R.hasV ? R.V.data() : nullptr, e->W(), mixed);
    if (rc) {
      R.state = 2;
      R.status = rc;
      R.run.reset();
      R.ctx->busy = false;
      continue;
    }
    // a stored basis (no second pass) only when its largest possible size
    // (Kcap + 1 blocks, in whole chunks) also fits the budget; the budget
    // then holds it until the request is done.  Served block solves keep FP64
    // bases, as batches do: the FP64 refinement of a mixed solve whose FP32
    // basis misses the mixed target runs only in csvd_solve_interval
    if (R.run->bjob) {
      BlockJob &B = *R.run->bjob;
      B.mixed = false;
      const int64_t blocks = ((int64_t)B.Kcap + 1 + kStoreChunk - 1) / kStoreChunk * kStoreChunk;
      const int64_t sb = blocks * B.h.n * B.h.Lp * (B.mixed ? 4 : 8);
      if (R.p.keep_basis != 0 && s->used + R.bytes + sb <= s->budget) {
        B.want_store = true;
        R.bytes += sb;
      } else {
        B.want_store = false;
      }
    }
    s->used += R.bytes;
    R.state = 1;
    if (R.run->block) {
      s->bowner[R.run->bjob.get()] = id;
      if (s->beng->start(R.run->bjob.get()) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "engine start failed");
    } else {
      s->owner[R.run->job.get()] = id;
      if (e->add(R.run->job.get()) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "engine add failed");
    }
    ++running;
  }
  return CSVD_OK;
}

static void srv_release(csvd_server *s, csvd_server::Req &R) {
  s->used -= R.bytes;
  R.ctx->busy = false;
  for (auto it = s->owner.begin(); it != s->owner.end();) {
    if (R.run && it->first == R.run->job.get()) it = s->owner.erase(it);
    else ++it;
  }
  for (auto it = s->bowner.begin(); it != s->bowner.end();) {
    if (R.run && it->first == R.run->bjob.get()) it = s->bowner.erase(it);
    else ++it;
  }
}

// finishes a request whose solves are done: dense steps and bookkeeping.
// Returns true instead when ell_adaptive started another round (the caller
// restarts the request's job).
static bool srv_finish(csvd_server *s, csvd_server::Req &R) {
  int r2 = run_finalize(*R.run);
  bool again = false;
  if (!r2) r2 = run_next_round(*R.run, &again);
  if (!r2 && again) return true;
  if (!r2 && R.p.check_solves) r2 = check_solves(*R.run);
  if (!r2) {
    if (R.run->job) R.ctx->job = std::move(R.run->job);
    R.ctx->spec = R.run->spec;
    r2 = finish_status(R.ctx);
  }
  R.status = r2;
  R.state = 2;
  srv_release(s, R);
  R.run.reset();
  return false;
}

extern "C" {

int csvd_server_create(csvd_server **srv, int64_t budget_bytes, int32_t max_batch, void *hip_stream) {
  if (!srv || budget_bytes <= 0 || max_batch < 1) return CSVD_EINVAL;
  std::unique_ptr<csvd_server> s(new csvd_server());
  s->st = (hipStream_t)hip_stream;
  s->budget = budget_bytes;
  s->max_batch = max_batch;
  for (int i = 0; i < 2; ++i) {
    s->eng[i].reset(new Engine(s->st, 32, i == 1));
    if (s->eng[i]->init() != hipSuccess) return CSVD_EDEVICE;
  }
  s->beng.reset(new BEngine(s->st));
  if (s->beng->init() != hipSuccess) return CSVD_EDEVICE;
  *srv = s.release();
  return CSVD_OK;
}

int csvd_server_submit(csvd_server *s, csvd_ctx *ctx, double a, double b, const csvd_params *p, const double *V_in,
                       int64_t *req) {
  if (!s || !ctx || !p || !req) return CSVD_EINVAL;
  int rc = check_params(ctx, a, b, p);
  if (rc) return srv_err(s, rc, ctx->err);
  if (pick_window(p) != 32) return srv_err(s, CSVD_EINVAL, "served requests use the server's window (0 or 32)");
  if (ctx->st != s->st) return srv_err(s, CSVD_EINVAL, "context stream differs from the server stream");
  if (ctx->busy) return srv_err(s, CSVD_ESTATE, "the context already has a live request");
  if (p->solver == CSVD_SOLVER_BLOCK && pad_L(p->L) > kBlockMaxLp)
    return srv_err(s, CSVD_EINVAL, "served block solves need L <= 64 (wider L: solver AUTO or SINGLE)");
  const int64_t bytes = request_bytes(ctx, p);
  if (bytes > s->budget) return srv_err(s, CSVD_ENOMEM, "request footprint exceeds the server budget");
  const int64_t id = s->next_id++;
  auto &R = s->reqs[id];
  R.ctx = ctx;
  R.a = a;
  R.b = b;
  R.p = *p;
  R.bytes = bytes;
  if (V_in) {
    R.V.assign(V_in, V_in + (size_t)ctx->n * p->L);
    R.hasV = true;
  }
  s->queue.push_back(id);
  ctx->busy = true;
  ctx->solved = false;
  *req = id;
  return CSVD_OK;
}

int csvd_server_step(csvd_server *s, int32_t steps, int32_t *n_active) {
  if (!s) return CSVD_EINVAL;
  int rc = srv_admit(s);
  if (rc) return rc;
  int done_steps = 0;
  do {
    bool any = false;
    if (s->beng->active() > 0) {
      any = true;
      for (int q = 0; q < kBlockPoll; ++q)
        if (s->beng->step(nullptr, false) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "block step failed");
      std::vector<BlockJob *> fin;
      if (s->beng->poll(&fin) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "block poll failed");
      for (BlockJob *j : fin) {
        auto it = s->bowner.find(j);
        if (it == s->bowner.end()) continue;
        const int64_t rid = it->second;
        auto &R = s->reqs[rid];
        bool more = false;
        int r2 = run_after_round(*R.run, &more);
        if (!r2 && more) {
          if (s->beng->start(j) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "block start failed");
          continue;
        }
        if (r2) {
          s->bowner.erase(it);
          R.status = r2;
          R.state = 2;
          srv_release(s, R);
          R.run.reset();
          continue;
        }
        // srv_finish releases the request (and its entry in bowner) unless
        // ell_adaptive started another round
        if (srv_finish(s, R)) {
          if (s->beng->start(j) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "block start failed");
          continue;
        }
      }
    }
    for (int ei = 0; ei < 2; ++ei) {
      Engine &e = *s->eng[ei];
      if (e.active() == 0) continue;
      any = true;
      if (e.run_window(nullptr, 0) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "window launch failed");
      std::vector<Job *> fin;
      if (e.collect(&fin) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "collect failed");
      for (Job *j : fin) {
        auto it = s->owner.find(j);
        if (it == s->owner.end()) continue;
        const int64_t rid = it->second;
        auto &R = s->reqs[rid];
        s->owner.erase(it);
        bool more = false;
        int r2 = run_after_round(*R.run, &more);
        if (!r2 && more) {
          s->owner[j] = rid;
          if (e.add(j) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "engine add failed");
          continue;
        }
        if (!r2) {
          r2 = run_finalize(*R.run);
          bool again = false;
          if (!r2) r2 = run_next_round(*R.run, &again);
          if (!r2 && again) {  // another round (ell_adaptive)
            s->owner[j] = rid;
            if (e.add(j) != hipSuccess) return srv_err(s, CSVD_EDEVICE, "engine add failed");
            continue;
          }
        }
        if (!r2 && R.p.check_solves) r2 = check_solves(*R.run);
        if (!r2) {
          R.ctx->job = std::move(R.run->job);
          R.ctx->spec = R.run->spec;
          r2 = finish_status(R.ctx);
        }
        R.status = r2;
        R.state = 2;
        srv_release(s, R);
        R.run.reset();
      }
    }
    rc = srv_admit(s);
    if (rc) return rc;
    if (!any) break;
    done_steps += 32;
  } while (done_steps < steps);
  if (n_active) {
    int na = 0;
    for (auto &kv : s->reqs)
      if (kv.second.state == 0 || kv.second.state == 1) ++na;
    *n_active = na;
  }
  return CSVD_OK;
}

int csvd_server_poll(csvd_server *s, int64_t req, int32_t *done, int32_t *status) {
  if (!s || !done) return CSVD_EINVAL;
  auto it = s->reqs.find(req);
  if (it == s->reqs.end()) return srv_err(s, CSVD_EINVAL, "unknown request id");
  *done = it->second.state >= 2 ? 1 : 0;
  if (status) *status = it->second.state == 3 ? CSVD_ESTATE : it->second.status;
  return CSVD_OK;
}

int csvd_server_cancel(csvd_server *s, int64_t req) {
  if (!s) return CSVD_EINVAL;
  auto it = s->reqs.find(req);
  if (it == s->reqs.end()) return srv_err(s, CSVD_EINVAL, "unknown request id");
  auto &R = it->second;
  if (R.state == 0) {
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), req), s->queue.end());
    R.ctx->busy = false;
  } else if (R.state == 1) {
    if (R.run->block) s->beng->remove(R.run->bjob.get());
    else
      for (int ei = 0; ei < 2; ++ei) s->eng[ei]->remove(R.run->job.get());
    srv_release(s, R);
    R.run.reset();
  } else {
    return CSVD_OK;
  }
  R.state = 3;
  R.status = CSVD_ESTATE;
  return CSVD_OK;
}

const char *csvd_server_last_error(const csvd_server *s) { return s ? s->err.c_str() : "null server"; }

void csvd_server_destroy(csvd_server *s) {
  if (!s) return;
  // requests that never finished release their contexts (which, by the
  // contract of csvd_server_submit, are still alive)
  for (auto &kv : s->reqs)
    if (kv.second.state == 0 || kv.second.state == 1) kv.second.ctx->busy = false;
  delete s;
}

}  // extern "C"
