// Batched Lanczos / multi-shift Galerkin kernels for gfx950.
//
// What is computed (Algorithm 1/2, steps 1-2): for every problem ("job") and
// every right-hand side column l, one real Lanczos process on G = A^T A
// started from V_in[:, l] builds v_0, v_1, ... with
//     G v_k = beta_{k+1} v_{k+1} + alpha_k v_k + beta_k v_{k-1}.
// Since G and V_in are real, the Krylov space of (z I - G) for every complex
// shift z equals that of G, so one basis serves all N/2 shifts.  For each
// shift the Galerkin solution y_k = V_k (z I - T_k)^{-1} e_1 ||V_in[:, l]|| is
// updated progressively through the LU factorisation of z I - T_k without
// pivoting (pivots eta_k have Im eta_k >= Im z > 0, so they never vanish):
//     eta_0 = z - alpha_0,  zeta_0 = ||V_in[:, l]||
//     lambda_k = e_k / eta_{k-1},  e_k = -beta_k
//     eta_k = (z - alpha_k) - lambda_k e_k,  zeta_k = -lambda_k zeta_{k-1}
//     p_k = (v_k - e_k p_{k-1}) / eta_k,  y_k = y_{k-1} + zeta_k p_k
// with residual norm beta_{k+1} |zeta_k / eta_k|.  These are the iterates of
// COCG on (z I - G) y = V_in[:, l] in exact arithmetic.  The vector updates of
// y and p are deferred and applied once per window of W steps, as a
// combination of the W stored basis vectors, so the per-shift state is read
// and written once per window instead of once per step.
//
// Stage order per Lanczos step (one launch each, all jobs at once):
//   K1  u = A v_k, per-tile partial sums of ||u_col||^2        (alpha_k)
//   R1  deterministic reduction of the partials -> alpha_k
//   K2  w = A^T u - alpha_k v_k - beta_k v_{k-1}, partial ||w_col||^2,
//       and v_k written into window slot (k mod W), column-major
//   S2  beta_{k+1}, the per-shift pivots / coefficients, convergence flags,
//       and the engine clock advance (last block)
// and at the end of each window:
//   WC  window coefficients per (shift, column)
//   WA  y += a p + sum_i E_i v_i,  p = c p + sum_i D_i v_i  for all shifts.
#include "csvd_impl.h"

namespace csvd {

constexpr int kE = 8;                   // elements per thread per tile
constexpr int kTE = kThreads * kE;      // elements per tile (2048)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm avoids overflow in |b|^2
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ __forceinline__ double cabs_(double2 a) { return hypot(a.x, a.y); }

// job index of global tile g: toff[j] <= g < toff[j+1]
__device__ __forceinline__ int find_job(const int *__restrict__ toff, int njob, int g) {
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (toff[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static int grid_cap(int total, int cap) { return total < 1 ? 1 : (total < cap ? total : cap); }

// ------------------------------------------------------------------- K1
// Thread slot layout inside a tile: slot = ((row * G) + g) * Lp + col, so the
// lanes of one (row, g) read one contiguous segment of x per nonzero, and
// the G lane groups of a row split its nonzeros (k = g, g+G, ...) before a
// fixed-order LDS reduction.  G = 1 for short rows, up to 256/Lp for long ones.
__global__ __launch_bounds__(kThreads) void k1_spmm_alpha(const JobDesc *__restrict__ jobs, int njob,
                                                          const int *__restrict__ toff, int total,
                                                          const int64_t *__restrict__ clock) {
  __shared__ double red[kThreads];
  __shared__ double gsum[kThreads];
  const int t = threadIdx.x;
  const int64_t ck = *clock;
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int j = find_job(toff, njob, g);
    const JobDesc &J = jobs[j];
    const int tile = g - toff[j];
    const int k = (int)(ck - J.start_clock);
    const int Lp = J.Lp, lg = J.lgLp, m = J.m;
    const int G = J.G1, lgG = J.lgG1, E = J.E1, rpt = J.rpt1;
    const int64_t nL = (int64_t)J.n * Lp;
    const GLB double *__restrict__ x = gp(J.wring) + (int64_t)(k % 3) * nL;
    const int col = t & (Lp - 1);
    const int gi = (t >> lg) & (G - 1);
    const double sc = gp(J.inv_cur)[col];
    const GLB int *__restrict__ rp = gp(J.rp);
    const GLB int *__restrict__ ci = gp(J.ci);
    const GLB double *__restrict__ va = gp(J.va);
    GLB double *__restrict__ uo = gp(J.u);
    // gather the E row segments of this thread first, then walk them in
    // lock step so E independent load chains are in flight
    int pb[kE], plen[kE];
    int maxlen = 0;
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      pb[q] = 0;
      plen[q] = 0;
      if (q < E) {
        const int64_t row = (int64_t)tile * rpt + ((q * kThreads + t) >> (lg + lgG));
        if (row < m) {
          const int b0 = rp[row] + gi, e0 = rp[row + 1];
          pb[q] = b0;
          plen[q] = e0 > b0 ? (e0 - b0 + G - 1) >> lgG : 0;
          maxlen = plen[q] > maxlen ? plen[q] : maxlen;
        }
      }
    }
    double acc[kE];
#pragma unroll
    for (int q = 0; q < kE; ++q) acc[q] = 0.0;
    for (int i = 0; i < maxlen; ++i) {
#pragma unroll
      for (int q = 0; q < kE; ++q) {
        if (i < plen[q]) {
          const int p = pb[q] + (i << lgG);
          acc[q] = fma(va[p], x[((int64_t)ci[p] << lg) + col], acc[q]);
        }
      }
    }
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      if (q < E) {
        const int64_t row = (int64_t)tile * rpt + ((q * kThreads + t) >> (lg + lgG));
        double a_ = acc[q];
        if (G > 1) {
          gsum[t] = a_;
          __syncthreads();
          if (gi == 0)
            for (int h = 1; h < G; ++h) a_ += gsum[t + (h << lg)];
          __syncthreads();
        }
        if (gi == 0 && row < m) {
          const double y = a_ * sc;
          uo[(row << lg) + col] = y;
          sq = fma(y, y, sq);
        }
      }
    }
    red[t] = sq;
    __syncthreads();
    if (t < Lp) {
      double s = 0.0;
      for (int i = t; i < kThreads; i += Lp) s += red[i];
      gp(J.part1)[(int64_t)tile * Lp + t] = s;
    }
    __syncthreads();
  }
}

hipError_t launch_k1_spmm_alpha(const BatchLaunch &b, hipStream_t st) {
  hipLaunchKernelGGL(k1_spmm_alpha, dim3(grid_cap(b.total1, 4096)), dim3(kThreads), 0, st, b.jobs, b.njob, b.toff1,
                     b.total1, b.clock);
  return hipGetLastError();
}

// deterministic block sum of part[tile*Lp + col], tile = 0..tiles-1
__device__ double block_sum_strided(const double *__restrict__ part_, int tiles, int Lp, int col, double *red) {
  const int t = threadIdx.x;
  const GLB double *__restrict__ part = gp(part_);
  double s = 0.0;
  for (int i = t; i < tiles; i += kThreads) s += part[(int64_t)i * Lp + col];
  red[t] = s;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------- R1
__global__ __launch_bounds__(kThreads) void r1_alpha(const JobDesc *__restrict__ jobs, int njob,
                                                     const int *__restrict__ toffc) {
  __shared__ double red[kThreads];
  const int g = blockIdx.x;
  const int j = find_job(toffc, njob, g);
  const JobDesc &J = jobs[j];
  const int col = g - toffc[j];
  const double s = block_sum_strided(J.part1, J.tiles1, J.Lp, col, red);
  if (threadIdx.x == 0) J.alpha[col] = s;
}

hipError_t launch_r1_alpha(const BatchLaunch &b, hipStream_t st) {
  hipLaunchKernelGGL(r1_alpha, dim3(b.totalc), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffc);
  return hipGetLastError();
}

// ------------------------------------------------------------------- K2
// Same slot layout as K1 over the rows of A^T; the lane group g = 0 of each
// (row, col) finishes the Lanczos update and stages v_k for the transposed
// window store (rpt contiguous rows per column).
template <bool MIXED>
__global__ __launch_bounds__(kThreads) void k2_spmm_lanczos(const JobDesc *__restrict__ jobs, int njob,
                                                            const int *__restrict__ toff, int total,
                                                            const int64_t *__restrict__ clock) {
  __shared__ double red[kThreads];
  __shared__ double gsum[kThreads];
  __shared__ double tr[kTE + kMaxLp];
  const int t = threadIdx.x;
  const int64_t ck = *clock;
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int j = find_job(toff, njob, g);
    const JobDesc &J = jobs[j];
    const int tile = g - toff[j];
    const int k = (int)(ck - J.start_clock);
    const int Lp = J.Lp, lg = J.lgLp, n = J.n;
    const int G = J.G2, lgG = J.lgG2, E = J.E2, rpt = J.rpt2;
    const int64_t nL = (int64_t)n * Lp;
    const GLB double *__restrict__ cur = gp(J.wring) + (int64_t)(k % 3) * nL;
    const GLB double *__restrict__ prv = gp(J.wring) + (int64_t)((k + 2) % 3) * nL;
    GLB double *__restrict__ nxt = gp(J.wring) + (int64_t)((k + 1) % 3) * nL;
    const int col = t & (Lp - 1);
    const int gi = (t >> lg) & (G - 1);
    const double a = gp(J.alpha)[col], c = gp(J.coup)[col], ic = gp(J.inv_cur)[col], ip = gp(J.inv_prev)[col];
    const GLB int *__restrict__ rp = gp(J.rpT);
    const GLB int *__restrict__ ci = gp(J.ciT);
    const GLB double *__restrict__ va = gp(J.vaT);
    const GLB double *__restrict__ u = gp(J.u);
    int pb[kE], plen[kE];
    int maxlen = 0;
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      pb[q] = 0;
      plen[q] = 0;
      if (q < E) {
        const int64_t row = (int64_t)tile * rpt + ((q * kThreads + t) >> (lg + lgG));
        if (row < n) {
          const int b0 = rp[row] + gi, e0 = rp[row + 1];
          pb[q] = b0;
          plen[q] = e0 > b0 ? (e0 - b0 + G - 1) >> lgG : 0;
          maxlen = plen[q] > maxlen ? plen[q] : maxlen;
        }
      }
    }
    double acc[kE];
#pragma unroll
    for (int q = 0; q < kE; ++q) acc[q] = 0.0;
    for (int i = 0; i < maxlen; ++i) {
#pragma unroll
      for (int q = 0; q < kE; ++q) {
        if (i < plen[q]) {
          const int p = pb[q] + (i << lgG);
          acc[q] = fma(va[p], u[((int64_t)ci[p] << lg) + col], acc[q]);
        }
      }
    }
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      if (q < E) {
        const int rloc = (q * kThreads + t) >> (lg + lgG);
        const int64_t row = (int64_t)tile * rpt + rloc;
        double a_ = acc[q];
        if (G > 1) {
          gsum[t] = a_;
          __syncthreads();
          if (gi == 0)
            for (int h = 1; h < G; ++h) a_ += gsum[t + (h << lg)];
          __syncthreads();
        }
        if (gi == 0) {
          double v = 0.0;
          if (row < n) {
            const int64_t e = (row << lg) + col;
            v = cur[e] * ic;
            const double w = a_ - a * v - c * (prv[e] * ip);
            nxt[e] = w;
            sq = fma(w, w, sq);
          }
          tr[col * (rpt + 1) + rloc] = v;
        }
      }
    }
    red[t] = sq;
    __syncthreads();
    if (t < Lp) {
      double s = 0.0;
      for (int i = t; i < kThreads; i += Lp) s += red[i];
      gp(J.part2)[(int64_t)tile * Lp + t] = s;
    }
    // window slot k mod W, column-major: rpt contiguous rows per column
    const int slotw = k % J.W;
    const int64_t row0 = (int64_t)tile * rpt;
    for (int li = t; li < rpt * Lp; li += kThreads) {
      const int c2 = li / rpt;
      const int r = li - c2 * rpt;
      const int64_t row = row0 + r;
      if (row < n) {
        const double v = tr[c2 * (rpt + 1) + r];
        const int64_t idx = ((int64_t)slotw * Lp + c2) * J.npad + row;
        if (MIXED) gp(J.winf)[idx] = (float)v;
        else gp(J.win)[idx] = v;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_k2_spmm_lanczos(const BatchLaunch &b, hipStream_t st) {
  if (b.mixed)
    hipLaunchKernelGGL(k2_spmm_lanczos<true>, dim3(grid_cap(b.total2, 4096)), dim3(kThreads), 0, st, b.jobs, b.njob,
                       b.toff2, b.total2, b.clock);
  else
    hipLaunchKernelGGL(k2_spmm_lanczos<false>, dim3(grid_cap(b.total2, 4096)), dim3(kThreads), 0, st, b.jobs,
                       b.njob, b.toff2, b.total2, b.clock);
  return hipGetLastError();
}

// ------------------------------------------------------------------- S2
__global__ __launch_bounds__(kThreads) void s2_step(const JobDesc *__restrict__ jobs, int njob,
                                                    const int *__restrict__ toffc, int totalc,
                                                    const int64_t *__restrict__ clock, int64_t *clock_mut,
                                                    int *ticket) {
  __shared__ double red[kThreads];
  __shared__ int live;
  const int g = blockIdx.x;
  const int t = threadIdx.x;
  const int j = find_job(toffc, njob, g);
  const JobDesc &J = jobs[j];
  const int l = g - toffc[j];
  const int Lp = J.Lp;
  const int64_t ck = *clock;
  const int k = (int)(ck - J.start_clock);
  const double b2 = block_sum_strided(J.part2, J.tiles2, Lp, l, red);
  const double beta = sqrt(b2);
  const double alpha = J.alpha[l];
  const double b0 = J.beta0[l];
  const double coup = J.coup[l];
  const int slot = k % J.W;
  if (t == 0) {
    live = 0;
    J.w_e[(int64_t)slot * Lp + l] = (k == 0) ? 0.0 : -coup;
  }
  __syncthreads();
  // breakdown: the Krylov space of this column is (numerically) invariant
  const bool brk = !(beta > 1e-15 * fmax(fabs(alpha) + coup, 1e-300));
  if (t < J.S) {
    const int s = t;
    const int64_t pr = (int64_t)s * Lp + l;
    const double2 z = J.shift[s];
    const double2 d = make_double2(z.x - alpha, z.y);
    int dn = J.done[pr];
    double2 et, ze;
    if (dn) {
      et = make_double2(1.0, 0.0);
      ze = make_double2(0.0, 0.0);
    } else if (k == 0) {
      et = d;
      ze = make_double2(b0, 0.0);
    } else {
      const double e = -coup;
      const double2 lam = cdiv(make_double2(e, 0.0), J.eta[pr]);
      et = make_double2(d.x - lam.x * e, d.y - lam.y * e);
      const double2 zp = J.zeta[pr];
      ze = make_double2(-(lam.x * zp.x - lam.y * zp.y), -(lam.x * zp.y + lam.y * zp.x));
    }
    const int64_t ws = (int64_t)slot * J.S * Lp + pr;
    J.w_eta[ws] = et;
    J.w_zeta[ws] = ze;
    if (!dn) {
      J.eta[pr] = et;
      J.zeta[pr] = ze;
      const double r = (b0 > 0.0) ? beta * cabs_(ze) / (cabs_(et) * b0) : 0.0;
      J.res[pr] = r;
      if (r <= J.tol || brk || b0 == 0.0) {
        J.done[pr] = 1;
        J.conv_iter[pr] = k;
        dn = 1;
      }
    }
    if (!dn) atomicOr(&live, 1);
  }
  __syncthreads();
  if (t == 0) {
    const double icur = J.inv_cur[l];
    J.inv_prev[l] = icur;
    if (live && !brk) {
      J.inv_cur[l] = 1.0 / beta;
      J.coup[l] = beta;
    } else {
      J.inv_cur[l] = 0.0;
      J.coup[l] = 0.0;
    }
    if (l == 0 && k < kHist) {
      J.nrm_hist[2 * k] = alpha;
      J.nrm_hist[2 * k + 1] = beta;
    }
    // advance the engine clock once every block of this launch is done
    __threadfence();
    const int tk = atomicAdd(ticket, 1);
    if (tk == totalc - 1) {
      *clock_mut = ck + 1;
      *ticket = 0;
      __threadfence();
    }
  }
}

hipError_t launch_s2_step(const BatchLaunch &b, hipStream_t st) {
  hipLaunchKernelGGL(s2_step, dim3(b.totalc), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffc, b.totalc, b.clock,
                     b.clock_mut, b.ticket);
  return hipGetLastError();
}

// ------------------------------------------------------------------- WC
// One thread per (job, shift, real column).  The window holds steps
// k0 .. k0+wlen-1 in slots 0 .. wlen-1 (windows start at multiples of W).
__global__ void wc_coef(const JobDesc *__restrict__ jobs, int njob, const int *__restrict__ toffp, int totalp,
                        const int64_t *__restrict__ clock, int wlen, int parity) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= totalp) return;
  const int j = find_job(toffp, njob, g);
  const JobDesc &J = jobs[j];
  const int idx = g - toffp[j];          // s * L + l over real columns
  const int s = idx / J.L, l = idx - s * J.L;
  const int Lp = J.Lp, S = J.S, W = J.W;
  const int k_end = (int)(*clock - J.start_clock) - 1;  // last completed step
  const int k0 = k_end - wlen + 1;
  const int64_t pr = (int64_t)s * Lp + l;
  const int64_t ci = (int64_t)l * S + s;
  const int dn = J.done[pr];
  const int skip = dn && J.conv_iter[pr] < k0;
  J.skip_pair[pr] = skip;
  if (!dn) atomicAdd(&J.active[parity], 1);
  if (skip) {
    J.cA[ci] = make_double2(0.0, 0.0);
    J.cC[ci] = make_double2(0.0, 0.0);
    return;
  }
  const int64_t stride = (int64_t)S * Lp;
  // backward pass: F_q = zeta_q + g_{q+1} F_{q+1},  E_q = F_q / eta_q
  double2 F = make_double2(0.0, 0.0);
  double2 gnext = make_double2(0.0, 0.0);
  for (int q = wlen - 1; q >= 0; --q) {
    const double2 et = J.w_eta[q * stride + pr];
    const double2 ze = J.w_zeta[q * stride + pr];
    const double2 gF = cmul(gnext, F);
    F = make_double2(ze.x + gF.x, ze.y + gF.y);
    J.cE[ci * W + q] = cdiv(F, et);
    const double e = J.w_e[(int64_t)q * Lp + l];
    gnext = cdiv(make_double2(-e, 0.0), et);  // g_q = -e_q / eta_q
  }
  J.cA[ci] = cmul(gnext, F);  // a = g_{k0} F_{k0}
  // D_q = (1/eta_q) prod_{r>q} g_r ;  c = prod_{r>=k0} g_r
  double2 prod = make_double2(1.0, 0.0);
  for (int q = wlen - 1; q >= 0; --q) {
    const double2 et = J.w_eta[q * stride + pr];
    J.cD[ci * W + q] = cdiv(prod, et);
    const double e = J.w_e[(int64_t)q * Lp + l];
    prod = cmul(prod, cdiv(make_double2(-e, 0.0), et));
  }
  J.cC[ci] = prod;
}

hipError_t launch_window_coef(const BatchLaunch &b, int wlen, int parity, hipStream_t st) {
  hipLaunchKernelGGL(wc_coef, dim3((b.totalp + 255) / 256), dim3(256), 0, st, b.jobs, b.njob, b.toffp, b.totalp,
                     b.clock, wlen, parity);
  return hipGetLastError();
}

// ------------------------------------------------------------------- WA
// Block = (job, real column l, 256-row tile, shift group); thread = one row.
// The window basis values of the row stay in registers; the coefficients of
// the block's shifts (uniform across the block) are staged once in LDS and
// read as broadcasts.
constexpr int kWaLds = 1024;  // complex coefficient pairs staged per block

template <int WMAX, bool MIXED>
__global__ __launch_bounds__(kThreads) void wa_apply(const JobDesc *__restrict__ jobs, int njob,
                                                     const int *__restrict__ toffw, int wlen) {
  __shared__ double2 shE[kWaLds], shD[kWaLds];
  __shared__ double2 shA[kMaxShifts], shC[kMaxShifts];
  __shared__ int shSkip[kMaxShifts];
  const int g = blockIdx.x;
  const int j = find_job(toffw, njob, g);
  const JobDesc &J = jobs[j];
  const int rtiles = (J.n + kThreads - 1) / kThreads;
  const int idx0 = g - toffw[j];
  const int sgi = idx0 % J.nsg;
  const int idx = idx0 / J.nsg;
  const int l = idx / rtiles;
  const int rt = idx - l * rtiles;
  const int s_lo = sgi * J.Sg;
  const int s_hi = (s_lo + J.Sg < J.S) ? s_lo + J.Sg : J.S;
  const int ns = s_hi - s_lo;
  const int Lp = J.Lp, S = J.S, W = J.W;
  // stage coefficients: shifts s_lo..s_hi-1 of column l (index (l*S+s)*W+q)
  {
    const GLB double2 *__restrict__ gE = gp(J.cE) + ((int64_t)l * S + s_lo) * W;
    const GLB double2 *__restrict__ gD = gp(J.cD) + ((int64_t)l * S + s_lo) * W;
    for (int e = threadIdx.x; e < ns * W; e += kThreads) {
      shE[e] = gE[e];
      shD[e] = gD[e];
    }
    if (threadIdx.x < ns) {
      const int s = s_lo + threadIdx.x;
      shA[threadIdx.x] = gp(J.cA)[(int64_t)l * S + s];
      shC[threadIdx.x] = gp(J.cC)[(int64_t)l * S + s];
      shSkip[threadIdx.x] = gp(J.skip_pair)[(int64_t)s * Lp + l];
    }
  }
  __syncthreads();
  const int64_t row = (int64_t)rt * kThreads + threadIdx.x;
  if (row >= J.n) return;
  const int64_t npad = J.npad;
  double v[WMAX];
#pragma unroll
  for (int q = 0; q < WMAX; ++q) {
    if (q < wlen) {
      const int64_t wi = ((int64_t)q * Lp + l) * npad + row;
      v[q] = MIXED ? (double)gp(J.winf)[wi] : gp(J.win)[wi];
    }
  }
  for (int si = 0; si < ns; ++si) {
    if (shSkip[si]) continue;
    const int s = s_lo + si;
    const int64_t off = ((int64_t)s * Lp + l) * npad + row;
    double2 x, p;
    if (MIXED) {
      const float2 xf = gp(J.Xf)[off], pf = gp(J.Pf)[off];
      x = make_double2(xf.x, xf.y);
      p = make_double2(pf.x, pf.y);
    } else {
      x = gp(J.X)[off];
      p = gp(J.P)[off];
    }
    const double2 a = shA[si], c = shC[si];
    double xr = x.x + a.x * p.x - a.y * p.y;
    double xi = x.y + a.x * p.y + a.y * p.x;
    double pr_ = c.x * p.x - c.y * p.y;
    double pi_ = c.x * p.y + c.y * p.x;
    const double2 *E = shE + si * W;
    const double2 *D = shD + si * W;
#pragma unroll
    for (int q = 0; q < WMAX; ++q) {
      if (q < wlen) {
        const double2 eq = E[q], dq = D[q];
        xr = fma(eq.x, v[q], xr);
        xi = fma(eq.y, v[q], xi);
        pr_ = fma(dq.x, v[q], pr_);
        pi_ = fma(dq.y, v[q], pi_);
      }
    }
    if (MIXED) {
      gp(J.Xf)[off] = make_float2((float)xr, (float)xi);
      gp(J.Pf)[off] = make_float2((float)pr_, (float)pi_);
    } else {
      gp(J.X)[off] = make_double2(xr, xi);
      gp(J.P)[off] = make_double2(pr_, pi_);
    }
  }
}

hipError_t launch_window_apply(const BatchLaunch &b, int wlen, hipStream_t st) {
  dim3 g(b.totalw), blk(kThreads);
  if (b.mixed) {
    if (b.Wmax <= 16) hipLaunchKernelGGL((wa_apply<16, true>), g, blk, 0, st, b.jobs, b.njob, b.toffw, wlen);
    else if (b.Wmax <= 32) hipLaunchKernelGGL((wa_apply<32, true>), g, blk, 0, st, b.jobs, b.njob, b.toffw, wlen);
    else hipLaunchKernelGGL((wa_apply<64, true>), g, blk, 0, st, b.jobs, b.njob, b.toffw, wlen);
  } else {
    if (b.Wmax <= 16) hipLaunchKernelGGL((wa_apply<16, false>), g, blk, 0, st, b.jobs, b.njob, b.toffw, wlen);
    else if (b.Wmax <= 32) hipLaunchKernelGGL((wa_apply<32, false>), g, blk, 0, st, b.jobs, b.njob, b.toffw, wlen);
    else hipLaunchKernelGGL((wa_apply<64, false>), g, blk, 0, st, b.jobs, b.njob, b.toffw, wlen);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ job set-up
// per-column norms of ring[0] and the initial per-column / per-pair state
__global__ __launch_bounds__(kThreads) void k_job_init_cols(JobDesc J) {
  __shared__ double red[kThreads];
  const int l = blockIdx.x;
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t r = t; r < J.n; r += kThreads) {
    const double v = J.wring[r * J.Lp + l];
    s = fma(v, v, s);
  }
  red[t] = s;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0) {
    const double b0 = sqrt(red[0]);
    J.beta0[l] = b0;
    J.inv_cur[l] = b0 > 0.0 ? 1.0 / b0 : 0.0;
    J.inv_prev[l] = 0.0;
    J.coup[l] = 0.0;
    J.alpha[l] = 0.0;
  }
  for (int s2 = t; s2 < J.S; s2 += kThreads) {
    const int64_t pr = (int64_t)s2 * J.Lp + l;
    J.eta[pr] = make_double2(1.0, 0.0);
    J.zeta[pr] = make_double2(0.0, 0.0);
    J.done[pr] = 0;
    J.conv_iter[pr] = -1;
    J.res[pr] = 1.0;
    J.skip_pair[pr] = 0;
  }
}

hipError_t launch_job_init(const JobDesc &hj, const double *Vcol, int64_t ldv, hipStream_t st) {
  const int64_t nL = (int64_t)hj.n * hj.Lp;
  hipError_t e = hipMemsetAsync(hj.wring, 0, sizeof(double) * 3 * nL, st);
  if (e != hipSuccess) return e;
  const int64_t xs = (int64_t)hj.S * hj.Lp * hj.npad;
  if (hj.X) {
    e = hipMemsetAsync(hj.X, 0, sizeof(double2) * xs, st);
    if (e == hipSuccess) e = hipMemsetAsync(hj.P, 0, sizeof(double2) * xs, st);
  } else {
    e = hipMemsetAsync(hj.Xf, 0, sizeof(float2) * xs, st);
    if (e == hipSuccess) e = hipMemsetAsync(hj.Pf, 0, sizeof(float2) * xs, st);
  }
  if (e != hipSuccess) return e;
  e = launch_col_to_row(hj.n, hj.L, Vcol, ldv, hj.wring, hj.Lp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_job_init_cols, dim3(hj.Lp), dim3(kThreads), 0, st, hj);
  return hipGetLastError();
}

// ---------------------------------------------------------------- moments
// S_k[:, l] = 2 sum_s Re(c_{s,k} Y_s[:, l]),  out column (k*L + l), ld npad.
template <bool MIXED>
__global__ __launch_bounds__(kThreads) void k_moments(JobDesc J, const double2 *__restrict__ coef, int K,
                                                      double *__restrict__ out) {
  const int l = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (row >= J.npad) return;
  double acc[16];
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int kk = (K - k0 < 16) ? K - k0 : 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    if (row < J.n) {
      for (int s = 0; s < J.S; ++s) {
        const int64_t off = ((int64_t)s * J.Lp + l) * J.npad + row;
        double2 y;
        if (MIXED) {
          float2 f = J.Xf[off];
          y = make_double2(f.x, f.y);
        } else {
          y = J.X[off];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q < kk) {
            const double2 c = coef[s * K + k0 + q];
            acc[q] += 2.0 * (c.x * y.x - c.y * y.y);
          }
      }
    }
    for (int q = 0; q < kk; ++q) out[((int64_t)(k0 + q) * J.L + l) * J.npad + row] = acc[q];
  }
}

hipError_t launch_moments(const JobDesc &hj, const double2 *coef, int K, double *out, hipStream_t st) {
  dim3 g((unsigned)((hj.npad + kThreads - 1) / kThreads), hj.L);
  if (hj.X) hipLaunchKernelGGL(k_moments<false>, g, dim3(kThreads), 0, st, hj, coef, K, out);
  else hipLaunchKernelGGL(k_moments<true>, g, dim3(kThreads), 0, st, hj, coef, K, out);
  return hipGetLastError();
}

__global__ void k_get_solution(JobDesc J, int s, double *__restrict__ re, double *__restrict__ im) {
  const int l = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (row >= J.n) return;
  const int64_t off = ((int64_t)s * J.Lp + l) * J.npad + row;
  double2 y;
  if (J.X) {
    y = J.X[off];
  } else {
    float2 f = J.Xf[off];
    y = make_double2(f.x, f.y);
  }
  re[(int64_t)l * J.n + row] = y.x;
  im[(int64_t)l * J.n + row] = y.y;
}

hipError_t launch_get_solution(const JobDesc &hj, int j, double *re, double *im, hipStream_t st) {
  dim3 g((unsigned)((hj.n + kThreads - 1) / kThreads), hj.L);
  hipLaunchKernelGGL(k_get_solution, g, dim3(kThreads), 0, st, hj, j, re, im);
  return hipGetLastError();
}

__global__ void k_zero(double *p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_zero(double *p, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int64_t g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

}  // namespace csvd
