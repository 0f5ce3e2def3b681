// Block Lanczos kernels for gfx950 (Algorithm 1/2, steps 1-2): the sparse
// products, the per-shift recurrences and the moment coefficients.  The
// orthogonalisation of each new block lives in k_bstep.hip.
//
// One real block Lanczos process on G = A^T A of width Lp (the L right-hand
// sides plus seeded padding columns) spans the block Krylov space of every
// shifted system (z I - G) Y = V, since G and V are real.  Step k:
//   W = A^T (A Q_k) - Q_{k-1} B_k^T,  A_k = sym(Q_k^T W),
//   W - Q_k A_k (after reorthogonalisation) = Q_{k+1} B_{k+1}
// and for every shift z the block LU of (z I - T_k) without pivoting
//   H_k = z I - A_k - B_k H_{k-1}^{-1} B_k^T,  Z_{k+1} = B_{k+1} H_k^{-1} Z_k
// (Im H_k is positive definite, so every H_k is invertible) gives the
// residual norms ||Z_{k+1}(:, l)|| of the block Galerkin solutions.  After
// convergence the block tridiagonal systems are solved backwards,
//   Y_{K-1} = H_{K-1}^{-1} Z_{K-1},  Y_k = H_k^{-1} (Z_k + B_{k+1}^T Y_{k+1}),
// the moment coefficients F_k = sum_s 2 Re(c_sk Y_{s,k}) are formed, and a
// second pass regenerates Q_k bit for bit and accumulates S += Q_k F_k.
#include "csvd_impl.h"

namespace csvd {

__device__ __forceinline__ int bfind(const int *__restrict__ toff, int njob, int g) {
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (toff[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static int bgrid(int total, int cap) { return total < 1 ? 1 : (total < cap ? total : cap); }

constexpr int kEB = 8;  // max thread slots per tile in the sparse products

__device__ __forceinline__ double2 cmulb(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdivb(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}

// ------------------------------------------------------ sparse products
// y = M x for the rows of one tile; slot layout ((row * G) + g) * Lp + col as
// in the single-vector kernels (G lane groups split each row's nonzeros).
__device__ __forceinline__ void tile_spmm(const GLB int *__restrict__ rp, const GLB int *__restrict__ ci,
                                          const GLB double *__restrict__ va, const GLB double *__restrict__ x,
                                          GLB double *__restrict__ y, int64_t nrows, int tile, int rpt, int lg,
                                          int G, int lgG, int E, double *gsum) {
  const int t = threadIdx.x;
  const int Lp = 1 << lg;
  const int col = t & (Lp - 1);
  const int gi = (t >> lg) & (G - 1);
  for (int q = 0; q < E; ++q) {
    const int rloc = (q * kThreads + t) >> (lg + lgG);
    const int64_t row = (int64_t)tile * rpt + rloc;
    double acc = 0.0;
    if (row < nrows) {
      const int en = rp[row + 1];
#pragma unroll 4
      for (int p = rp[row] + gi; p < en; p += G) acc = fma(va[p], x[((int64_t)ci[p] << lg) + col], acc);
    }
    if (G > 1) {
      gsum[t] = acc;
      __syncthreads();
      if (gi == 0)
        for (int h = 1; h < G; ++h) acc += gsum[t + (h << lg)];
      __syncthreads();
    }
    if (gi == 0 && row < nrows) y[(row << lg) + col] = acc;
  }
}

__global__ __launch_bounds__(kThreads) void b_spmm_a(const BJobDesc *__restrict__ jobs, int njob,
                                                     const int *__restrict__ toff, int total,
                                                     const int64_t *__restrict__ clock) {
  __shared__ double gsum[kThreads];
  const int64_t ck = *clock;
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int j = bfind(toff, njob, g);
    const BJobDesc &J = jobs[j];
    const int k = (int)(ck - J.start_clock);
    if (k >= J.Kstop) continue;
    const int64_t nL = (int64_t)J.n * J.Lp;
    tile_spmm(gp(J.rp), gp(J.ci), gp(J.va), gp(J.Q) + (int64_t)(k % 3) * nL, gp(J.U), J.m, g - toff[j], J.rpt1,
              J.lgLp, J.G1, J.lgG1, J.E1, gsum);
  }
}

__global__ __launch_bounds__(kThreads) void b_spmm_at(const BJobDesc *__restrict__ jobs, int njob,
                                                      const int *__restrict__ toff, int total,
                                                      const int64_t *__restrict__ clock) {
  __shared__ double gsum[kThreads];
  const int64_t ck = *clock;
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int j = bfind(toff, njob, g);
    const BJobDesc &J = jobs[j];
    if ((int)(ck - J.start_clock) >= J.Kstop) continue;
    tile_spmm(gp(J.rpT), gp(J.ciT), gp(J.vaT), gp(J.U), gp(J.W), J.n, g - toff[j], J.rpt2, J.lgLp, J.G2, J.lgG2,
              J.E2, gsum);
  }
}

hipError_t launch_b_spmm_a(const BBatch &b, hipStream_t st) {
  hipLaunchKernelGGL(b_spmm_a, dim3(bgrid(b.total1, 4096)), dim3(kThreads), 0, st, b.jobs, b.njob, b.toff1, b.total1,
                     b.clock);
  return hipGetLastError();
}

hipError_t launch_b_spmm_at(const BBatch &b, hipStream_t st) {
  hipLaunchKernelGGL(b_spmm_at, dim3(bgrid(b.total2, 4096)), dim3(kThreads), 0, st, b.jobs, b.njob, b.toff2, b.total2,
                     b.clock);
  return hipGetLastError();
}

// ------------------------------------------------------ per-shift block LU
// One block per (job, shift).  H in LDS (complex, stride Lp+1), inverted in
// place by Gauss-Jordan elimination without pivoting.
__global__ __launch_bounds__(kThreads) void b_shift(const BJobDesc *__restrict__ jobs, int njob,
                                                    const int *__restrict__ toffs, const int64_t *__restrict__ clock,
                                                    int init) {
  __shared__ double2 H[kBlockMaxLp * (kBlockMaxLp + 1)];
  __shared__ double2 colk[kBlockMaxLp];
  const int g = blockIdx.x;
  const int j = bfind(toffs, njob, g);
  const BJobDesc &J = jobs[j];
  const int s = g - toffs[j];
  const int Lp = J.Lp, L2 = Lp * Lp, L = J.L;
  const int ld = Lp + 1;
  const int t = threadIdx.x;
  const int k = (int)(*clock - J.start_clock);
  if (k >= J.Kstop) return;
  const int64_t hbase = (int64_t)s * (J.Kcap + 1) * L2;
  GLB double2 *__restrict__ Hinv = gp(J.Hinv) + hbase;
  GLB double2 *__restrict__ Zh = gp(J.Zh) + hbase;
  GLB double2 *__restrict__ T1 = gp(J.ctmp) + (int64_t)s * 2 * L2;
  GLB double2 *__restrict__ T2 = T1 + L2;
  if (init) {
    for (int e = t; e < L2; e += kThreads) Zh[e] = make_double2(gp(J.Bh)[e], 0.0);  // Z_0 = R_0
    return;
  }
  const double2 z = gp(J.shift)[s];
  const GLB double *__restrict__ Ak = gp(J.Ah) + (int64_t)k * L2;
  const GLB double *__restrict__ Bk = gp(J.Bh) + (int64_t)k * L2;
  const GLB double *__restrict__ Bk1 = gp(J.Bh) + (int64_t)(k + 1) * L2;
  if (k > 0) {
    // T1 = Hinv_{k-1} B_k^T
    const GLB double2 *__restrict__ Hp = Hinv + (int64_t)(k - 1) * L2;
    for (int e = t; e < L2; e += kThreads) {
      const int i = e / Lp, jj = e - i * Lp;
      double2 acc = make_double2(0.0, 0.0);
      for (int c = 0; c < Lp; ++c) {
        const double bv = Bk[jj * Lp + c];
        const double2 h = Hp[i * Lp + c];
        acc.x = fma(h.x, bv, acc.x);
        acc.y = fma(h.y, bv, acc.y);
      }
      T1[e] = acc;
    }
    __syncthreads();
  }
  for (int e = t; e < L2; e += kThreads) {
    const int i = e / Lp, jj = e - i * Lp;
    double2 h = make_double2((i == jj ? z.x : 0.0) - Ak[e], (i == jj) ? z.y : 0.0);
    if (k > 0) {
      for (int c = 0; c < Lp; ++c) {
        const double bv = Bk[i * Lp + c];
        const double2 tv = T1[c * Lp + jj];
        h.x = fma(-bv, tv.x, h.x);
        h.y = fma(-bv, tv.y, h.y);
      }
    }
    H[i * ld + jj] = h;
  }
  __syncthreads();
  // Gauss-Jordan inverse in place
  for (int c = 0; c < Lp; ++c) {
    const double2 piv = H[c * ld + c];
    const double2 inv = cdivb(make_double2(1.0, 0.0), piv);
    if (t < Lp) colk[t] = H[t * ld + c];
    __syncthreads();
    if (t < Lp) H[c * ld + t] = (t == c) ? inv : cmulb(H[c * ld + t], inv);
    __syncthreads();
    for (int e = t; e < L2; e += kThreads) {
      const int i = e / Lp, jj = e - i * Lp;
      if (i == c) continue;
      const double2 f = colk[i];
      if (jj == c) {
        const double2 v = cmulb(f, inv);
        H[i * ld + jj] = make_double2(-v.x, -v.y);
      } else {
        const double2 r = cmulb(f, H[c * ld + jj]);
        H[i * ld + jj] = make_double2(H[i * ld + jj].x - r.x, H[i * ld + jj].y - r.y);
      }
    }
    __syncthreads();
  }
  GLB double2 *__restrict__ Hk = Hinv + (int64_t)k * L2;
  for (int e = t; e < L2; e += kThreads) Hk[e] = H[(e / Lp) * ld + (e % Lp)];
  // T2 = Hinv_k Z_k (columns < L), Z_{k+1} = B_{k+1} T2
  const GLB double2 *__restrict__ Zk = Zh + (int64_t)k * L2;
  for (int e = t; e < Lp * L; e += kThreads) {
    const int i = e / L, jj = e - i * L;
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < Lp; ++c) {
      const double2 r = cmulb(H[i * ld + c], Zk[c * Lp + jj]);
      acc.x += r.x;
      acc.y += r.y;
    }
    T2[i * Lp + jj] = acc;
  }
  __syncthreads();
  GLB double2 *__restrict__ Zn = Zh + (int64_t)(k + 1) * L2;
  for (int e = t; e < Lp * L; e += kThreads) {
    const int i = e / L, jj = e - i * L;
    double2 acc = make_double2(0.0, 0.0);
    for (int c = i; c < Lp; ++c) {  // B_{k+1} is upper triangular
      const double bv = Bk1[i * Lp + c];
      const double2 tv = T2[c * Lp + jj];
      acc.x = fma(bv, tv.x, acc.x);
      acc.y = fma(bv, tv.y, acc.y);
    }
    Zn[i * Lp + jj] = acc;
  }
  __syncthreads();
  if (t < L) {
    double nr = 0.0;
    for (int i = 0; i < Lp; ++i) {
      const double2 v = Zn[i * Lp + t];
      nr += v.x * v.x + v.y * v.y;
    }
    const double b0 = gp(J.beta0)[t];
    const double r = b0 > 0.0 ? sqrt(nr) / b0 : 0.0;
    gp(J.res)[(int64_t)s * Lp + t] = r;
    if (r > J.tol) atomicAdd(gp(J.active) + (k & 1), 1);
  }
  if (s == 0 && t == 0) gp(J.active)[(k + 1) & 1] = 0;
}

hipError_t launch_b_shift(const BBatch &b, int init, hipStream_t st) {
  hipLaunchKernelGGL(b_shift, dim3(b.totals), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffs, b.clock, init);
  return hipGetLastError();
}

// ------------------------------------------------------ backward solution
// Y_k = H_k^{-1} (Z_k + B_{k+1}^T Y_{k+1}), k = K-1 .. 0; Y_k overwrites Z_k
// (columns < L).  The columns are independent: one workgroup per (shift,
// group of 16 columns), H_k^{-1} staged in LDS for each step.
constexpr int kBsCols = 16;

__global__ __launch_bounds__(kThreads) void b_backsolve(BJobDesc J, int K) {
  __shared__ double2 Hs[kBlockMaxLp * kBlockMaxLp];
  __shared__ double2 Ts[kBlockMaxLp * kBsCols], Yn[kBlockMaxLp * kBsCols];
  const int ng = (J.L + kBsCols - 1) / kBsCols;
  const int s = blockIdx.x / ng, cg = blockIdx.x - s * ng;
  const int Lp = J.Lp, L2 = Lp * Lp, L = J.L;
  const int t = threadIdx.x;
  const int jj = t & (kBsCols - 1), col = cg * kBsCols + jj;
  const bool live = col < L;
  const int64_t hbase = (int64_t)s * (J.Kcap + 1) * L2;
  const GLB double2 *__restrict__ Hinv = gp(J.Hinv) + hbase;
  GLB double2 *__restrict__ Zh = gp(J.Zh) + hbase;
  for (int k = K - 1; k >= 0; --k) {
    const GLB double2 *__restrict__ Hk = Hinv + (int64_t)k * L2;
    for (int e = t; e < L2; e += kThreads) Hs[e] = Hk[e];
    // T = Z_k + B_{k+1}^T Y_{k+1} for this thread's rows
    const GLB double *__restrict__ Bk1 = gp(J.Bh) + (int64_t)(k + 1) * L2;
    for (int i = t >> 4; i < Lp; i += kThreads / kBsCols) {
      double2 acc = live ? Zh[(int64_t)k * L2 + i * Lp + col] : make_double2(0.0, 0.0);
      if (k < K - 1) {
        for (int c = 0; c <= i; ++c) {  // (B^T)[i][c] = B[c][i], B upper
          const double bv = Bk1[c * Lp + i];
          const double2 y = Yn[c * kBsCols + jj];
          acc.x = fma(bv, y.x, acc.x);
          acc.y = fma(bv, y.y, acc.y);
        }
      }
      Ts[i * kBsCols + jj] = acc;
    }
    __syncthreads();
    for (int i = t >> 4; i < Lp; i += kThreads / kBsCols) {
      double2 acc = make_double2(0.0, 0.0);
      for (int c = 0; c < Lp; ++c) {
        const double2 r = cmulb(Hs[i * Lp + c], Ts[c * kBsCols + jj]);
        acc.x += r.x;
        acc.y += r.y;
      }
      Yn[i * kBsCols + jj] = acc;
      if (live) Zh[(int64_t)k * L2 + i * Lp + col] = acc;
    }
    __syncthreads();
  }
}

hipError_t launch_b_backsolve(const BJobDesc &hj, int K, hipStream_t st) {
  const int ng = (hj.L + kBsCols - 1) / kBsCols;
  hipLaunchKernelGGL(b_backsolve, dim3(hj.S * ng), dim3(kThreads), 0, st, hj, K);
  return hipGetLastError();
}

// F_k(c, kk*L + l) = sum_s 2 Re(c_{s,kk} Y_{s,k}(c, l)), stored column-major
// per step: F[k][(kk*L + l) * Lp + c].
__global__ void b_fcoef(BJobDesc J, int K) {
  const int Lp = J.Lp, L2 = Lp * Lp, L = J.L, KL = J.Kmom * L;
  const int64_t total = (int64_t)K * KL * Lp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % Lp);
    const int64_t r = e / Lp;
    const int oc = (int)(r % KL);
    const int k = (int)(r / KL);
    const int kk = oc / L, l = oc - kk * L;
    double acc = 0.0;
    for (int s = 0; s < J.S; ++s) {
      const double2 y = gp(J.Zh)[((int64_t)s * (J.Kcap + 1) + k) * L2 + c * Lp + l];
      const double2 cm = gp(J.cmom)[s * J.cstride + kk];
      acc += 2.0 * (cm.x * y.x - cm.y * y.y);
    }
    gp(J.F)[e] = acc;
  }
}

hipError_t launch_b_fcoef(const BJobDesc &hj, int K, hipStream_t st) {
  const int64_t total = (int64_t)K * hj.Kmom * hj.L * hj.Lp;
  int64_t g = (total + 255) / 256;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(b_fcoef, dim3((unsigned)g), dim3(256), 0, st, hj, K);
  return hipGetLastError();
}

__global__ void b_tick(int64_t *clock) { *clock += 1; }

hipError_t launch_b_tick(int64_t *clock, hipStream_t st) {
  hipLaunchKernelGGL(b_tick, dim3(1), dim3(1), 0, st, clock);
  return hipGetLastError();
}

}  // namespace csvd
