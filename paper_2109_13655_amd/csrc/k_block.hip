// Block Lanczos kernels for gfx950 (Algorithm 1/2, steps 1-2).
//
// One real block Lanczos process on G = A^T A of width Lp (the L right-hand
// sides plus seeded padding columns) spans the block Krylov space of every
// shifted system (z I - G) Y = V, since G and V are real.  Step k:
//   W   = A^T (A Q_k) - Q_{k-1} B_k^T
//   A_k = sym(Q_k^T W),  C_k = Q_k^T (W - Q_k A_k)       (CGS2 against Q_k)
//   W2  = W - Q_k (A_k + C_k)
//   W2  = Q_{k+1} B_{k+1}                                 (CholeskyQR2)
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

// ------------------------------------------------------ buffer selection
__device__ __forceinline__ GLB double *bbuf(const BJobDesc &J, int code, int k) {
  const int64_t nL = (int64_t)J.n * J.Lp;
  switch (code) {
    case BQ_PREV: return gp(J.Q) + (int64_t)((k + 2) % 3) * nL;
    case BQ_CUR: return gp(J.Q) + (int64_t)(k % 3) * nL;
    case BQ_NEXT: return gp(J.Q) + (int64_t)((k + 1) % 3) * nL;
    case BW: return gp(J.W);
    case BW2: return gp(J.W2);
    case BVPAD: return gp(J.Vpad);
    default: return nullptr;
  }
}

// S(c, col) staged row-major in LDS (stride Lp)
__device__ void stage_small(const BJobDesc &J, int code, int k, double *Ssh) {
  const int Lp = J.Lp, L2 = Lp * Lp;
  const int64_t hk = (int64_t)k * L2;
  for (int e = threadIdx.x; e < L2; e += kThreads) {
    const int c = e / Lp, col = e - c * Lp;
    double v;
    switch (code) {
      case BM_BK_T: v = gp(J.Bh)[hk + (int64_t)col * Lp + c]; break;
      case BM_AK: v = gp(J.Ah)[hk + e]; break;
      case BM_AK_CK: v = gp(J.Ah)[hk + e] + gp(J.Ch)[hk + e]; break;
      case BM_R1INV: v = gp(J.R1inv)[e]; break;
      case BM_MK: v = gp(J.Mh)[hk + e]; break;
      default: v = gp(J.Mh)[(int64_t)J.Kcap * L2 + e]; break;  // BM_MINIT
    }
    Ssh[e] = v;
  }
}

// ------------------------------------------------------------ row products
// Y = Z - X S (or Y = X S), rows of one chunk; thread = (row of the group, col).
__global__ __launch_bounds__(kThreads) void b_rowmm(const BJobDesc *__restrict__ jobs, int njob,
                                                    const int *__restrict__ toff, const int64_t *__restrict__ clock,
                                                    int Xc, int Zc, int Yc, int smat) {
  __shared__ double Ssh[kBlockMaxLp * kBlockMaxLp];
  __shared__ double Xs[kThreads];
  const int g = blockIdx.x;
  const int j = bfind(toff, njob, g);
  const BJobDesc &J = jobs[j];
  const int k = (int)(*clock - J.start_clock);
  if (k >= J.Kstop) return;
  const int chunk = g - toff[j];
  const int Lp = J.Lp, lg = J.lgLp;
  stage_small(J, smat, k, Ssh);
  // Z may alias Y (in-place update): each thread reads Z[e] before writing Y[e]
  const GLB double *__restrict__ X = bbuf(J, Xc, k);
  const GLB double *Z = bbuf(J, Zc, k);
  GLB double *Y = bbuf(J, Yc, k);
  const int t = threadIdx.x;
  const int col = t & (Lp - 1);
  const int rl = t >> lg;              // row inside the group
  const int rpg = kThreads >> lg;      // rows per group
  const int64_t r0 = (int64_t)chunk * kChunk;
  int64_t r1 = r0 + kChunk;
  if (r1 > J.n) r1 = J.n;
  __syncthreads();
  for (int64_t rb = r0; rb < r1; rb += rpg) {
    const int64_t row = rb + rl;
    Xs[t] = (row < r1) ? X[(row << lg) + col] : 0.0;
    __syncthreads();
    if (row < r1) {
      double acc = 0.0;
      const double *xr = Xs + (rl << lg);
      for (int c = 0; c < Lp; ++c) acc = fma(xr[c], Ssh[(c << lg) + col], acc);
      const int64_t e = (row << lg) + col;
      Y[e] = (Z ? Z[e] : 0.0) - (Z ? acc : -acc);
    }
    __syncthreads();
  }
}

hipError_t launch_b_rowmm(const BBatch &b, int X, int Z, int Y, int smat, hipStream_t st) {
  hipLaunchKernelGGL(b_rowmm, dim3(b.totalr), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffr, b.clock, X, Z, Y, smat);
  return hipGetLastError();
}

// ------------------------------------------------------------ Gram matrices
// partial P = X^T Y over one chunk of rows.  Thread t owns the outputs
// e = t + 256 i: fixed column c2 = t mod Lp and rows c1 = t / Lp + i (256/Lp).
__global__ __launch_bounds__(kThreads) void b_gram_part(const BJobDesc *__restrict__ jobs, int njob,
                                                        const int *__restrict__ toff,
                                                        const int64_t *__restrict__ clock, int Xc, int Yc) {
  constexpr int RB = 16;  // rows staged per batch
  constexpr int MO = kBlockMaxLp * kBlockMaxLp / kThreads;
  __shared__ double Xs[RB * kBlockMaxLp], Ys[RB * kBlockMaxLp];
  const int g = blockIdx.x;
  const int j = bfind(toff, njob, g);
  const BJobDesc &J = jobs[j];
  const int k = (int)(*clock - J.start_clock);
  if (k >= J.Kstop) return;
  const int chunk = g - toff[j];
  const int Lp = J.Lp, lg = J.lgLp, L2 = Lp * Lp;
  const GLB double *__restrict__ X = bbuf(J, Xc, k);
  const GLB double *__restrict__ Y = bbuf(J, Yc, k);
  const int t = threadIdx.x;
  const int c2 = t & (Lp - 1);
  const int c1base = t >> lg;
  const int c1step = kThreads >> lg;
  const int nout = (L2 + kThreads - 1) / kThreads;
  const int64_t r0 = (int64_t)chunk * kChunk;
  int64_t r1 = r0 + kChunk;
  if (r1 > J.n) r1 = J.n;
  double acc[MO];
#pragma unroll
  for (int i = 0; i < MO; ++i) acc[i] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += RB) {
    for (int e = t; e < RB * Lp; e += kThreads) {
      const int64_t row = rb + (e >> lg);
      const int cc = e & (Lp - 1);
      Xs[e] = (row < r1) ? X[(row << lg) + cc] : 0.0;
      Ys[e] = (row < r1) ? Y[(row << lg) + cc] : 0.0;
    }
    __syncthreads();
    if (t < L2) {
      for (int rr = 0; rr < RB; ++rr) {
        const double y = Ys[(rr << lg) + c2];
        const double *xr = Xs + (rr << lg) + c1base;
#pragma unroll
        for (int i = 0; i < MO; ++i)
          if (i < nout) acc[i] = fma(xr[i * c1step], y, acc[i]);
      }
    }
    __syncthreads();
  }
  GLB double *__restrict__ P = gp(J.gpart) + (int64_t)chunk * L2;
#pragma unroll
  for (int i = 0; i < MO; ++i) {
    const int e = t + i * kThreads;
    if (i < nout && e < L2) P[e] = acc[i];
  }
}

// dest 0: A_k = sym(sum), 1: C_k = sum, 2: G = sum.  Grid (njob, 64).
__global__ __launch_bounds__(kThreads) void b_gram_reduce(const BJobDesc *__restrict__ jobs,
                                                          const int64_t *__restrict__ clock, int dest) {
  const BJobDesc &J = jobs[blockIdx.x];
  const int Lp = J.Lp, L2 = Lp * Lp;
  const int e = blockIdx.y * kThreads + threadIdx.x;
  if (e >= L2) return;
  const int k = (int)(*clock - J.start_clock);
  if (k >= J.Kstop) return;
  const GLB double *__restrict__ P = gp(J.gpart);
  double s = 0.0;
  for (int c = 0; c < J.rchunks; ++c) s += P[(int64_t)c * L2 + e];
  if (dest == 0) {
    const int et = (e & (Lp - 1)) * Lp + (e / Lp);
    double s2 = 0.0;
    for (int c = 0; c < J.rchunks; ++c) s2 += P[(int64_t)c * L2 + et];
    gp(J.Ah)[(int64_t)k * L2 + e] = 0.5 * (s + s2);
  } else if (dest == 1) {
    gp(J.Ch)[(int64_t)k * L2 + e] = s;
  } else {
    gp(J.G)[e] = s;
  }
}

hipError_t launch_b_gram(const BBatch &b, int X, int Y, int dest, hipStream_t st) {
  hipLaunchKernelGGL(b_gram_part, dim3(b.totalr), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffr, b.clock, X, Y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(b_gram_reduce, dim3(b.njob, kBlockMaxLp * kBlockMaxLp / kThreads), dim3(kThreads), 0, st,
                     b.jobs, b.clock, dest);
  return hipGetLastError();
}

// ----------------------------------------------------------- Cholesky step
// R = chol(G) (upper, G = R^T R); a non-positive pivot restarts once from
// G + s I with s = 1e-14 trace(G) (shifted CholeskyQR).  Rinv by back
// substitution, one column per thread.
__global__ __launch_bounds__(kThreads) void b_chol(const BJobDesc *__restrict__ jobs,
                                                   const int64_t *__restrict__ clock, int mode, int init) {
  __shared__ double A[kBlockMaxLp][kBlockMaxLp + 1];
  __shared__ double Ri[kBlockMaxLp][kBlockMaxLp + 1];
  __shared__ int dead[kBlockMaxLp];
  __shared__ double thr;
  const BJobDesc &J = jobs[blockIdx.x];
  const int Lp = J.Lp, L2 = Lp * Lp;
  const int k = (int)(*clock - J.start_clock);
  if (k >= J.Kstop) return;
  const int t = threadIdx.x;
  const GLB double *__restrict__ G = gp(J.G);
  // Deflation threshold on the pivots.  First pass: a column whose part
  // outside the span of the earlier columns is below kDeflTol * ||A^T A||
  // (or, for the starting block, kDeflTol * its largest column norm) is
  // dropped.  Second pass: the block is already near orthonormal, so the
  // threshold is kDeflTol on unit columns.
  if (t == 0) {
    double sc;
    if (mode == 2) {
      sc = 1.0;
    } else if (init) {
      double mx = 0.0;
      for (int i = 0; i < Lp; ++i) mx = fmax(mx, G[i * Lp + i]);
      sc = sqrt(mx);
    } else {
      sc = J.dscale;
    }
    thr = (kDeflTol * sc) * (kDeflTol * sc);
  }
  for (int e = t; e < L2; e += kThreads) {
    const int i = e / Lp, jj = e - i * Lp;
    A[i][jj] = G[e];
  }
  __syncthreads();
  // right-looking Cholesky; a deflated column gets a zero row in R
  for (int c = 0; c < Lp; ++c) {
    if (t == 0) {
      const double d = A[c][c];
      const int dd = !(d > thr);
      dead[c] = dd;
      A[c][c] = dd ? 0.0 : sqrt(d);
    }
    __syncthreads();
    const int dd = dead[c];
    for (int jj = c + 1 + t; jj < Lp; jj += kThreads) A[c][jj] = dd ? 0.0 : A[c][jj] / A[c][c];
    __syncthreads();
    if (!dd) {
      const int rem = Lp - c - 1;
      for (int e = t; e < rem * rem; e += kThreads) {
        const int i = c + 1 + e / rem, jj = c + 1 + e % rem;
        if (jj >= i) A[i][jj] -= A[c][i] * A[c][jj];
      }
    }
    __syncthreads();
  }
  if (mode == 2 && t == 0) {
    int nd = 0;
    for (int c = 0; c < Lp; ++c) nd += dead[c];
    gp(J.flags)[0] = nd;
  }
  // upper R: A[i][j], j >= i, zero rows at deflated columns.  Its
  // pseudo-inverse on the kept columns, column by column (deflated rows and
  // columns of Ri are zero).
  if (t < Lp) {
    const int c = t;
    for (int i = Lp - 1; i >= 0; --i) {
      double v = 0.0;
      if (i <= c && !dead[i] && !dead[c]) {
        v = (i == c) ? 1.0 : 0.0;
        for (int l2 = i + 1; l2 <= c; ++l2) v -= A[i][l2] * Ri[l2][c];
        v /= A[i][i];
      }
      Ri[i][c] = v;
    }
  }
  __syncthreads();
  if (mode == 1) {
    for (int e = t; e < L2; e += kThreads) {
      const int i = e / Lp, jj = e - i * Lp;
      gp(J.R1)[e] = (jj >= i) ? A[i][jj] : 0.0;
      gp(J.R1inv)[e] = Ri[i][jj];
    }
    if (init && t < Lp) gp(J.beta0)[t] = sqrt(G[t * Lp + t]);
  } else {
    // M = R1inv R2inv (upper x upper), B = R2 R1
    const GLB double *__restrict__ R1 = gp(J.R1);
    const GLB double *__restrict__ R1i = gp(J.R1inv);
    const int64_t mdst = (int64_t)(init ? J.Kcap : k) * L2;
    const int64_t bdst = (int64_t)(init ? 0 : k + 1) * L2;
    for (int e = t; e < L2; e += kThreads) {
      const int i = e / Lp, jj = e - i * Lp;
      double m = 0.0, bb = 0.0;
      for (int l2 = i; l2 <= jj; ++l2) {
        m += R1i[i * Lp + l2] * Ri[l2][jj];
        bb += ((l2 >= i) ? A[i][l2] : 0.0) * R1[l2 * Lp + jj];
      }
      gp(J.Mh)[mdst + e] = (jj >= i) ? m : 0.0;
      gp(J.Bh)[bdst + e] = (jj >= i) ? bb : 0.0;
    }
  }
}

hipError_t launch_b_chol(const BBatch &b, int mode, int init, hipStream_t st) {
  hipLaunchKernelGGL(b_chol, dim3(b.njob), dim3(kThreads), 0, st, b.jobs, b.clock, mode, init);
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
// One block per shift of one job: Y_k overwrites Z_k (columns < L).
__global__ __launch_bounds__(kThreads) void b_backsolve(BJobDesc J, int K) {
  const int s = blockIdx.x;
  const int Lp = J.Lp, L2 = Lp * Lp, L = J.L;
  const int t = threadIdx.x;
  const int64_t hbase = (int64_t)s * (J.Kcap + 1) * L2;
  GLB double2 *__restrict__ Hinv = gp(J.Hinv) + hbase;
  GLB double2 *__restrict__ Zh = gp(J.Zh) + hbase;
  GLB double2 *__restrict__ T1 = gp(J.ctmp) + (int64_t)s * 2 * L2;
  GLB double2 *__restrict__ Yn = T1 + L2;  // Y_{k+1}
  for (int k = K - 1; k >= 0; --k) {
    // T1 = Z_k + B_{k+1}^T Y_{k+1}
    const GLB double *__restrict__ Bk1 = gp(J.Bh) + (int64_t)(k + 1) * L2;
    const GLB double2 *__restrict__ Zk = Zh + (int64_t)k * L2;
    for (int e = t; e < Lp * L; e += kThreads) {
      const int i = e / L, jj = e - i * L;
      double2 acc = Zk[i * Lp + jj];
      if (k < K - 1) {
        for (int c = 0; c <= i; ++c) {  // (B^T)[i][c] = B[c][i], B upper
          const double bv = Bk1[c * Lp + i];
          const double2 y = Yn[c * Lp + jj];
          acc.x = fma(bv, y.x, acc.x);
          acc.y = fma(bv, y.y, acc.y);
        }
      }
      T1[i * Lp + jj] = acc;
    }
    __syncthreads();
    const GLB double2 *__restrict__ Hk = Hinv + (int64_t)k * L2;
    for (int e = t; e < Lp * L; e += kThreads) {
      const int i = e / L, jj = e - i * L;
      double2 acc = make_double2(0.0, 0.0);
      for (int c = 0; c < Lp; ++c) {
        const double2 r = cmulb(Hk[i * Lp + c], T1[c * Lp + jj]);
        acc.x += r.x;
        acc.y += r.y;
      }
      Zh[(int64_t)k * L2 + i * Lp + jj] = acc;
    }
    __syncthreads();
    for (int e = t; e < Lp * L; e += kThreads) {
      const int i = e / L, jj = e - i * L;
      Yn[i * Lp + jj] = Zh[(int64_t)k * L2 + i * Lp + jj];
    }
    __syncthreads();
  }
}

hipError_t launch_b_backsolve(const BJobDesc &hj, int K, hipStream_t st) {
  hipLaunchKernelGGL(b_backsolve, dim3(hj.S), dim3(kThreads), 0, st, hj, K);
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
