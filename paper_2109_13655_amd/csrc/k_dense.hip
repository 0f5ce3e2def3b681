// Dense FP64 kernels for steps 3-5 of Algorithms 1/2 on gfx950.
//
//   * Householder QR of a tall column-major matrix (step 3: QR of S-hat;
//     step 4: [U~, B] = qr(A V~)), one launch per column, one block per
//     trailing column; reflectors stored LAPACK-style below the diagonal.
//   * Application of the reflector product to a block (to form V~ = Q [U_R; 0]
//     and U-hat = Q_X [P_sel; 0]); each block owns one column of the block
//     and runs the whole reflector sequence on it in one launch.
//   * One-sided Jacobi SVD steps (round-robin pairing, one block per pair),
//     for the small r x r matrices R^T and B.
//   * FP64 MFMA GEMM (v_mfma_f64_16x16x4f64) for V-hat = V~ Q_sel.
//   * Column norms, column scaling, sign normalisation and residual norms.
// All reductions are fixed-order block trees, so results are reproducible.
#include <algorithm>

#include "csvd_impl.h"

namespace csvd {

// Sum over a wave by a butterfly; lane 0's result (a fixed order of additions)
__device__ __forceinline__ double wave_sum0(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over the kThreads threads of a block in a fixed order: butterflies in
// each wave, then the waves' sums (lane 0) in order.  Every thread gets it.
__device__ __forceinline__ double block_reduce(double v, double *red) {
  static_assert(kThreads == 256, "four waves");
  const int t = threadIdx.x;
  v = wave_sum0(v);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// Reflector for column j (rows j..rows-1) of X: H = I - tau v v^T with
// v = [1; x_{j+1:}/(x_j - beta)], beta = -sign(x_j) ||x_{j:}||, X[j,j] <- beta.
__device__ void make_reflector(double *X, int64_t ld, int rows, int j, double *tau, double *red) {
  double *col = X + (int64_t)j * ld;
  double s = 0.0;
  for (int64_t i = j + 1 + threadIdx.x; i < rows; i += kThreads) s = fma(col[i], col[i], s);
  const double xn2 = block_reduce(s, red);
  const double x0 = col[j];
  if (xn2 == 0.0) {
    if (threadIdx.x == 0) tau[j] = 0.0;
    return;
  }
  const double beta = -copysign(sqrt(x0 * x0 + xn2), x0);
  const double scale = 1.0 / (x0 - beta);
  for (int64_t i = j + 1 + threadIdx.x; i < rows; i += kThreads) col[i] *= scale;
  if (threadIdx.x == 0) {
    tau[j] = (beta - x0) / beta;
    col[j] = beta;
  }
}

__global__ __launch_bounds__(kThreads) void k_hh_make(double *X, int64_t ld, int rows, int j, double *tau) {
  __shared__ double red[kThreads];
  make_reflector(X, ld, rows, j, tau, red);
}

// Apply H_j to column c = j+1+blockIdx.x; the block of column j+1 then
// builds reflector j+1.
__global__ __launch_bounds__(kThreads) void k_hh_step(double *X, int64_t ld, int rows, int j, double *tau) {
  __shared__ double red[kThreads];
  const int c = j + 1 + blockIdx.x;
  const double *v = X + (int64_t)j * ld;
  double *y = X + (int64_t)c * ld;
  const double tj = tau[j];
  if (tj != 0.0) {
    double s = 0.0;
    for (int64_t i = j + 1 + threadIdx.x; i < rows; i += kThreads) s = fma(v[i], y[i], s);
    const double d = (block_reduce(s, red) + y[j]) * tj;
    for (int64_t i = j + 1 + threadIdx.x; i < rows; i += kThreads) y[i] = fma(-d, v[i], y[i]);
    __syncthreads();  // every thread has read y[j] before it changes
    if (threadIdx.x == 0) y[j] -= d;
    __syncthreads();
  }
  if (c == j + 1 && c < rows) make_reflector(X, ld, rows, c, tau, red);
}

hipError_t launch_hh_make(double *X, int64_t ld, int rows, int j, double *tau, hipStream_t st) {
  hipLaunchKernelGGL(k_hh_make, dim3(1), dim3(kThreads), 0, st, X, ld, rows, j, tau);
  return hipGetLastError();
}

hipError_t launch_hh_step(double *X, int64_t ld, int rows, int cols, int j, double *tau, hipStream_t st) {
  if (cols - j - 1 <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hh_step, dim3(cols - j - 1), dim3(kThreads), 0, st, X, ld, rows, j, tau);
  return hipGetLastError();
}

// Z <- H_{j_first} ... (each block: one column of Z).  dir = -1 applies
// j = nref-1 .. 0 (Z <- Q Z with Q = H_0 H_1 ... H_{nref-1});
// dir = +1 applies j = 0 .. nref-1 (Z <- Q^T Z).
__global__ __launch_bounds__(kThreads) void k_hh_apply(const double *Xr, int64_t ldr, int rows, int nref, int dir,
                                                       const double *tau, double *Z, int64_t ldz) {
  __shared__ double red[kThreads];
  double *y = Z + (int64_t)blockIdx.x * ldz;
  for (int q = 0; q < nref; ++q) {
    const int j = dir < 0 ? nref - 1 - q : q;
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const double *v = Xr + (int64_t)j * ldr;
    double s = 0.0;
    for (int64_t i = j + 1 + threadIdx.x; i < rows; i += kThreads) s = fma(v[i], y[i], s);
    const double d = (block_reduce(s, red) + y[j]) * tj;
    for (int64_t i = j + 1 + threadIdx.x; i < rows; i += kThreads) y[i] = fma(-d, v[i], y[i]);
    __syncthreads();
    if (threadIdx.x == 0) y[j] -= d;
    __syncthreads();
  }
}

// nref reflectors; j encodes the direction: j < 0 -> Q Z, j >= 0 -> Q^T Z
hipError_t launch_hh_apply(const double *Xr, int64_t ldr, int rows, int nref_dir, const double *tau, double *Z,
                           int64_t ldz, int zcols, hipStream_t st) {
  if (zcols <= 0) return hipSuccess;
  const int nref = nref_dir < 0 ? -nref_dir : nref_dir;
  const int dir = nref_dir < 0 ? -1 : 1;
  hipLaunchKernelGGL(k_hh_apply, dim3(zcols), dim3(kThreads), 0, st, Xr, ldr, rows, nref, dir, tau, Z, ldz);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Jacobi
// A pair is rotated while |a_p^T a_q| > tol ||a_p|| ||a_q|| and both squared
// norms exceed floor2.  The norms multiply after their square roots, so the
// test cannot underflow; floor2 (the caller passes (eps^2 ||A||_F)^2, and
// rotations leave ||A||_F unchanged) keeps columns far below the rounding
// level of the whole matrix out of rotations: in denormal arithmetic a
// rotation need not reduce |a_p^T a_q|, and a sweep would never end
// rotation-free.  Above the floor |zeta| < 1 / (2 tol eps^2), which is finite.
__device__ inline bool rotate_pair(double app, double aqq, double apq, double tol, double floor2) {
  return apq != 0.0 && app > floor2 && aqq > floor2 && fabs(apq) > tol * (sqrt(app) * sqrt(aqq));
}

// Round-robin pairing over n (even) columns: index n-1 stays, the others
// rotate; step s pairs (n-1, s) and ((s+b) mod (n-1), (s-b) mod (n-1)).
__global__ __launch_bounds__(kThreads) void k_jacobi(double *A, int64_t lda, int rows, int ncol, double *V,
                                                     int64_t ldv, int vrows, int step, double tol, double floor2,
                                                     int *counter) {
  __shared__ double r0[4], r1[4], r2[4];
  const int b = blockIdx.x;
  const int n1 = ncol - 1;
  int p, q;
  if (b == 0) {
    p = step;
    q = n1;
  } else {
    p = (step + b) % n1;
    q = (step - b + n1) % n1;
  }
  if (p > q) {
    int tmp = p;
    p = q;
    q = tmp;
  }
  double *ap = A + (int64_t)p * lda, *aq = A + (int64_t)q * lda;
  double spp = 0.0, sqq = 0.0, spq = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += kThreads) {
    const double x = ap[i], y = aq[i];
    spp = fma(x, x, spp);
    sqq = fma(y, y, sqq);
    spq = fma(x, y, spq);
  }
  const int t = threadIdx.x;
  spp = wave_sum0(spp);
  sqq = wave_sum0(sqq);
  spq = wave_sum0(spq);
  if ((t & 63) == 0) {
    r0[t >> 6] = spp;
    r1[t >> 6] = sqq;
    r2[t >> 6] = spq;
  }
  __syncthreads();
  const double app = (r0[0] + r0[1]) + (r0[2] + r0[3]);
  const double aqq = (r1[0] + r1[1]) + (r1[2] + r1[3]);
  const double apq = (r2[0] + r2[1]) + (r2[2] + r2[3]);
  if (!rotate_pair(app, aqq, apq, tol, floor2)) return;
  const double zeta = (aqq - app) / (2.0 * apq);
  const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + tt * tt);
  const double s = c * tt;
  for (int64_t i = threadIdx.x; i < rows; i += kThreads) {
    const double x = ap[i], y = aq[i];
    ap[i] = c * x - s * y;
    aq[i] = s * x + c * y;
  }
  double *vp = V + (int64_t)p * ldv, *vq = V + (int64_t)q * ldv;
  for (int64_t i = threadIdx.x; i < vrows; i += kThreads) {
    const double x = vp[i], y = vq[i];
    vp[i] = c * x - s * y;
    vq[i] = s * x + c * y;
  }
  if (threadIdx.x == 0) atomicAdd(counter, 1);
}

hipError_t launch_jacobi_step(double *A, int64_t lda, int rows, int cols_even, double *V, int64_t ldv, int vrows,
                              int step, double tol, double floor2, int *counter, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi, dim3(cols_even / 2), dim3(kThreads), 0, st, A, lda, rows, cols_even, V, ldv, vrows,
                     step, tol, floor2, counter);
  return hipGetLastError();
}

// Block-pair one-sided Jacobi.  The ncol columns form nb = ncol / W blocks;
// launch `step` of a sweep pairs the blocks by the same round-robin as the
// per-column kernel pairs columns, and each workgroup copies its two blocks
// of A (rows) and V (vrows) to LDS and rotates pairs among their 2W columns
// there: on step 0 every pair (each block is in exactly one block pair, so
// every pair within a block is checked once per sweep), on the other steps
// the W x W pairs across the two blocks.  Each round has W disjoint pairs,
// one per wave; the wave's sums are xor butterflies.  The rotation and its
// test are those of k_jacobi.
template <int W, int RMAX>
__global__ __launch_bounds__(W * 64) void k_jacobi_blk(double *A, int64_t lda, int rows, int ncol, double *V,
                                                       int64_t ldv, int vrows, int step, double tol, double floor2,
                                                       int *counter) {
  static_assert(RMAX % 64 == 0, "whole rows per lane");
  constexpr int KR = RMAX / 64;  // rows per lane
  __shared__ double As[2 * W * RMAX], Vs[2 * W * RMAX];
  const int nb = ncol / W, n1 = nb - 1;
  const int b = blockIdx.x;
  int p, q;
  if (b == 0) {
    p = step;
    q = n1;
  } else {
    p = (step + b) % n1;
    q = (step - b + n1) % n1;
  }
  if (p > q) {
    const int tmp = p;
    p = q;
    q = tmp;
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  // local column c: block p for c < W, block q for c >= W
  auto gcol = [&](int c) { return c < W ? p * W + c : q * W + (c - W); };
  // each wave copies columns w and w + W of A and V: every load of the wave
  // is issued before the first LDS store
  {
    double ta[2][KR], tv[2][KR];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double *a = A + (int64_t)gcol(w + h * W) * lda;
      const double *v = V + (int64_t)gcol(w + h * W) * ldv;
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = l + 64 * k;
        ta[h][k] = i < rows ? a[i] : 0.0;
        tv[h][k] = i < vrows ? v[i] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = l + 64 * k;
        if (i < rows) As[(w + h * W) * RMAX + i] = ta[h][k];
        if (i < vrows) Vs[(w + h * W) * RMAX + i] = tv[h][k];
      }
  }
  __syncthreads();
  int rot = 0;
  const int nrounds = (step == 0) ? 2 * W - 1 : W;
  for (int r = 0; r < nrounds; ++r) {
    int x, y;
    if (step == 0) {  // round-robin over the 2W local columns, 2W - 1 fixed
      constexpr int m1 = 2 * W - 1;
      if (w == 0) {
        x = r;
        y = m1;
      } else {
        x = (r + w) % m1;
        y = (r - w + m1) % m1;
      }
      if (x > y) {
        const int tmp = x;
        x = y;
        y = tmp;
      }
    } else {
      x = w;
      y = W + (w + r) % W;
    }
    // the pair's rows stay in registers from the sums to the rotation; rows
    // past `rows` read as zero and add nothing (the sums never hold -0)
    double *ax = As + x * RMAX, *ay = As + y * RMAX;
    double u[KR], v[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = l + 64 * k;
      u[k] = i < rows ? ax[i] : 0.0;
      v[k] = i < rows ? ay[i] : 0.0;
    }
    double spp = 0.0, sqq = 0.0, spq = 0.0;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      spp = fma(u[k], u[k], spp);
      sqq = fma(v[k], v[k], sqq);
      spq = fma(u[k], v[k], spq);
    }
    // after the xor butterflies every lane holds the same sums (addition
    // commutes), so all lanes take the same decision
    const double app = wave_sum0(spp);
    const double aqq = wave_sum0(sqq);
    const double apq = wave_sum0(spq);
    if (rotate_pair(app, aqq, apq, tol, floor2)) {
      const double zeta = (aqq - app) / (2.0 * apq);
      const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double c = 1.0 / sqrt(1.0 + tt * tt);
      const double s = c * tt;
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = l + 64 * k;
        if (i < rows) {
          ax[i] = c * u[k] - s * v[k];
          ay[i] = s * u[k] + c * v[k];
        }
      }
      double *vx = Vs + x * RMAX, *vy = Vs + y * RMAX;
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = l + 64 * k;
        if (i < vrows) {
          const double a = vx[i], b = vy[i];
          vx[i] = c * a - s * b;
          vy[i] = s * a + c * b;
        }
      }
      ++rot;
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double *a = A + (int64_t)gcol(w + h * W) * lda;
    double *v = V + (int64_t)gcol(w + h * W) * ldv;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = l + 64 * k;
      if (i < rows) a[i] = As[(w + h * W) * RMAX + i];
      if (i < vrows) v[i] = Vs[(w + h * W) * RMAX + i];
    }
  }
  if (l == 0 && rot > 0) atomicAdd(counter, rot);
}

int jacobi_block_width(int n) {
  if (n <= 256) return 16;
  if (n <= 512) return 8;
  return 0;
}

int jacobi_padded_cols(int n) {
  const int w = jacobi_block_width(n);
  if (w == 0) return n + (n & 1);
  return (n + 2 * w - 1) / (2 * w) * (2 * w);
}

hipError_t launch_jacobi_blk(double *A, int64_t lda, int rows, int ncol, double *V, int64_t ldv, int vrows, int step,
                             double tol, double floor2, int *counter, hipStream_t st) {
  const int w = jacobi_block_width(ncol);  // the width the columns were padded for
  if (w == 0 || ncol % (2 * w) != 0 || rows > 4096 / w || vrows > 4096 / w || step < 0 || step >= ncol / w - 1)
    return hipErrorInvalidValue;
  if (w == 16)
    hipLaunchKernelGGL((k_jacobi_blk<16, 256>), dim3(ncol / 32), dim3(1024), 0, st, A, lda, rows, ncol, V, ldv, vrows,
                       step, tol, floor2, counter);
  else
    hipLaunchKernelGGL((k_jacobi_blk<8, 512>), dim3(ncol / 16), dim3(512), 0, st, A, lda, rows, ncol, V, ldv, vrows,
                       step, tol, floor2, counter);
  return hipGetLastError();
}

// ------------------------------------------------------------ small helpers
// dst[c * ldd + r] = src[c * lds + r] for r < rows, c < cols (column-major
// blocks with different leading dimensions; replaces strided 2-D copies)
__global__ __launch_bounds__(kThreads) void k_copy_block(const double *__restrict__ src, int64_t lds,
                                                         double *__restrict__ dst, int64_t ldd, int64_t rows) {
  const int c = blockIdx.y;
  const GLB double *s = gp(src) + (int64_t)c * lds;
  GLB double *d = gp(dst) + (int64_t)c * ldd;
  for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < rows; r += (int64_t)gridDim.x * kThreads)
    d[r] = s[r];
}

hipError_t launch_copy_block(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows, int cols,
                             hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int gx = (int)std::min<int64_t>((rows + kThreads - 1) / kThreads, 1024);
  hipLaunchKernelGGL(k_copy_block, dim3(gx, cols), dim3(kThreads), 0, st, src, lds, dst, ldd, rows);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_col_norms(const double *A, int64_t lda, int rows, double *out) {
  __shared__ double red[kThreads];
  const double *a = A + (int64_t)blockIdx.x * lda;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += kThreads) s = fma(a[i], a[i], s);
  const double r = block_reduce(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(r);
}

hipError_t launch_col_norms(const double *A, int64_t lda, int rows, int cols, double *out, hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_norms, dim3(cols), dim3(kThreads), 0, st, A, lda, rows, out);
  return hipGetLastError();
}

__global__ void k_scale_cols(double *A, int64_t lda, int rows, const double *s) {
  double *a = A + (int64_t)blockIdx.y * lda;
  const double f = s[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
    a[i] *= f;
}

hipError_t launch_scale_cols(double *A, int64_t lda, int rows, int cols, const double *s, hipStream_t st) {
  if (cols <= 0 || rows <= 0) return hipSuccess;
  int gx = (rows + 255) / 256;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(k_scale_cols, dim3(gx, cols), dim3(256), 0, st, A, lda, rows, s);
  return hipGetLastError();
}

// Largest |V[:, c]| entry (first index on ties) made positive; U follows.
__global__ __launch_bounds__(kThreads) void k_sign_fix(double *U, int64_t ldu, int urows, double *V, int64_t ldv,
                                                       int vrows) {
  __shared__ double bv[kThreads];
  __shared__ int bi[kThreads];
  const int c = blockIdx.x, t = threadIdx.x;
  const double *v = V + (int64_t)c * ldv;
  double best = -1.0;
  int besti = 0;
  for (int i = t; i < vrows; i += kThreads) {
    const double a = fabs(v[i]);
    if (a > best) {
      best = a;
      besti = i;
    }
  }
  bv[t] = best;
  bi[t] = besti;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      if (bv[t + off] > bv[t] || (bv[t + off] == bv[t] && bi[t + off] < bi[t])) {
        bv[t] = bv[t + off];
        bi[t] = bi[t + off];
      }
    }
    __syncthreads();
  }
  const bool neg = v[bi[0]] < 0.0;
  __syncthreads();
  if (!neg) return;
  double *vv = V + (int64_t)c * ldv;
  for (int i = t; i < vrows; i += kThreads) vv[i] = -vv[i];
  double *uu = U + (int64_t)c * ldu;
  for (int i = t; i < urows; i += kThreads) uu[i] = -uu[i];
}

hipError_t launch_sign_fix(double *U, int64_t ldu, int urows, double *V, int64_t ldv, int vrows, int cols,
                           hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_fix, dim3(cols), dim3(kThreads), 0, st, U, ldu, urows, V, ldv, vrows);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_resid_cols(const double *X, const double *Y, int64_t ldy,
                                                         const double *s, int rows, int cols, double *out) {
  __shared__ double red[kThreads];
  const int c = blockIdx.x;
  const double sc = s[c];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += kThreads) {
    const double d = X[i * cols + c] - sc * Y[(int64_t)c * ldy + i];
    acc = fma(d, d, acc);
  }
  const double r = block_reduce(acc, red);
  if (threadIdx.x == 0) out[c] = r;
}

hipError_t launch_resid_cols(const double *X, const double *Y, int64_t ldy, const double *s, int rows, int cols,
                             double *out, hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid_cols, dim3(cols), dim3(kThreads), 0, st, X, Y, ldy, s, rows, cols, out);
  return hipGetLastError();
}

// -------------------------------------------------------------- MFMA GEMM
// C = alpha A B + beta C, column-major, FP64 on the matrix cores.
// Block: 64 x 64 tile of C, 4 waves, each wave a 32 x 32 quadrant made of
// 2 x 2 MFMA 16x16 tiles; K is staged through LDS 16 at a time.
// Operand layout of v_mfma_f64_16x16x4f64 (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the result lane l holds
// D[l / 16 + 4 v][l % 16], v = 0..3 (rows interleaved by lane group; checked
// on the device with unit and random operands).
typedef double d4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------- blocked QR
// Householder QR in panels of kHB columns (LAPACK's blocked form): each panel
// is factored by the reflector kernels above; its reflectors are gathered as
// I - V T V^T (T upper triangular, from V^T V and tau), and the trailing
// columns are updated with two tall products on FP64 MFMA:
//   W = V^T C  (partial sums per workgroup over row chunks, fixed-order
//              reduction),  C -= V (T^T W).
// Q Z is applied the same way panel by panel, from the last: Z -= V (T (V^T Z)).
// V is read as a view of the factored columns: column i of the panel that
// starts at j0 is 0 above row j0 + i, 1 at row j0 + i, X below.
typedef double v4dd __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4dd mfma4d(double a, double b, v4dd c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double vview(const double *X, int64_t ld, int j0, int i, int jb, int64_t r) {
  const int64_t d = (int64_t)j0 + i;
  if (i >= jb || r < d) return 0.0;
  if (r == d) return 1.0;
  return X[(j0 + i) * ld + r];
}

constexpr int kTGChunk = 64;
constexpr int kTGMaxVB = 256;

// partial W over the row chunks of workgroup vb: part[vb][i][c], i < kHB,
// c < p2.  C(r, c) is column-major (ldc), or (cv = 1) the same V view.
__global__ __launch_bounds__(256) void k_tg_part(const double *__restrict__ X, int64_t ld, int j0, int jb,
                                                  int64_t rows, const double *__restrict__ C, int64_t ldc, int cv,
                                                  int p2, int nvb, double *__restrict__ part) {
  __shared__ double Vs[kTGChunk][kHB + 1];
  __shared__ double Cs[kTGChunk][64 + 1];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const int vb = blockIdx.x, col0 = blockIdx.y * 64;
  const int64_t r0 = j0, nchunk = (rows - r0 + kTGChunk - 1) / kTGChunk;
  // wave w: output tiles (ti, tj) = (w >> 2 ... ): 2 x 4 tiles of 16 x 16 over 4 waves
  v4dd acc[2];
  acc[0] = acc[1] = v4dd{0.0, 0.0, 0.0, 0.0};
  // thread t stages row t % 64 of the chunk for columns t / 64 + 4 u; the
  // column index is the same across the wave (scalar addressing)
  static_assert(kTGChunk == 64, "one row per lane");
  constexpr int NV = kTGChunk * kHB / 256, NC = kTGChunk * 64 / 256;
  const int wi = __builtin_amdgcn_readfirstlane(w);
  for (int64_t ch = vb; ch < nchunk; ch += nvb) {
    const int64_t r = r0 + ch * kTGChunk + l;
    const bool rok = r < rows;
    // every load of the chunk is issued before the first LDS store
    double vv[NV], cc[NC];
#pragma unroll
    for (int u = 0; u < NV; ++u) vv[u] = rok ? vview(X, ld, j0, wi + 4 * u, jb, r) : 0.0;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const int c = col0 + wi + 4 * u;
      double v = 0.0;
      if (rok && c < p2) v = cv ? vview(X, ld, j0, c, jb, r) : C[(int64_t)c * ldc + r];
      cc[u] = v;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NV; ++u) Vs[l][wi + 4 * u] = vv[u];
#pragma unroll
    for (int u = 0; u < NC; ++u) Cs[l][wi + 4 * u] = cc[u];
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int tau = w + 4 * s2;  // 0..7: ti = tau / 4, tj = tau % 4
      const int ti = tau >> 2, tj = tau & 3;
#pragma unroll
      for (int ks = 0; ks < kTGChunk / 4; ++ks) {
        const int k = 4 * ks + q;
        acc[s2] = mfma4d(Vs[k][16 * ti + rl], Cs[k][16 * tj + rl], acc[s2]);
      }
    }
  }
  double *P = part + (int64_t)vb * kHB * p2;
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2) {
    const int tau = w + 4 * s2;
    const int ti = tau >> 2, tj = tau & 3;
    const int c = col0 + 16 * tj + rl;
    if (c < p2)
#pragma unroll
      for (int v = 0; v < 4; ++v) P[(int64_t)(16 * ti + q + 4 * v) * p2 + c] = acc[s2][v];
  }
}

// W[i][c] = sum_vb part[vb][i][c] in a fixed order (8 interleaved sums)
__global__ __launch_bounds__(256) void k_tg_reduce(const double *__restrict__ part, int nvb, int total,
                                                    double *__restrict__ W) {
  __shared__ double sp[8][32];
  const int t = threadIdx.x, grp = t >> 5;
  const int o = blockIdx.x * 32 + (t & 31);
  double s = 0.0;
  if (o < total)
#pragma unroll 8
    for (int vb = grp; vb < nvb; vb += 8) s += part[(int64_t)vb * total + o];
  sp[grp][t & 31] = s;
  __syncthreads();
  if (grp == 0 && o < total) {
    double r = sp[0][t];
    for (int h = 1; h < 8; ++h) r += sp[h][t];
    W[o] = r;
  }
}

// T (kHB x kHB, row-major, upper) from G = V^T V (kHB x kHB row-major) and
// tau: T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j).
__global__ __launch_bounds__(256) void k_tmat(const double *__restrict__ G, const double *__restrict__ tau, int j0,
                                               int jb, double *__restrict__ T) {
  __shared__ double Ts[kHB][kHB + 1];
  const int t = threadIdx.x;
  for (int e = t; e < kHB * kHB; e += 256) Ts[e / kHB][e % kHB] = 0.0;
  __syncthreads();
  for (int j = 0; j < jb; ++j) {
    const double tj = tau[j0 + j];
    if (t < j) {
      double s = 0.0;
      for (int l2 = t; l2 < j; ++l2) s = fma(Ts[t][l2], G[l2 * kHB + j], s);
      Ts[t][j] = -tj * s;
    }
    if (t == 0) Ts[j][j] = tj;
    __syncthreads();
  }
  for (int e = t; e < kHB * kHB; e += 256) T[e] = Ts[e / kHB][e % kHB];
}

// C(r, c) -= sum_i V(r, i) W2(i, c), r >= j0, with W2 = T^T W (trans = 1) or
// T W; 64 rows x 64 columns per workgroup, C written back in column segments
// through LDS.
// W2 = op(T) W (kHB x p2, row-major; op(T) = T^T when trans): the product
// every row tile of the trailing update applies, formed once per panel
__global__ __launch_bounds__(256) void k_tw(const double *__restrict__ T, int trans, const double *__restrict__ W,
                                             int p2, double *__restrict__ W2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)kHB * p2) return;
  const int i = (int)(e / p2), c = (int)(e - (int64_t)i * p2);
  double s = 0.0;
  for (int k = 0; k < kHB; ++k) s = fma(trans ? T[k * kHB + i] : T[i * kHB + k], W[(int64_t)k * p2 + c], s);
  W2[e] = s;
}

__global__ __launch_bounds__(256) void k_tu(const double *__restrict__ X, int64_t ld, int j0, int jb, int64_t rows,
                                             const double *__restrict__ W2g, int p2, double *__restrict__ C,
                                             int64_t ldc) {
  __shared__ double W2[kHB][64 + 1];
  __shared__ double Cs[64][65];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const int64_t rb = (int64_t)j0 + (int64_t)blockIdx.x * 64;
  const int col0 = blockIdx.y * 64;
  for (int e = t; e < kHB * 64; e += 256) {
    const int i = e / 64, c = e % 64;
    W2[i][c] = (col0 + c < p2) ? W2g[(int64_t)i * p2 + col0 + c] : 0.0;
  }
  __syncthreads();
  v4dd acc[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) acc[tj] = v4dd{0.0, 0.0, 0.0, 0.0};
  const int64_t r = rb + 16 * w + rl;
#pragma unroll
  for (int ks = 0; ks < kHB / 4; ++ks) {
    const int k = 4 * ks + q;
    const double a = (r < rows) ? vview(X, ld, j0, k, jb, r) : 0.0;
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = mfma4d(a, W2[k][16 * tj + rl], acc[tj]);
  }
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) Cs[16 * tj + rl][16 * w + q + 4 * v] = acc[tj][v];
  __syncthreads();
  // every load of the tile's C entries is issued before the first store
  constexpr int NE = 64 * 64 / 256;
  double cv[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = t + 256 * u, c = e >> 6, rr = e & 63;
    const int64_t row = rb + rr;
    cv[u] = (col0 + c < p2 && row < rows) ? C[(int64_t)(col0 + c) * ldc + row] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = t + 256 * u, c = e >> 6, rr = e & 63;
    const int64_t row = rb + rr;
    if (col0 + c < p2 && row < rows) C[(int64_t)(col0 + c) * ldc + row] = cv[u] - Cs[c][rr];
  }
}

// Panel factorisation: reflector j of the panel [j0, jend) in three
// row-parallel launches.  pf_dots: per row block, T_c = sum_{r > j} X(r, j)
// X(r, c) for c = j .. jend-1 (T_j = ||x(j+1:)||^2).  pf_coef (one block):
// fixed-order sums, beta = -sign(x_j) sqrt(x_j^2 + T_j), scale = 1/(x_j -
// beta), tau = (beta - x_j)/beta and w_c = tau (X(j, c) + scale T_c) for c > j.
// pf_update: X(r, j) <- scale X(r, j) (the reflector, r > j), X(j, j) <- beta,
// X(r, c) -= w_c v_r for c > j (v_j = 1).  Same formulas as make_reflector
// and k_hh_step, with the work spread over all rows.
constexpr int kPFRows = 512;  // rows per workgroup in the panel kernels

__global__ __launch_bounds__(256) void k_pf_dots(const double *__restrict__ X, int64_t ld, int rows, int j, int jend,
                                                  double *__restrict__ part) {
  __shared__ double red[kHB][256 / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int nc = jend - j;
  const int64_t rb = (int64_t)j + 1 + (int64_t)blockIdx.x * kPFRows;
  double acc[kHB];
#pragma unroll
  for (int c = 0; c < kHB; ++c) acc[c] = 0.0;
  // both rows of a thread are loaded before the first product (same order
  // of the products as a row-by-row loop)
  static_assert(kPFRows == 2 * 256, "two rows per thread");
  double xr[2], xc[2][kHB];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t r = rb + t + 256 * h;
    const bool ok = r < rows;
    xr[h] = ok ? X[(int64_t)j * ld + r] : 0.0;
#pragma unroll
    for (int c = 0; c < kHB; ++c) xc[h][c] = (ok && c < nc) ? X[(int64_t)(j + c) * ld + r] : 0.0;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (rb + t + 256 * h < rows)
#pragma unroll
      for (int c = 0; c < kHB; ++c)
        if (c < nc) acc[c] = fma(xr[h], xc[h][c], acc[c]);
  // fixed-order reduction: within the wave by xor-shuffles, then over waves
#pragma unroll
  for (int c = 0; c < kHB; ++c) {
    double v = acc[c];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[c][wv] = v;
  }
  __syncthreads();
  if (t < nc) part[(int64_t)blockIdx.x * kHB + t] = red[t][0] + red[t][1] + red[t][2] + red[t][3];
}

constexpr int kPFTile = 64;  // partial rows per LDS tile of pf_coef

__global__ __launch_bounds__(256) void k_pf_coef(const double *__restrict__ part, int nb, double *__restrict__ X,
                                                  int64_t ld, int j, int jend, double *__restrict__ tau,
                                                  double *__restrict__ coef) {
  // coef[0] = scale, coef[1] = beta, coef[2 + c] = w for column j + c (c >= 1)
  constexpr int kPer = kPFTile * kHB / 256;  // partials each thread stages per tile
  __shared__ double P[kPFTile * kHB];
  __shared__ double T[kHB];
  __shared__ double sh[2];
  const int t = threadIdx.x, nc = jend - j;
  // the partials of a tile are staged with all loads in flight, then added
  // in block order (entries of columns >= nc were not written: never read)
  double s = 0.0;
  for (int b0 = 0; b0 < nb; b0 += kPFTile) {
    double v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = t + 256 * u, b = b0 + e / kHB, c = e % kHB;
      v[u] = (b < nb && c < nc) ? part[(int64_t)b * kHB + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) P[t + 256 * u] = v[u];
    __syncthreads();
    if (t < nc) {
      const int nbt = min(kPFTile, nb - b0);
      for (int b = 0; b < nbt; ++b) s += P[b * kHB + t];
    }
    __syncthreads();
  }
  if (t < nc) T[t] = s;
  __syncthreads();
  if (t == 0) {
    const double x0 = X[(int64_t)j * ld + j], xn2 = T[0];
    double scale = 0.0, beta = x0, tj = 0.0;
    if (xn2 != 0.0) {
      beta = -copysign(sqrt(x0 * x0 + xn2), x0);
      scale = 1.0 / (x0 - beta);
      tj = (beta - x0) / beta;
    }
    tau[j] = tj;
    sh[0] = scale;
    sh[1] = tj;
    coef[0] = scale;
    coef[1] = beta;
  }
  __syncthreads();
  if (t >= 1 && t < nc) coef[2 + t] = sh[1] * (X[(int64_t)(j + t) * ld + j] + sh[0] * T[t]);
}

__global__ __launch_bounds__(256) void k_pf_update(double *__restrict__ X, int64_t ld, int rows, int j, int jend,
                                                    const double *__restrict__ coef) {
  const int nc = jend - j;
  const double scale = coef[0], beta = coef[1];
  const int64_t r = (int64_t)j + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  double v;
  if (r == j) {
    v = 1.0;
    X[(int64_t)j * ld + j] = beta;
  } else {
    v = X[(int64_t)j * ld + r] * scale;
    X[(int64_t)j * ld + r] = v;
  }
  // the row's entries of columns j+1 .. jend-1 are loaded before the first store
  double xv[kHB];
#pragma unroll
  for (int c = 1; c < kHB; ++c) xv[c] = c < nc ? X[(int64_t)(j + c) * ld + r] : 0.0;
#pragma unroll
  for (int c = 1; c < kHB; ++c)
    if (c < nc) X[(int64_t)(j + c) * ld + r] = xv[c] - coef[2 + c] * v;
}

static hipError_t panel_factor(double *X, int64_t ld, int rows, int j0, int jend, double *tau, double *part,
                               double *coef, hipStream_t st) {
  for (int j = j0; j < jend; ++j) {
    const int64_t below = (int64_t)rows - j - 1;
    const int nb = (int)std::max<int64_t>(1, (below + kPFRows - 1) / kPFRows);
    hipLaunchKernelGGL(k_pf_dots, dim3(nb), dim3(256), 0, st, X, ld, rows, j, jend, part);
    hipLaunchKernelGGL(k_pf_coef, dim3(1), dim3(256), 0, st, part, nb, X, ld, j, jend, tau, coef);
    const int nu = (int)((rows - j + 255) / 256);
    hipLaunchKernelGGL(k_pf_update, dim3(nu), dim3(256), 0, st, X, ld, rows, j, jend, coef);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t hh_blocked_ws_doubles(int cols) {
  const int p2 = std::max(cols, kHB);
  return (size_t)kTGMaxVB * kHB * p2 + (size_t)kHB * p2 + (size_t)kHB * kHB +
         (size_t)((cols + kHB - 1) / kHB) * kHB * kHB;
}

static int tg_nvb(int64_t rows_from) {
  const int64_t nch = (rows_from + kTGChunk - 1) / kTGChunk;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nch, kTGMaxVB));
}

// W (kHB x p2, row-major) = V^T C over rows [j0, rows)
static hipError_t tall_vtc(const double *X, int64_t ld, int j0, int jb, int64_t rows, const double *C, int64_t ldc,
                           int cv, int p2, double *part, double *W, hipStream_t st) {
  const int nvb = tg_nvb(rows - j0);
  hipLaunchKernelGGL(k_tg_part, dim3(nvb, (p2 + 63) / 64), dim3(256), 0, st, X, ld, j0, jb, rows, C, ldc, cv, p2, nvb,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int total = kHB * p2;
  hipLaunchKernelGGL(k_tg_reduce, dim3((total + 31) / 32), dim3(256), 0, st, part, nvb, total, W);
  return hipGetLastError();
}

hipError_t hh_qr_blocked(double *X, int64_t ld, int rows, int cols, double *tau, double *ws, hipStream_t st) {
  const int p2max = std::max(cols, kHB);
  double *part = ws, *W = part + (size_t)kTGMaxVB * kHB * p2max, *G = W + (size_t)kHB * p2max;
  double *Tall = G + (size_t)kHB * kHB;
  hipError_t e;
  for (int j0 = 0; j0 < cols; j0 += kHB) {
    const int jb = std::min(kHB, cols - j0);
    // partial sums of the panel kernels reuse the head of part (before use
    // by the tall products of this panel)
    if ((e = panel_factor(X, ld, rows, j0, j0 + jb, tau, part, W, st)) != hipSuccess) return e;
    double *T = Tall + (size_t)(j0 / kHB) * kHB * kHB;
    if ((e = tall_vtc(X, ld, j0, jb, rows, nullptr, 0, 1, kHB, part, G, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tmat, dim3(1), dim3(256), 0, st, G, tau, j0, jb, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int c0 = j0 + jb, p2 = cols - c0;
    if (p2 <= 0) continue;
    double *C = X + (int64_t)c0 * ld;
    if ((e = tall_vtc(X, ld, j0, jb, rows, C, ld, 0, p2, part, W, st)) != hipSuccess) return e;
    // part is free again after the reduction into W: it holds T^T W
    hipLaunchKernelGGL(k_tw, dim3((unsigned)(((int64_t)kHB * p2 + 255) / 256)), dim3(256), 0, st, T, 1, W, p2, part);
    const dim3 g((unsigned)((rows - j0 + 63) / 64), (unsigned)((p2 + 63) / 64));
    hipLaunchKernelGGL(k_tu, g, dim3(256), 0, st, X, ld, j0, jb, (int64_t)rows, part, p2, C, ld);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t hh_apply_blocked(const double *X, int64_t ld, int rows, int nref, const double *ws, double *Z,
                            int64_t ldz, int ncols, double *ws_rw, hipStream_t st) {
  // Z <- Q Z, Q = H_0 ... H_{nref-1}: panels from the last to the first
  const int p2max = std::max(ncols, kHB);
  double *part = ws_rw, *W = part + (size_t)kTGMaxVB * kHB * p2max;
  const int pcols = std::max(nref, kHB);
  const double *Tall = ws + (size_t)kTGMaxVB * kHB * pcols + (size_t)kHB * pcols + (size_t)kHB * kHB;
  hipError_t e;
  if (ncols <= 0) return hipSuccess;
  const int np = (nref + kHB - 1) / kHB;
  for (int pi = np - 1; pi >= 0; --pi) {
    const int j0 = pi * kHB, jb = std::min(kHB, nref - j0);
    const double *T = Tall + (size_t)pi * kHB * kHB;
    if ((e = tall_vtc(X, ld, j0, jb, rows, Z, ldz, 0, ncols, part, W, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tw, dim3((unsigned)(((int64_t)kHB * ncols + 255) / 256)), dim3(256), 0, st, T, 0, W, ncols,
                       part);
    const dim3 g((unsigned)((rows - j0 + 63) / 64), (unsigned)((ncols + 63) / 64));
    hipLaunchKernelGGL(k_tu, g, dim3(256), 0, st, X, ld, j0, jb, (int64_t)rows, part, ncols, Z, ldz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// TA: A is given transposed in memory (element (r, k) at A[r * lda + k]).
template <bool TA>
__global__ __launch_bounds__(256) void k_gemm_mfma(int R, int N, int K, double alpha, const double *__restrict__ A,
                                                   int64_t lda, const double *__restrict__ B, int64_t ldb,
                                                   double beta, double *__restrict__ C, int64_t ldc) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = t; e < 1024; e += 256) {
      if (TA) {
        const int kk = e & 15, i = e >> 4;
        const int gr = row0 + i, gk = k0 + kk;
        As[kk][i] = (gr < R && gk < K) ? A[(int64_t)gr * lda + gk] : 0.0;
      } else {
        const int i = e & 63, kk = e >> 6;
        const int gr = row0 + i, gk = k0 + kk;
        As[kk][i] = (gr < R && gk < K) ? A[(int64_t)gk * lda + gr] : 0.0;
      }
      const int kb = e & 15, jb = e >> 4;
      const int gc = col0 + jb, gk2 = k0 + kb;
      Bs[kb][jb] = (gc < N && gk2 < K) ? B[(int64_t)gc * ldb + gk2] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int ka = kk + (lane >> 4);
      const double a0 = As[ka][wr + (lane & 15)];
      const double a1 = As[ka][wr + 16 + (lane & 15)];
      const double b0 = Bs[ka][wc + (lane & 15)];
      const double b1 = Bs[ka][wc + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) {
        const int gr = row0 + wr + a * 16 + (lane >> 4) + 4 * v;
        const int gc = col0 + wc + b * 16 + (lane & 15);
        if (gr < R && gc < N) {
          double *cp = C + (int64_t)gc * ldc + gr;
          const double prev = (beta != 0.0) ? beta * (*cp) : 0.0;
          *cp = alpha * acc[a][b][v] + prev;
        }
      }
}

hipError_t launch_gemm(int R, int N, int K, double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                       double beta, double *C, int64_t ldc, hipStream_t st) {
  if (R <= 0 || N <= 0) return hipSuccess;
  dim3 g((R + 63) / 64, (N + 63) / 64);
  hipLaunchKernelGGL(k_gemm_mfma<false>, g, dim3(256), 0, st, R, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  return hipGetLastError();
}

hipError_t launch_gemm_ta(int R, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                          int64_t ldb, double beta, double *C, int64_t ldc, hipStream_t st) {
  if (R <= 0 || N <= 0) return hipSuccess;
  dim3 g((R + 63) / 64, (N + 63) / 64);
  hipLaunchKernelGGL(k_gemm_mfma<true>, g, dim3(256), 0, st, R, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  return hipGetLastError();
}

}  // namespace csvd
