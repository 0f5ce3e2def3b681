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

__device__ __forceinline__ double block_reduce(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  const double r = red[0];
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
// Round-robin pairing over n (even) columns: index n-1 stays, the others
// rotate; step s pairs (n-1, s) and ((s+b) mod (n-1), (s-b) mod (n-1)).
__global__ __launch_bounds__(kThreads) void k_jacobi(double *A, int64_t lda, int rows, int ncol, double *V,
                                                     int64_t ldv, int vrows, int step, double tol, int *counter) {
  __shared__ double r0[kThreads], r1[kThreads], r2[kThreads];
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
  r0[t] = spp;
  r1[t] = sqq;
  r2[t] = spq;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      r0[t] += r0[t + off];
      r1[t] += r1[t + off];
      r2[t] += r2[t + off];
    }
    __syncthreads();
  }
  const double app = r0[0], aqq = r1[0], apq = r2[0];
  if (apq == 0.0 || !(fabs(apq) > tol * sqrt(app * aqq))) return;
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
                              int step, double tol, int *counter, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi, dim3(cols_even / 2), dim3(kThreads), 0, st, A, lda, rows, cols_even, V, ldv, vrows,
                     step, tol, counter);
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
