// Sparse kernels for gfx950: CSR transpose, generic CSR x dense products,
// layout transposes and CSR validation.
//
// Layout conventions: "row-major block" = rows x k doubles with the k
// entries of a row contiguous (what a CSR gather wants: one row of the
// operand is one coalesced segment); "column-major" = Fortran order with a
// leading dimension.
#include "csvd_impl.h"

namespace csvd {

// ---------------------------------------------------------------- transpose
// Builds CSR(A^T) from CSR(A).  Histogram of column indices, exclusive scan,
// scatter with per-column cursors, then each column segment is sorted by row
// index, so the result is unique and independent of atomic ordering.

__global__ void k_col_hist(int nnz, const int *__restrict__ ci, int *__restrict__ cnt) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[ci[k]], 1);
}

// Exclusive scan of cnt[0..len) into out[0..len] (out[len] = total) with a
// single block of 1024 threads; each thread owns a contiguous chunk.
__global__ __launch_bounds__(1024) void k_scan_single(int len, const int *__restrict__ cnt, int *__restrict__ out) {
  __shared__ long long part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (len + 1023) / 1024;
  const int64_t b = t * chunk;
  const int64_t e = (b + chunk < len) ? b + chunk : len;
  long long s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    long long v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  long long run = (t == 0) ? 0 : part[t - 1];
  for (int64_t i = b; i < e; ++i) {
    out[i] = (int)run;
    run += cnt[i];
  }
  if (t == 1023) out[len] = (int)part[1023];
}

__global__ void k_scatter_T(int m, const int *__restrict__ rp, const int *__restrict__ ci,
                            const double *__restrict__ va, int *__restrict__ cursor, int *__restrict__ ciT,
                            double *__restrict__ vaT) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      int pos = atomicAdd(&cursor[ci[k]], 1);
      ciT[pos] = (int)i;
      vaT[pos] = va[k];
    }
  }
}

// Insertion sort of each column segment by row index (segments are short for
// sparse matrices; dense-ish columns cost O(len^2) once at create time).
__global__ void k_sort_segments(int n, const int *__restrict__ rpT, int *__restrict__ ciT, double *__restrict__ vaT) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const int b = rpT[j], e = rpT[j + 1];
    for (int k = b + 1; k < e; ++k) {
      int key = ciT[k];
      double val = vaT[k];
      int q = k - 1;
      while (q >= b && ciT[q] > key) {
        ciT[q + 1] = ciT[q];
        vaT[q + 1] = vaT[q];
        --q;
      }
      ciT[q + 1] = key;
      vaT[q + 1] = val;
    }
  }
}

static int grid_for(int64_t work, int per_block = kThreads, int cap = 8192) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// work: n + 1 ints (cursor) of scratch.
hipError_t launch_csr_transpose(int m, int n, int nnz, const int *rp, const int *ci, const double *va,
                                int *rpT, int *ciT, double *vaT, int *work, hipStream_t st) {
  hipError_t e = hipMemsetAsync(work, 0, sizeof(int) * (size_t)(n + 1), st);
  if (e != hipSuccess) return e;
  if (nnz > 0) hipLaunchKernelGGL(k_col_hist, dim3(grid_for(nnz)), dim3(kThreads), 0, st, nnz, ci, work);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, n, work, rpT);
  e = hipMemcpyAsync(work, rpT, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_scatter_T, dim3(grid_for(m)), dim3(kThreads), 0, st, m, rp, ci, va, work, ciT, vaT);
    hipLaunchKernelGGL(k_sort_segments, dim3(grid_for(n)), dim3(kThreads), 0, st, n, rpT, ciT, vaT);
  }
  return hipGetLastError();
}

// ------------------------------------------------------- generic products
// y (rows x k, row-major) = A (CSR, rows) * x (row-major, k columns).  One
// thread per output element; threads of the same row read the same (col,
// val) pair (a broadcast) and consecutive x entries (a coalesced segment).
__global__ void k_spmm_rowmajor(int rows, int64_t k, const int *__restrict__ rp, const int *__restrict__ ci,
                                const double *__restrict__ va, const double *__restrict__ x,
                                double *__restrict__ y) {
  const int64_t total = (int64_t)rows * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;
    const int64_t c = e - i * k;
    double acc = 0.0;
    const int b = rp[i], en = rp[i + 1];
    for (int q = b; q < en; ++q) acc = fma(va[q], x[(int64_t)ci[q] * k + c], acc);
    y[e] = acc;
  }
}

// y = M x for one column (k = 1): one wave per row, the lanes take the
// nonzeros p = lane, lane + 64, ... of the row and their partial sums are
// added in a fixed butterfly order, so a row of tens of thousands of
// nonzeros is spread over a wave instead of one thread.
__global__ __launch_bounds__(kThreads) void k_spmv_wave(int rows, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, const double *__restrict__ va,
                                                        const double *__restrict__ x, double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t nwave = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t row = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); row < rows; row += nwave) {
    double acc = 0.0;
    const int e = rp[row + 1];
    for (int p = rp[row] + lane; p < e; p += 64) acc = fma(va[p], x[ci[p]], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) y[row] = acc;
  }
}

hipError_t launch_spmm_rowmajor(int rows, int64_t k, const int *rp, const int *ci, const double *va,
                                const double *x, double *y, hipStream_t st) {
  if (rows <= 0 || k <= 0) return hipSuccess;
  if (k == 1) {
    hipLaunchKernelGGL(k_spmv_wave, dim3(grid_for(rows, kThreads / 64, 16384)), dim3(kThreads), 0, st, rows, rp, ci,
                       va, x, y);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_spmm_rowmajor, dim3(grid_for((int64_t)rows * k, kThreads, 65536)), dim3(kThreads), 0, st,
                     rows, k, rp, ci, va, x, y);
  return hipGetLastError();
}

// ------------------------------------------------------------ transposes
// 32 x 32 tiles through LDS (+1 padding against bank conflicts).
__global__ void k_col_to_row(int rows, int cols, const double *__restrict__ src, int64_t ld,
                             double *__restrict__ dst, int64_t dst_cols) {
  __shared__ double tile[32][33];
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows of 32
  for (int j = ty; j < 32; j += 8) {
    int r = r0 + tx, c = c0 + j;
    tile[j][tx] = (r < rows && c < cols) ? src[(int64_t)c * ld + r] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    int r = r0 + j, c = c0 + tx;
    if (r < rows && c < dst_cols) dst[(int64_t)r * dst_cols + c] = (c < cols) ? tile[tx][j] : 0.0;
  }
}

__global__ void k_row_to_col(int rows, int cols, const double *__restrict__ src, int64_t src_cols,
                             double *__restrict__ dst, int64_t ld) {
  __shared__ double tile[32][33];
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    int r = r0 + j, c = c0 + tx;
    tile[j][tx] = (r < rows && c < cols) ? src[(int64_t)r * src_cols + c] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    int r = r0 + tx, c = c0 + j;
    if (r < rows && c < cols) dst[(int64_t)c * ld + r] = tile[tx][j];
  }
}

// dst (rows x dst_cols row-major) <- src (rows x cols column-major, ld);
// columns cols..dst_cols-1 are zero-filled.
hipError_t launch_col_to_row(int rows, int cols, const double *src, int64_t ld, double *dst, int64_t dst_cols,
                             hipStream_t st) {
  if (rows <= 0 || dst_cols <= 0) return hipSuccess;
  dim3 g((rows + 31) / 32, (int)((dst_cols + 31) / 32));
  hipLaunchKernelGGL(k_col_to_row, g, dim3(256), 0, st, rows, cols, src, ld, dst, dst_cols);
  return hipGetLastError();
}

hipError_t launch_row_to_col(int rows, int cols, const double *src, int64_t src_cols, double *dst, int64_t ld,
                             hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 g((rows + 31) / 32, (cols + 31) / 32);
  hipLaunchKernelGGL(k_row_to_col, g, dim3(256), 0, st, rows, cols, src, src_cols, dst, ld);
  return hipGetLastError();
}

// ------------------------------------------------------------ validation
// flags[0]: bad rowptr (non-monotone or wrong ends); flags[1]: column out of
// range or not strictly increasing in its row; flags[2]: non-finite value.
__global__ void k_check_csr(int m, int n, const int *__restrict__ rp, const int *__restrict__ ci,
                            const double *__restrict__ va, int nnz, int *__restrict__ flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int b = rp[i], e = rp[i + 1];
    if (e < b || b < 0 || e > nnz || (i == 0 && b != 0) || (i == m - 1 && e != nnz)) {
      atomicOr(&flags[0], 1);
      continue;
    }
    for (int k = b; k < e; ++k) {
      int c = ci[k];
      if (c < 0 || c >= n || (k > b && c <= ci[k - 1])) atomicOr(&flags[1], 1);
      double v = va[k];
      if (!(v - v == 0.0)) atomicOr(&flags[2], 1);
    }
  }
}

hipError_t launch_check_csr(int m, int n, const int *rp, const int *ci, const double *va, int nnz, int *flags,
                            hipStream_t st) {
  hipError_t e = hipMemsetAsync(flags, 0, 3 * sizeof(int), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_csr, dim3(grid_for(m)), dim3(kThreads), 0, st, m, n, rp, ci, va, nnz, flags);
  return hipGetLastError();
}

}  // namespace csvd
