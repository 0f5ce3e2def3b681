// Sparse products of the block Lanczos step (operator apply, Algorithm 1
// step 1): U = A Q_k and W = A^T U on row-major n x Lp blocks, CSR FP64.
//
// Rows with few nonzeros (G = 1): Lp/4 lanes share a row, four columns each
// (two 16-byte loads per gathered row), so a wave works on 256/Lp rows at
// once, and four nonzeros of a row are gathered before their products are
// added in order.  Long rows: a tile of rows is spread over the 256 threads
// as (row, lane group, column), the Lp threads of a row read one 8*Lp-byte
// row of the gathered block per nonzero, and G lane groups split the
// nonzeros of the row; their partial sums are added in a fixed order through
// LDS.  Both add each row's products in the order of its nonzeros.
#include "csvd_impl.h"

namespace csvd {

typedef double v2d __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int bfind_sp(const int *__restrict__ toff, int njob, int g) {
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (toff[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static int bgrid_sp(int total, int cap) { return total < 1 ? 1 : (total < cap ? total : cap); }

// ------------------------------------------------------ sparse products
// y = M x for the rows of one tile; slot layout ((row * G) + g) * Lp + col as
// in the single-vector kernels (G lane groups split each row's nonzeros).
__device__ __forceinline__ void tile_spmm(const GLB int *__restrict__ rp, const GLB int *__restrict__ ci,
                                          const GLB double *__restrict__ va, const GLB double *__restrict__ x,
                                          GLB double *__restrict__ y, int64_t nrows, int tile, int rpt, int lg,
                                          int G, int lgG, int E, int tlong, double *gsum) {
  const int t = threadIdx.x;
  const int Lp = 1 << lg;
  const int col = t & (Lp - 1);
  const int gi = (t >> lg) & (G - 1);
  for (int q = 0; q < E; ++q) {
    const int rloc = (q * kThreads + t) >> (lg + lgG);
    const int64_t row = (int64_t)tile * rpt + rloc;
    double acc = 0.0;
    bool own = false;  // a row this tile writes (long rows are summed from their segments)
    if (row < nrows) {
      const int b = rp[row], en = rp[row + 1];
      own = en - b <= tlong;
      if (own) {
#pragma unroll 4
        for (int p = b + gi; p < en; p += G) acc = fma(va[p], x[((int64_t)ci[p] << lg) + col], acc);
      }
    }
    if (G > 1) {
      gsum[t] = acc;
      __syncthreads();
      if (gi == 0)
        for (int h = 1; h < G; ++h) acc += gsum[t + (h << lg)];
      __syncthreads();
    }
    if (gi == 0 && own) y[(row << lg) + col] = acc;
  }
}

// y = M x for one tile of kThreads / (LP / 4) rows (G = 1)
template <int LP>
__device__ __forceinline__ void tile_rows4(const GLB int *__restrict__ rp, const GLB int *__restrict__ ci,
                                           const GLB double *__restrict__ va, const GLB double *__restrict__ x,
                                           GLB double *__restrict__ y, int64_t nrows, int tile, int tlong) {
  constexpr int LPR = LP / 4, RPT = kThreads / LPR, UNR = 4;
  const int t = threadIdx.x, c0 = (t % LPR) * 4;
  const int64_t row = (int64_t)tile * RPT + t / LPR;
  if (row < nrows && rp[row + 1] - rp[row] <= tlong) {  // long rows: from their segments
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int e = rp[row + 1];
    int p = rp[row];
    for (; p + UNR <= e; p += UNR) {
      int c[UNR];
      double v[UNR];
      v2d xv[UNR][2];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        c[u] = ci[p + u];
        v[u] = va[p + u];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const GLB v2d *xp = reinterpret_cast<const GLB v2d *>(x + (int64_t)c[u] * LP + c0);
        xv[u][0] = xp[0];
        xv[u][1] = xp[1];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        acc[0] = fma(v[u], xv[u][0].x, acc[0]);
        acc[1] = fma(v[u], xv[u][0].y, acc[1]);
        acc[2] = fma(v[u], xv[u][1].x, acc[2]);
        acc[3] = fma(v[u], xv[u][1].y, acc[3]);
      }
    }
    for (; p < e; ++p) {
      const double v = va[p];
      const GLB v2d *xp = reinterpret_cast<const GLB v2d *>(x + (int64_t)ci[p] * LP + c0);
      const v2d x0 = xp[0], x1 = xp[1];
      acc[0] = fma(v, x0.x, acc[0]);
      acc[1] = fma(v, x0.y, acc[1]);
      acc[2] = fma(v, x1.x, acc[2]);
      acc[3] = fma(v, x1.y, acc[3]);
    }
    GLB v2d *yp = reinterpret_cast<GLB v2d *>(y + row * LP + c0);
    yp[0] = v2d{acc[0], acc[1]};
    yp[1] = v2d{acc[2], acc[3]};
  }
}

__device__ __forceinline__ void tile_any(const GLB int *__restrict__ rp, const GLB int *__restrict__ ci,
                                         const GLB double *__restrict__ va, const GLB double *__restrict__ x,
                                         GLB double *__restrict__ y, int64_t nrows, int tile, int rpt, int lg, int G,
                                         int lgG, int E, int tlong, double *gsum) {
  if (G == 1) {
    switch (lg) {
      case 4: tile_rows4<16>(rp, ci, va, x, y, nrows, tile, tlong); return;
      case 5: tile_rows4<32>(rp, ci, va, x, y, nrows, tile, tlong); return;
      default: tile_rows4<64>(rp, ci, va, x, y, nrows, tile, tlong); return;
    }
  }
  tile_spmm(rp, ci, va, x, y, nrows, tile, rpt, lg, G, lgG, E, tlong, gsum);
}

__global__ __launch_bounds__(kThreads) void b_spmm_a(const BJobDesc *__restrict__ jobs, int njob,
                                                     const int *__restrict__ toff, int total,
                                                     StepClock clock) {
  __shared__ double gsum[kThreads];
  const int64_t ck = sclock(clock);
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int j = bfind_sp(toff, njob, g);
    const BJobDesc &J = jobs[j];
    const int k = (int)(ck - J.start_clock);
    if (k >= J.Kstop) continue;
    const int64_t nL = (int64_t)J.n * J.Lp;
    tile_any(gp(J.rp), gp(J.ci), gp(J.va), qblock(J, k), gp(J.U), J.m, g - toff[j], J.rpt1, J.lgLp, J.G1,
             J.lgG1, J.E1, J.tlong, gsum);
  }
}

__global__ __launch_bounds__(kThreads) void b_spmm_at(const BJobDesc *__restrict__ jobs, int njob,
                                                      const int *__restrict__ toff, int total,
                                                      StepClock clock) {
  __shared__ double gsum[kThreads];
  const int64_t ck = sclock(clock);
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int j = bfind_sp(toff, njob, g);
    const BJobDesc &J = jobs[j];
    if ((int)(ck - J.start_clock) >= J.Kstop) continue;
    tile_any(gp(J.rpT), gp(J.ciT), gp(J.vaT), gp(J.U), gp(J.W), J.n, g - toff[j], J.rpt2, J.lgLp, J.G2, J.lgG2,
             J.E2, J.tlong, gsum);
  }
}

hipError_t launch_b_spmm_a(const BBatch &b, hipStream_t st) {
  hipLaunchKernelGGL(b_spmm_a, dim3(bgrid_sp(b.total1, 4096)), dim3(kThreads), 0, st, b.jobs, b.njob, b.toff1, b.total1,
                     step_clock(b));
  return hipGetLastError();
}

hipError_t launch_b_spmm_at(const BBatch &b, hipStream_t st) {
  hipLaunchKernelGGL(b_spmm_at, dim3(bgrid_sp(b.total2, 4096)), dim3(kThreads), 0, st, b.jobs, b.njob, b.toff2, b.total2,
                     step_clock(b));
  return hipGetLastError();
}

// ---------------------------------------------------------- long rows
// Segment s of a long row: partial row sum_{p in [sgb_s, sge_s)} va_p x(ci_p)
// into sgp(s, :), with the lane layout of tile_rows4 (one segment per Lp/4
// lanes, four columns per lane, the products added in nonzero order).
template <int LP>
__global__ __launch_bounds__(kThreads) void b_spmm_seg(BJobDesc J, int side, int k) {
  constexpr int LPR = LP / 4, RPT = kThreads / LPR, UNR = 4;
  const GLB int *__restrict__ ci = gp(side == 1 ? J.ci : J.ciT);
  const GLB double *__restrict__ va = gp(side == 1 ? J.va : J.vaT);
  const GLB double *__restrict__ x = side == 1 ? qblock(J, k) : gp(J.U);
  const GLB int *__restrict__ sb = gp(side == 1 ? J.sgb1 : J.sgb2);
  const GLB int *__restrict__ se = gp(side == 1 ? J.sge1 : J.sge2);
  GLB double *__restrict__ part = gp(side == 1 ? J.sgp1 : J.sgp2);
  const int nseg = side == 1 ? J.nseg1 : J.nseg2;
  const int t = threadIdx.x, c0 = (t % LPR) * 4;
  for (int64_t tile = blockIdx.x; tile * RPT < nseg; tile += gridDim.x) {
    const int64_t s = tile * RPT + t / LPR;
    if (s >= nseg) continue;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int e = se[s];
    int p = sb[s];
    for (; p + UNR <= e; p += UNR) {
      int c[UNR];
      double v[UNR];
      v2d xv[UNR][2];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        c[u] = ci[p + u];
        v[u] = va[p + u];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const GLB v2d *xp = reinterpret_cast<const GLB v2d *>(x + (int64_t)c[u] * LP + c0);
        xv[u][0] = xp[0];
        xv[u][1] = xp[1];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        acc[0] = fma(v[u], xv[u][0].x, acc[0]);
        acc[1] = fma(v[u], xv[u][0].y, acc[1]);
        acc[2] = fma(v[u], xv[u][1].x, acc[2]);
        acc[3] = fma(v[u], xv[u][1].y, acc[3]);
      }
    }
    for (; p < e; ++p) {
      const double v = va[p];
      const GLB v2d *xp = reinterpret_cast<const GLB v2d *>(x + (int64_t)ci[p] * LP + c0);
      const v2d x0 = xp[0], x1 = xp[1];
      acc[0] = fma(v, x0.x, acc[0]);
      acc[1] = fma(v, x0.y, acc[1]);
      acc[2] = fma(v, x1.x, acc[2]);
      acc[3] = fma(v, x1.y, acc[3]);
    }
    GLB v2d *yp = reinterpret_cast<GLB v2d *>(part + s * LP + c0);
    yp[0] = v2d{acc[0], acc[1]};
    yp[1] = v2d{acc[2], acc[3]};
  }
}

// Long row r: y(lrow_r, :) = sum of its segments' partial rows, in order.
__global__ __launch_bounds__(kThreads) void b_spmm_comb(BJobDesc J, int side) {
  const GLB int *__restrict__ lrow = gp(side == 1 ? J.lrow1 : J.lrow2);
  const GLB int *__restrict__ lseg = gp(side == 1 ? J.lseg1 : J.lseg2);
  const GLB double *__restrict__ part = gp(side == 1 ? J.sgp1 : J.sgp2);
  GLB double *__restrict__ y = gp(side == 1 ? J.U : J.W);
  const int nlong = side == 1 ? J.nlong1 : J.nlong2;
  const int Lp = J.Lp;
  const int64_t total = (int64_t)nlong * Lp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / Lp;
    const int c = (int)(e - r * Lp);
    double acc = 0.0;
    for (int s = lseg[r]; s < lseg[r + 1]; ++s) acc += part[(int64_t)s * Lp + c];
    y[(int64_t)lrow[r] * Lp + c] = acc;
  }
}

hipError_t launch_b_spmm_long(const BJobDesc &hj, int side, int k, hipStream_t st) {
  const int nseg = side == 1 ? hj.nseg1 : hj.nseg2, nlong = side == 1 ? hj.nlong1 : hj.nlong2;
  if (nseg == 0) return hipSuccess;
  const int rpt = kThreads * 4 / hj.Lp;
  const int gs = bgrid_sp((nseg + rpt - 1) / rpt, 8192);
  switch (hj.Lp) {
    case 16: hipLaunchKernelGGL(b_spmm_seg<16>, dim3(gs), dim3(kThreads), 0, st, hj, side, k); break;
    case 32: hipLaunchKernelGGL(b_spmm_seg<32>, dim3(gs), dim3(kThreads), 0, st, hj, side, k); break;
    default: hipLaunchKernelGGL(b_spmm_seg<64>, dim3(gs), dim3(kThreads), 0, st, hj, side, k); break;
  }
  const int gc = bgrid_sp((int)(((int64_t)nlong * hj.Lp + kThreads - 1) / kThreads), 8192);
  hipLaunchKernelGGL(b_spmm_comb, dim3(gc), dim3(kThreads), 0, st, hj, side);
  return hipGetLastError();
}

}  // namespace csvd
