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
// the moment coefficients F_k = sum_s 2 Re(c_sk Y_{s,k}) are formed, and
// S += Q_k F_k is accumulated from the stored basis, or from a second pass
// that regenerates Q_k bit for bit.
#include <algorithm>

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


// ------------------------------------------------------ per-shift block LU
// One workgroup per (job, shift).  The four products of a step run on FP64
// MFMA (16x16x4) with operands staged in LDS; each wave owns a 16-row band
// of the Lp x Lp result in the MFMA output layout: lane l holds rows
// 16 w + l/16 + 4 v (v < 4) of the 16-column tiles tj, column 16 tj + l%16.
// H_k is inverted in that register layout by Gauss-Jordan elimination
// without pivoting (Im H_k is positive definite); the pivot row and column
// of each elimination step are broadcast through double-buffered LDS, one
// barrier per step.  All Lp columns of Z are carried (the first L are the
// right-hand sides).
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma4b(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// element v of a v4d / tile tj of a 4-tile array with runtime indexes
// (select chains: no scratch, no code growth)
__device__ __forceinline__ double pick4b(const v4d &x, int v) {
  return v == 0 ? x[0] : (v == 1 ? x[1] : (v == 2 ? x[2] : x[3]));
}
__device__ __forceinline__ double pick_tile(const v4d (&x)[4], int tj, int v) {
  return tj == 0 ? x[0][v] : (tj == 1 ? x[1][v] : (tj == 2 ? x[2][v] : x[3][v]));
}

template <int LP>
__global__ __launch_bounds__(kThreads) void b_shift(const BJobDesc *__restrict__ jobs, int njob,
                                                    const int *__restrict__ toffs, int64_t clock,
                                                    int init) {
  constexpr int NT = LP / 16, KS = LP / 4, L2 = LP * LP, SS = LP + 1;
  __shared__ double LB[LP * SS];
  __shared__ double Pr[LP * SS], Pi[LP * SS];
  __shared__ double2 rowb[2][LP], colb[2][LP];
  __shared__ double rsum[4][LP];
  const int g = blockIdx.x;
  const int j = bfind(toffs, njob, g);
  const BJobDesc &J = jobs[j];
  if (J.Lp != LP) return;
  const int s = g - toffs[j];
  const int L = J.L;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const int k = (int)(clock - J.start_clock);
  if (k >= J.Kstop) return;
  const int64_t hbase = (int64_t)s * (J.Kcap + 1) * L2;
  GLB double2 *__restrict__ Hinv = gp(J.Hinv) + hbase;
  GLB double2 *__restrict__ Zh = gp(J.Zh) + hbase;
  if (init) {
    for (int e = t; e < L2; e += kThreads) Zh[e] = make_double2(gp(J.Bh)[e], 0.0);  // Z_0 = R_0
    return;
  }
  const bool act = w < NT;
  const double2 z = gp(J.shift)[s];
  const GLB double *__restrict__ Ak = gp(J.Ah) + (int64_t)k * L2;
  const GLB double *__restrict__ Bk = gp(J.Bh) + (int64_t)k * L2;
  const GLB double *__restrict__ Bk1 = gp(J.Bh) + (int64_t)(k + 1) * L2;
  // ---- stage B_k and H_{k-1}^{-1}
  constexpr int IT = (L2 + kThreads - 1) / kThreads;
  {
    double bv[IT];
    double2 hv[IT];
    const GLB double2 *__restrict__ Hp = Hinv + (int64_t)(k > 0 ? k - 1 : 0) * L2;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      bv[it] = (e < L2) ? Bk[e] : 0.0;
      hv[it] = make_double2(0.0, 0.0);
      if (e < L2 && k > 0) {
        const double2 h = Hp[e];
        hv[it] = h;
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      if (e < L2) {
        LB[(e / LP) * SS + (e % LP)] = bv[it];
        Pr[(e / LP) * SS + (e % LP)] = hv[it].x;
        Pi[(e / LP) * SS + (e % LP)] = hv[it].y;
      }
    }
  }
  __syncthreads();
  v4d Dr[4], Di[4];
  // ---- T1 = H_{k-1}^{-1} B_k^T
  if (k > 0 && act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) Dr[tj] = Di[tj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + q;
      const double ar = Pr[(16 * w + rl) * SS + c], ai = Pi[(16 * w + rl) * SS + c];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const double b = LB[(16 * tj + rl) * SS + c];  // (B^T)(c, 16 tj + rl)
        Dr[tj] = mfma4b(ar, b, Dr[tj]);
        Di[tj] = mfma4b(ai, b, Di[tj]);
      }
    }
  }
  __syncthreads();
  if (k > 0 && act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + q + 4 * v, jj = 16 * tj + rl;
        Pr[i * SS + jj] = Dr[tj][v];
        Pi[i * SS + jj] = Di[tj][v];
      }
  }
  __syncthreads();
  // ---- H = z I - A_k - B_k T1
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + q + 4 * v, jj = 16 * tj + rl;
        Dr[tj][v] = (i == jj ? z.x : 0.0) - Ak[i * LP + jj];
        Di[tj][v] = (i == jj ? z.y : 0.0);
      }
    if (k > 0) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int c = 4 * ks + q;
        const double a = -LB[(16 * w + rl) * SS + c];
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          Dr[tj] = mfma4b(a, Pr[c * SS + 16 * tj + rl], Dr[tj]);
          Di[tj] = mfma4b(a, Pi[c * SS + 16 * tj + rl], Di[tj]);
        }
      }
    }
    // pivot row and column 0
    if (w == 0 && q == 0)
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) rowb[0][16 * tj + rl] = make_double2(Dr[tj][0], Di[tj][0]);
    if (rl == 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) colb[0][16 * w + q + 4 * v] = make_double2(Dr[0][v], Di[0][v]);
  }
  __syncthreads();
  // ---- Gauss-Jordan inverse in registers
#pragma unroll 1
  for (int c = 0; c < LP; ++c) {
    const int cb = c & 1;
    const double2 p = colb[cb][c];
    const double den = p.x * p.x + p.y * p.y;
    const double2 inv = make_double2(p.x / den, -p.y / den);
    if (act) {
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const int jj = 16 * tj + rl;
        const double2 rj = rowb[cb][jj];
        const double2 gj = cmulb(rj, inv);  // scaled pivot row entry
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * w + q + 4 * v;
          const double2 f = colb[cb][i];
          double2 h = make_double2(Dr[tj][v], Di[tj][v]);
          if (i == c && jj == c) {
            h = inv;
          } else if (i == c) {
            h = gj;
          } else if (jj == c) {
            const double2 fi = cmulb(f, inv);
            h = make_double2(-fi.x, -fi.y);
          } else {
            const double2 d = cmulb(f, gj);
            h = make_double2(h.x - d.x, h.y - d.y);
          }
          Dr[tj][v] = h.x;
          Di[tj][v] = h.y;
        }
      }
      if (c + 1 < LP) {
        const int c1 = c + 1;
        const int vv = (c1 & 15) >> 2, tc = c1 >> 4;
        if (w == c1 / 16 && q == (c1 & 3))
#pragma unroll
          for (int tj = 0; tj < NT; ++tj)
            rowb[cb ^ 1][16 * tj + rl] = make_double2(pick4b(Dr[tj], vv), pick4b(Di[tj], vv));
        if (rl == (c1 & 15))
#pragma unroll
          for (int v = 0; v < 4; ++v)
            colb[cb ^ 1][16 * w + q + 4 * v] = make_double2(pick_tile(Dr, tc, v), pick_tile(Di, tc, v));
      }
    }
    __syncthreads();
  }
  // ---- store H_k^{-1}; stage it for the next product
  GLB double2 *__restrict__ Hk = Hinv + (int64_t)k * L2;
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + q + 4 * v, jj = 16 * tj + rl;
        Hk[i * LP + jj] = make_double2(Dr[tj][v], Di[tj][v]);
        Pr[i * SS + jj] = Dr[tj][v];
        Pi[i * SS + jj] = Di[tj][v];
      }
  }
  __syncthreads();
  // ---- T2 = H_k^{-1} Z_k
  const GLB double2 *__restrict__ Zk = Zh + (int64_t)k * L2;
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) Dr[tj] = Di[tj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + q;
      const double ar = Pr[(16 * w + rl) * SS + c], ai = Pi[(16 * w + rl) * SS + c];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const double2 zz = Zk[c * LP + 16 * tj + rl];
        Dr[tj] = mfma4b(ar, zz.x, Dr[tj]);
        Dr[tj] = mfma4b(-ai, zz.y, Dr[tj]);
        Di[tj] = mfma4b(ar, zz.y, Di[tj]);
        Di[tj] = mfma4b(ai, zz.x, Di[tj]);
      }
    }
  }
  __syncthreads();
  {
    double bv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      bv[it] = (e < L2) ? Bk1[e] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      if (e < L2) LB[(e / LP) * SS + (e % LP)] = bv[it];
    }
  }
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + q + 4 * v, jj = 16 * tj + rl;
        Pr[i * SS + jj] = Dr[tj][v];
        Pi[i * SS + jj] = Di[tj][v];
      }
  }
  __syncthreads();
  // ---- Z_{k+1} = B_{k+1} T2 and the residual norms of the first L columns
  GLB double2 *__restrict__ Zn = Zh + (int64_t)(k + 1) * L2;
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) Dr[tj] = Di[tj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + q;
      const double a = LB[(16 * w + rl) * SS + c];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        Dr[tj] = mfma4b(a, Pr[c * SS + 16 * tj + rl], Dr[tj]);
        Di[tj] = mfma4b(a, Pi[c * SS + 16 * tj + rl], Di[tj]);
      }
    }
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      double ss = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + q + 4 * v, jj = 16 * tj + rl;
        Zn[i * LP + jj] = make_double2(Dr[tj][v], Di[tj][v]);
        ss += Dr[tj][v] * Dr[tj][v] + Di[tj][v] * Di[tj][v];
      }
      ss += __shfl_xor(ss, 16);
      ss += __shfl_xor(ss, 32);
      if (q == 0) rsum[w][16 * tj + rl] = ss;
    }
  }
  __syncthreads();
  if (t < L) {
    double nr = 0.0;
#pragma unroll
    for (int ww = 0; ww < NT; ++ww) nr += rsum[ww][t];
    const double b0 = gp(J.beta0)[t];
    const double r = b0 > 0.0 ? sqrt(nr) / b0 : 0.0;
    gp(J.res)[(int64_t)s * LP + t] = r;
    if (r > J.tol) atomicAdd(gp(J.active) + (k & 1), 1);
  }
  if (s == 0 && t == 0) gp(J.active)[(k + 1) & 1] = 0;
}

hipError_t launch_b_shift(const BBatch &b, int init, hipStream_t st) {
  if (b.lpmask & 1)
    hipLaunchKernelGGL(b_shift<16>, dim3(b.totals), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffs, b.clock, init);
  if (b.lpmask & 2)
    hipLaunchKernelGGL(b_shift<32>, dim3(b.totals), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffs, b.clock, init);
  if (b.lpmask & 4)
    hipLaunchKernelGGL(b_shift<64>, dim3(b.totals), dim3(kThreads), 0, st, b.jobs, b.njob, b.toffs, b.clock, init);
  return hipGetLastError();
}

// ------------------------------------------------------ backward solution
// Y_k = H_k^{-1} (Z_k + B_{k+1}^T Y_{k+1}), k = K-1 .. 0; Y_k overwrites Z_k
// (columns < L).  The columns are independent: one workgroup per (shift,
// group of 16 columns).  Both products of a step are FP64 MFMA tiles: wave w
// owns rows 16 w .. 16 w + 15 of T = Z_k + B_{k+1}^T Y_{k+1} and of
// Y_k = H_k^{-1} T, real and imaginary part (A operand from LDS in rows, B
// operand from the column tiles, accumulator in the MFMA output layout).
// The recurrence is sequential in k, so the operands of step k - 1 (H^{-1},
// B, the wave's Z tile) are loaded into registers while step k computes and
// staged in LDS at the start of the next step.
constexpr int kBsCols = 16;

template <int LP>
__global__ __launch_bounds__(kThreads) void b_backsolve(BJobDesc J, int K) {
  constexpr int L2 = LP * LP, SS = LP + 1, TS = kBsCols + 1, KS = LP / 4;
  constexpr int IT = (L2 + kThreads - 1) / kThreads;
  __shared__ double Hr[LP * SS], Hi[LP * SS], Bs[LP * SS];
  __shared__ double Tr[LP * TS], Ti[LP * TS], Yr[LP * TS], Yi[LP * TS];
  const int L = J.L, ng = (L + kBsCols - 1) / kBsCols;
  const int s = blockIdx.x / ng, cg = blockIdx.x - s * ng;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const bool act = w < LP / 16;
  const int col = cg * kBsCols + rl;  // this lane's column in the MFMA output layout
  const bool live = col < L;
  const int64_t hbase = (int64_t)s * (J.Kcap + 1) * L2;
  const GLB double2 *__restrict__ Hinv = gp(J.Hinv) + hbase;
  GLB double2 *__restrict__ Zh = gp(J.Zh) + hbase;
  double2 hv[IT], zv[4], zn[4];
  double bv[IT];
  // operands of step k: H_k^{-1}, B_{k+1} (none for the last step) and the
  // wave's tile of Z_k (rows 16 w + q + 4 v, column col)
  auto fetch = [&](int k, double2 (&z)[4]) {
    const GLB double2 *__restrict__ Hk = Hinv + (int64_t)k * L2;
    const GLB double *__restrict__ Bk1 = gp(J.Bh) + (int64_t)(k + 1) * L2;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      hv[it] = make_double2(0.0, 0.0);
      if (e < L2) hv[it] = Hk[e];
      bv[it] = (e < L2 && k < K - 1) ? Bk1[e] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      z[v] = make_double2(0.0, 0.0);
      if (act && live) z[v] = Zh[(int64_t)k * L2 + (16 * w + q + 4 * v) * LP + col];
    }
  };
  if (K > 0) fetch(K - 1, zv);
  for (int k = K - 1; k >= 0; --k) {
    __syncthreads();  // the previous step is done with Hr, Hi, Bs, Tr, Ti and wrote Yr, Yi
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      if (e < L2) {
        const int r = e / LP, c = e - r * LP;
        Hr[r * SS + c] = hv[it].x;
        Hi[r * SS + c] = hv[it].y;
        Bs[r * SS + c] = bv[it];
      }
    }
    __syncthreads();
    if (k > 0) fetch(k - 1, zn);
    if (act) {
      // T = Z_k + B_{k+1}^T Y_{k+1}; (B^T)(i, c) = B(c, i)
      v4d Dr = v4d{zv[0].x, zv[1].x, zv[2].x, zv[3].x};
      v4d Di = v4d{zv[0].y, zv[1].y, zv[2].y, zv[3].y};
      if (k < K - 1) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int c = 4 * ks + q;
          const double a = Bs[c * SS + 16 * w + rl];
          Dr = mfma4b(a, Yr[c * TS + rl], Dr);
          Di = mfma4b(a, Yi[c * TS + rl], Di);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Tr[(16 * w + q + 4 * v) * TS + rl] = Dr[v];
        Ti[(16 * w + q + 4 * v) * TS + rl] = Di[v];
      }
    }
    __syncthreads();
    if (act) {
      // Y_k = H_k^{-1} T: real part Hr Tr - Hi Ti, imaginary part Hr Ti + Hi Tr
      v4d Dr = v4d{0.0, 0.0, 0.0, 0.0}, Di = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int c = 4 * ks + q;
        const double ar = Hr[(16 * w + rl) * SS + c], ai = Hi[(16 * w + rl) * SS + c];
        const double br = Tr[c * TS + rl], bi = Ti[c * TS + rl];
        Dr = mfma4b(ar, br, Dr);
        Dr = mfma4b(-ai, bi, Dr);
        Di = mfma4b(ar, bi, Di);
        Di = mfma4b(ai, br, Di);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + q + 4 * v;
        Yr[i * TS + rl] = Dr[v];
        Yi[i * TS + rl] = Di[v];
        if (live) Zh[(int64_t)k * L2 + i * LP + col] = make_double2(Dr[v], Di[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) zv[v] = zn[v];
  }
}

hipError_t launch_b_backsolve(const BJobDesc &hj, int K, hipStream_t st) {
  const int ng = (hj.L + kBsCols - 1) / kBsCols;
  if (K <= 0) return hipSuccess;
  switch (hj.Lp) {
    case 16: hipLaunchKernelGGL(b_backsolve<16>, dim3(hj.S * ng), dim3(kThreads), 0, st, hj, K); break;
    case 32: hipLaunchKernelGGL(b_backsolve<32>, dim3(hj.S * ng), dim3(kThreads), 0, st, hj, K); break;
    case 64: hipLaunchKernelGGL(b_backsolve<64>, dim3(hj.S * ng), dim3(kThreads), 0, st, hj, K); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// F_k(c, kk*L + l) = sum_s 2 Re(c_{s,kk} Y_{s,k}(c, l)), stored column-major
// per step: F[k][(kk*L + l) * Lp + c].  One workgroup per (step k, group of
// 16 rows c): each thread reads the entries (c, l) of its kFcPairs pairs for
// every shift once (consecutive l, coalesced) and keeps up to kFcMom moment
// sums per pair, summed over the shifts in order; the sums of one kk go out
// through LDS so that the stores run along c.
constexpr int kFcPairs = 4, kFcMom = 9;

__global__ __launch_bounds__(kThreads) void b_fcoef(BJobDesc J, int K) {
  static_assert(16 * kBlockMaxLp <= kThreads * kFcPairs, "pairs per workgroup");
  __shared__ double Fs[16 * kBlockMaxLp];
  const int Lp = J.Lp, L2 = Lp * Lp, L = J.L, KL = J.Kmom * L;
  const int ncg = Lp / 16;
  const int k = blockIdx.x / ncg, g = blockIdx.x - k * ncg;
  const int t = threadIdx.x, np = 16 * L;
  GLB double *Fk = gp(J.F) + (int64_t)k * KL * Lp;
  for (int kk0 = 0; kk0 < J.Kmom; kk0 += kFcMom) {
    const int nk = min(kFcMom, J.Kmom - kk0);
    double acc[kFcPairs][kFcMom];
#pragma unroll
    for (int u = 0; u < kFcPairs; ++u)
#pragma unroll
      for (int q = 0; q < kFcMom; ++q) acc[u][q] = 0.0;
    for (int s = 0; s < J.S; ++s) {
      const GLB double2 *__restrict__ Y = gp(J.Zh) + ((int64_t)s * (J.Kcap + 1) + k) * L2;
      double2 y[kFcPairs];
#pragma unroll
      for (int u = 0; u < kFcPairs; ++u) {
        const int p = t + u * kThreads;
        y[u] = make_double2(0.0, 0.0);
        if (p < np) y[u] = Y[(16 * g + p / L) * Lp + p % L];
      }
#pragma unroll
      for (int q = 0; q < kFcMom; ++q) {
        if (q < nk) {
          const double2 cm = gp(J.cmom)[s * J.cstride + kk0 + q];
#pragma unroll
          for (int u = 0; u < kFcPairs; ++u) acc[u][q] += 2.0 * (cm.x * y[u].x - cm.y * y[u].y);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kFcMom; ++q) {
      if (q < nk) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kFcPairs; ++u) {
          const int p = t + u * kThreads;
          if (p < np) Fs[(p % L) * 16 + p / L] = acc[u][q];
        }
        __syncthreads();
        for (int e = t; e < np; e += kThreads) {
          const int l = e >> 4, cl = e & 15;
          Fk[((int64_t)(kk0 + q) * L + l) * Lp + 16 * g + cl] = Fs[e];
        }
      }
    }
  }
}

hipError_t launch_b_fcoef(const BJobDesc &hj, int K, hipStream_t st) {
  if (K <= 0) return hipSuccess;
  if (hj.L > hj.Lp || hj.Lp % 16 != 0 || hj.Lp > kBlockMaxLp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(b_fcoef, dim3((unsigned)(K * (hj.Lp / 16))), dim3(kThreads), 0, st, hj, K);
  return hipGetLastError();
}

// ------------------------------------------------------ moment accumulation
// S(r, col) += sum_b sum_c Q_{k0+b}(r, c) F_{k0+b}(c, col), S column-major
// (ld npad), F column-major per step (Lp x KL).  A product with a long
// contraction (T Lp) and a thin result, bound by the FP64 MFMA rate.
// Workgroup tile: 64 WR rows x COLS columns, each wave WR tiles of 16 rows
// (MFMA 16x16x4; lane (rl, q) supplies Q(row rl, c) with c = 4 q + ks of
// the chunk).  The contraction runs in chunks of 16 indices: while the MFMAs
// of one chunk run from one LDS buffer, the next chunk of F is loaded into
// registers (then stored into the other buffer) and the next Q fragments are
// loaded ahead, one barrier per chunk.  At the end the result is added to S
// through an LDS transpose so that each column segment is written whole.
constexpr int kMomKC = 16;            // contraction indices per staged chunk
constexpr int kMomWR = 1;             // 16-row tiles per wave
constexpr int kMomOcc = 3;            // workgroups per CU the registers are sized for
constexpr int kMomCols = 96;          // result columns per workgroup

// QT = float: the basis blocks come from the FP32 copies of a mixed-precision
// stored basis and are widened to FP64 as they are loaded (same products).
template <int LP, int WR, int OCC, int COLS, typename QT>
__global__ __launch_bounds__(kThreads, OCC) void b_moments(BJobDesc J, int k0, int T) {
  static_assert(LP % kMomKC == 0, "chunks of 16 contraction indices");
  constexpr int NTL = COLS / 16, NCH = LP / kMomKC;
  // LDS row stride of the staged F chunk (measured: COLS + 1 or + 2 runs 4%
  // faster than + 4, + 8 or more is slower; + 2 keeps rows 16-byte aligned)
  constexpr int FS = COLS + 2;
  constexpr int FL = kMomKC * COLS / kThreads;  // F loads per thread and chunk
  static_assert(FL * kThreads == kMomKC * COLS, "whole chunks");
  constexpr int FBUF = kMomKC * FS, ROWS = 64 * WR, CS = ROWS + 1;
  // epilogue column group: the transpose buffer reuses the F buffers
  constexpr int CG = (64 * CS <= 2 * FBUF && COLS % 64 == 0) ? 64 : 32;
  static_assert(CG * CS <= 2 * FBUF && COLS % CG == 0, "transpose fits the F buffers");
  __shared__ double sm[2 * FBUF];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const int64_t n = J.n;
  const int KL = J.Kmom * J.L;
  // workgroups go to the 8 XCDs round-robin by id: the column groups of a
  // row tile are consecutive workgroups of one XCD, so they share its L2
  // for the basis rows (row tiles padded to a multiple of 8)
  const int ngrp = (KL + COLS - 1) / COLS;
  const int xcd = blockIdx.x % 8, j = blockIdx.x / 8;
  const int64_t rb = ((int64_t)(j / ngrp) * 8 + xcd) * ROWS;
  const int col0 = (j % ngrp) * COLS;
  if (rb >= n) return;
  v4d acc[WR][NTL];
#pragma unroll
  for (int r = 0; r < WR; ++r)
#pragma unroll
    for (int i = 0; i < NTL; ++i) acc[r][i] = v4d{0.0, 0.0, 0.0, 0.0};
  double fv[FL], a[WR][4], an[WR][4];
  // chunk g: step k0 + g / NCH, contraction indices 16 (g % NCH) + 0..15
  auto load_f = [&](int g) {
    const GLB double *__restrict__ Fk =
        gp(J.F) + (int64_t)(k0 + g / NCH) * KL * LP + (g % NCH) * kMomKC;
#pragma unroll
    for (int i = 0; i < FL; ++i) {
      const int e = t + i * kThreads, col = e >> 4, c = e & 15;
      fv[i] = (col0 + col < KL) ? Fk[(int64_t)(col0 + col) * LP + c] : 0.0;
    }
  };
  auto store_f = [&](int buf) {
    double *Fs = sm + buf * FBUF;
#pragma unroll
    for (int i = 0; i < FL; ++i) {
      const int e = t + i * kThreads;
      Fs[(e & 15) * FS + (e >> 4)] = fv[i];
    }
  };
  auto load_q = [&](int g, double (&x)[WR][4]) {
    if constexpr (sizeof(QT) == 4) {
      const GLB float *__restrict__ Qk = q32block(J, k0 + g / NCH) + (g % NCH) * kMomKC + 4 * q;
#pragma unroll
      for (int r = 0; r < WR; ++r) {
        const int64_t row = rb + 16 * (w * WR + r) + rl;
        if (row < n) {
          const v4f x0 = *reinterpret_cast<const GLB v4f *>(Qk + row * LP);
          x[r][0] = (double)x0.x;
          x[r][1] = (double)x0.y;
          x[r][2] = (double)x0.z;
          x[r][3] = (double)x0.w;
        } else {
          x[r][0] = x[r][1] = x[r][2] = x[r][3] = 0.0;
        }
      }
    } else {
      const GLB double *__restrict__ Qk = qblock(J, k0 + g / NCH) + (g % NCH) * kMomKC + 4 * q;
#pragma unroll
      for (int r = 0; r < WR; ++r) {
        const int64_t row = rb + 16 * (w * WR + r) + rl;
        if (row < n) {
          const GLB v2d *p = reinterpret_cast<const GLB v2d *>(Qk + row * LP);
          const v2d x0 = p[0], x1 = p[1];
          x[r][0] = x0.x;
          x[r][1] = x0.y;
          x[r][2] = x1.x;
          x[r][3] = x1.y;
        } else {
          x[r][0] = x[r][1] = x[r][2] = x[r][3] = 0.0;
        }
      }
    }
  };
  const int G = T * NCH;
  load_f(0);
  load_q(0, a);
  store_f(0);
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    const bool more = g + 1 < G;
    if (more) {
      load_f(g + 1);
      load_q(g + 1, an);
    }
    const double *Fs = sm + (g & 1) * FBUF + q * 4 * FS + rl;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int tt = 0; tt < NTL; ++tt) {
        const double b = Fs[ks * FS + 16 * tt];
#pragma unroll
        for (int r = 0; r < WR; ++r) acc[r][tt] = mfma4b(a[r][ks], b, acc[r][tt]);
      }
    if (more) {
      store_f((g + 1) & 1);
#pragma unroll
      for (int r = 0; r < WR; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) a[r][i] = an[r][i];
    }
    __syncthreads();
  }
  // add to S in column segments of ROWS rows, CG columns at a time
  double *Cs = sm;
#pragma unroll
  for (int cg = 0; cg < COLS; cg += CG) {
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < NTL; ++tt) {
      if (16 * tt >= cg && 16 * tt < cg + CG)
#pragma unroll
        for (int r = 0; r < WR; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) Cs[(16 * tt - cg + rl) * CS + 16 * (w * WR + r) + q + 4 * v] = acc[r][tt][v];
    }
    __syncthreads();
    for (int e = t; e < CG * ROWS; e += kThreads) {
      const int cl = e / ROWS, rr = e % ROWS;
      const int col = col0 + cg + cl;
      const int64_t row = rb + rr;
      if (col < KL && row < n) {
        const int gcol = (col / J.L) * J.sL + J.soff + col % J.L;  // column of S (groups of a wide L)
        GLB double *sp = gp(J.Sout) + (int64_t)gcol * J.npad + row;
        *sp += Cs[cl * CS + rr];
      }
    }
  }
}

hipError_t launch_b_moments(const BJobDesc &hj, int k0, int T, hipStream_t st) {
  if (T <= 0) return hipSuccess;
  const int KL = hj.Kmom * hj.L;
  constexpr int ROWS = 64 * kMomWR, C = kMomCols;
  const int64_t tiles8 = (hj.n + 8 * ROWS - 1) / (8 * ROWS) * 8;  // row tiles padded to a multiple of 8
  const dim3 g((unsigned)(tiles8 * ((KL + C - 1) / C)));
#define CSVD_MOM(LPV, QTV) \
  hipLaunchKernelGGL((b_moments<LPV, kMomWR, kMomOcc, C, QTV>), g, dim3(kThreads), 0, st, hj, k0, T)
  if (hj.store32) {
    switch (hj.Lp) {
      case 16: CSVD_MOM(16, float); break;
      case 32: CSVD_MOM(32, float); break;
      default: CSVD_MOM(64, float); break;
    }
  } else {
    switch (hj.Lp) {
      case 16: CSVD_MOM(16, double); break;
      case 32: CSVD_MOM(32, double); break;
      default: CSVD_MOM(64, double); break;
    }
  }
#undef CSVD_MOM
  return hipGetLastError();
}

// FP32 copy of one basis block (the blocks gamma does not write: Q_0 and the
// Householder-orthonormalised blocks of robust steps), rounded to nearest
__global__ void b_store32(BJobDesc J, int kb) {
  const GLB double *__restrict__ src = qblock(J, kb);
  GLB float *__restrict__ dst = q32block(J, kb);
  const int64_t cnt = (int64_t)J.n * J.Lp;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

hipError_t launch_b_store32(const BJobDesc &hj, int kb, hipStream_t st) {
  if (!hj.store32) return hipSuccess;
  const int64_t cnt = (int64_t)hj.n * hj.Lp;
  const unsigned grid = (unsigned)std::min<int64_t>((cnt + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(b_store32, dim3(grid), dim3(kThreads), 0, st, hj, kb);
  return hipGetLastError();
}

// ------------------------------------------------------ starting block
// B[r * Lp + c] = R(r, c) for r <= c, 0 below: the triangle of a Householder
// QR stored column-major (ld) in X.
__global__ void b_r0(const double *__restrict__ X, int64_t ld, int Lp, double *__restrict__ B) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Lp * Lp) return;
  const int r = e / Lp, c = e - r * Lp;
  B[e] = (r <= c) ? X[(int64_t)c * ld + r] : 0.0;
}

hipError_t launch_b_r0(const double *X, int64_t ld, int Lp, double *B, hipStream_t st) {
  hipLaunchKernelGGL(b_r0, dim3((Lp * Lp + 255) / 256), dim3(256), 0, st, X, ld, Lp, B);
  return hipGetLastError();
}

// Z = the first cols columns of the rows x rows identity, column-major (ld)
__global__ void b_eye(double *__restrict__ Z, int64_t ld, int64_t rows, int cols) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / rows, r = e - c * rows;
    Z[c * ld + r] = (r == c) ? 1.0 : 0.0;
  }
}

hipError_t launch_b_eye(double *Z, int64_t ld, int64_t rows, int cols, hipStream_t st) {
  int64_t g = (rows * cols + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(b_eye, dim3((unsigned)g), dim3(256), 0, st, Z, ld, rows, cols);
  return hipGetLastError();
}

// Convergence snapshot of every job of a batch into host memory (4 ints per
// job): part 0 the active count after the job's newest step (written by the
// shift recurrences), part 1 its flags[0..2] (written by the step kernels).
// Jobs whose first step has not run get -1.
__global__ void b_setclock(int64_t *clk, int64_t value) { *clk = value; }
__global__ void b_tick(int64_t *clk) { *clk += 1; }

hipError_t launch_b_setclock(int64_t *clk, int64_t value, hipStream_t st) {
  hipLaunchKernelGGL(b_setclock, dim3(1), dim3(1), 0, st, clk, value);
  return hipGetLastError();
}

hipError_t launch_b_tick(int64_t *clk, hipStream_t st) {
  hipLaunchKernelGGL(b_tick, dim3(1), dim3(1), 0, st, clk);
  return hipGetLastError();
}

__global__ void b_snap(const BJobDesc *__restrict__ jobs, int njob, int64_t clock, int part, int *host) {
  for (int i = threadIdx.x; i < njob; i += blockDim.x) {
    const BJobDesc &J = jobs[i];
    const int steps = (int)(clock - J.start_clock);
    int *h = host + 4 * i;
    if (steps <= 0) {
      h[part == 0 ? 0 : 1] = -1;
      continue;
    }
    const int klast = min(steps - 1, J.Kstop - 1);
    if (part == 0) {
      h[0] = J.active[klast & 1];
    } else {
      h[1] = J.flags[0];
      h[2] = J.flags[1];
      h[3] = J.flags[2];
    }
  }
}

hipError_t launch_b_snap(const BBatch &b, int part, int *host, hipStream_t st) {
  hipLaunchKernelGGL(b_snap, dim3(1), dim3(64), 0, st, b.jobs, b.njob, b.clock, part, host);
  return hipGetLastError();
}

}  // namespace csvd
