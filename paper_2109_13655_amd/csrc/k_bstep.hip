// Block Lanczos step on the n x Lp blocks (Lp = 16, 32 or 64), FP64 MFMA.
//
// Step k turns W = A^T A Q_k into Q_{k+1} by block classical Gram-Schmidt
// against Q_k, applied twice, and CholeskyQR2:
//
//   alpha:  W' = W - Q_{k-1} B_k^T (in place);  P = Q_k^T W'
//   beta:   W2 = W' - Q_k P (in place);  C = Q_k^T W2,  G2 = W2^T W2
//   small1: A_k = sym(P);  R1 = chol(G2 - C^T C);  T = C R1^-1
//   gamma0: Y = W2 R1^-1 - Q_k T (not stored);  G3 = Y^T Y
//   small2: R2 = chol(G3);  M = R1^-1 R2^-1;  N = T R2^-1;  B_{k+1} = R2 R1
//   gamma:  Q_{k+1} = Y R2^-1 = W2 M - Q_k N
//
// The first projection is applied explicitly and stored, and the second one
// (C, of the size of the rounding errors of the first) acts on W2: the new
// block is then exact to working precision relative to its own size.  With
// the two coefficients combined (W' - Q_k (P + C)) the result carries errors
// of eps ||W'|| along Q_k, which dominate when the new block is much smaller
// than W' (a nearly invariant starting block: rounds after the first, or a
// good starting guess) and spoil the solutions at the 1e-8 level.
//
// When the first Cholesky factor is well conditioned (rho = ||R1||_F
// ||R1^-1||_F / Lp <= onepass_rho, no deflated column; rho >= 1, and rho
// close to 1 bounds cond(R1) close to 1), Y = W2 R1^-1 - Q_k T is already
// orthonormal to working accuracy: small1 then takes M = R1^-1, N = T,
// B_{k+1} = R1 and marks the step (flags[1]), and gamma0, its reduction and
// small2 return at once.
//
// A new direction whose Cholesky pivot falls below kDeflTol^2 times its own
// squared norm before the projection is rounding noise (the space is
// exhausted) and is deflated: zero row in R, zero column of Q_{k+1}.  The
// second pass of the method (regenerating Q_k for the moments) runs alpha
// without Gram matrices, which then also forms W2 with P from the history of
// the first pass, and gamma: the same products in the same order, so the
// basis is reproduced bit for bit.
//
// Tall kernels: a job's rows are cut into 128-row chunks; each of its nvb
// workgroups (8 waves, one 16-row panel each, two waves per SIMD) walks the
// chunks vb, vb + nvb, ... and keeps its Gram partial sums in MFMA
// accumulators.  The partials are reduced in a fixed order, so results do not
// depend on timing or on which other jobs share the launch.
#include "csvd_impl.h"

namespace csvd {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int kPanel = 64;              // rows staged at a time for the Gram products (4 panels)
constexpr int kTallThreads = 512;       // threads of the tall kernels (8 waves)
constexpr int kTallRows = 128;          // rows per chunk of the tall kernels (8 panels)
constexpr int kSS = kBlockMaxLp + 1;    // LDS row stride of staged Lp x Lp matrices
constexpr int kPSMax = kBlockMaxLp + 16;  // LDS row stride of staged panels (largest)
constexpr int kMaxTiles = 4;            // Gram output tiles per wave (Lp = 64: 16 + 10 over 8 waves)

__device__ __forceinline__ int bfind2(const int *__restrict__ toff, int njob, int g) {
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (toff[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// panel row stride in LDS (LP == 16 ? 16 : LP + 16): consecutive rows land
// 32 banks apart

// D[nt] += X(rows row0 .. row0 + 15) S for the 16-column tiles nt < Lp/16.
// MFMA f64 16x16x4: lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16)
// and holds D(l / 16 + 4 v, l % 16).  The contraction index c is split as
// c = q * KS + ks (q = l / 16), so each lane reads KS consecutive entries of
// its row with wide loads.
template <int LP>
__device__ __forceinline__ void load_rows(const GLB double *__restrict__ X, int64_t row0, int64_t n,
                                          double (&a)[LP / 4]) {
  constexpr int KS = LP / 4;
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
  const int64_t row = row0 + rl;
#pragma unroll
  for (int i = 0; i < KS; ++i) a[i] = 0.0;
  if (row < n) {
    const GLB v2d *p = reinterpret_cast<const GLB v2d *>(X + row * LP + q * KS);
#pragma unroll
    for (int i = 0; i < KS / 2; ++i) {
      const v2d v = p[i];
      a[2 * i] = v.x;
      a[2 * i + 1] = v.y;
    }
  }
}

template <int LP>
__device__ __forceinline__ void rows_mm(const double (&a)[LP / 4], const double *S, v4d (&D)[4]) {
  constexpr int KS = LP / 4, NT = LP / 16;
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const double *sr = S + (q * KS + ks) * kSS + rl;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) D[nt] = mfma4(a[ks], sr[16 * nt], D[nt]);
  }
}

template <int LP>
__device__ __forceinline__ void panel_mm(const GLB double *__restrict__ X, int64_t row0, int64_t n,
                                         const double *S, v4d (&D)[4]) {
  double a[LP / 4];
  load_rows<LP>(X, row0, n, a);
  rows_mm<LP>(a, S, D);
}

// element (row0 + l/16 + 4v, 16 nt + l%16) of a row-major n x Lp block
template <int LP>
__device__ __forceinline__ void load_dl(const GLB double *__restrict__ X, int64_t row0, int64_t n, v4d (&D)[4]) {
  constexpr int NT = LP / 16;
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = row0 + q + 4 * v;
      D[nt][v] = (row < n) ? X[row * LP + 16 * nt + rl] : 0.0;
    }
  }
}

template <int LP>
__device__ __forceinline__ void store_dl(GLB double *__restrict__ X, int64_t row0, int64_t n, const v4d (&D)[4]) {
  constexpr int NT = LP / 16;
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = row0 + q + 4 * v;
      if (row < n) X[row * LP + 16 * nt + rl] = D[nt][v];
    }
  }
}

// the same rows rounded to FP32 (the stored basis of mixed precision)
template <int LP>
__device__ __forceinline__ void store_dl32(GLB float *__restrict__ X, int64_t row0, int64_t n, const v4d (&D)[4]) {
  constexpr int NT = LP / 16;
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = row0 + q + 4 * v;
      if (row < n) X[row * LP + 16 * nt + rl] = (float)D[nt][v];
    }
  }
}

__device__ __forceinline__ void zero4(v4d (&D)[4]) {
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) D[nt] = v4d{0.0, 0.0, 0.0, 0.0};
}

// Gram output tile tau of a wave: tau < nfull -> tile (ti, tj) of X^T Y
// (mat 0, nfull = NT^2 or 0); else the upper tiles ti <= tj of Y^T Y (mat 1),
// row by row.
__device__ __forceinline__ void gram_tile(int tau, int NT, int nfull, int &mat, int &ti, int &tj) {
  if (tau < nfull) {
    mat = 0;
    ti = tau / NT;
    tj = tau - ti * NT;
  } else {
    int u = tau - nfull;
    ti = 0;
    while (u >= NT - ti) {
      u -= NT - ti;
      ++ti;
    }
    mat = 1;
    tj = ti + u;
  }
}

// Accumulates this wave's Gram tiles over the 128 rows of a chunk: the eight
// waves' panels (Q part and new part, D layout) are staged 64 rows at a time
// (waves 0-3, then 4-7), and each wave runs its tiles over the staged rows.
template <int LP>
__device__ __forceinline__ void gram_chunk(const v4d (&Xd)[4], const v4d (&Yd)[4], int nfull, int ntile, double *Xs,
                                           double *Ys, v4d (&acc)[kMaxTiles]) {
  constexpr int NT = LP / 16, PS = (LP == 16) ? 16 : LP + 16;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  for (int half = 0; half < 2; ++half) {
    if ((w >> 2) == half) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = 16 * (w & 3) + q + 4 * v;
          if (nfull) Xs[rr * PS + 16 * nt + rl] = Xd[nt][v];
          Ys[rr * PS + 16 * nt + rl] = Yd[nt][v];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxTiles; ++i) {
      const int tau = w + 8 * i;
      if (tau < ntile) {
        int mat, ti, tj;
        gram_tile(tau, NT, nfull, mat, ti, tj);
        const double *Am = mat == 0 ? Xs : Ys;
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
          const int rr = 4 * ks + q;
          acc[i] = mfma4(Am[rr * PS + 16 * ti + rl], Ys[rr * PS + 16 * tj + rl], acc[i]);
        }
      }
    }
    __syncthreads();
  }
}

// partial sums of workgroup vb: gpart[(vb * 2 + mat) * L2 + r * Lp + c]
__device__ __forceinline__ void store_gram(const BJobDesc &J, int vb, int nfull, int ntile,
                                           const v4d (&acc)[kMaxTiles]) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const int LP = J.Lp, NT = LP >> 4, L2 = LP * LP;
  GLB double *P = gp(J.gpart) + (int64_t)vb * 2 * L2;
#pragma unroll
  for (int i = 0; i < kMaxTiles; ++i) {
    const int tau = w + 8 * i;
    if (tau < ntile) {
      int mat, ti, tj;
      gram_tile(tau, NT, nfull, mat, ti, tj);
#pragma unroll
      for (int v = 0; v < 4; ++v) P[mat * L2 + (16 * ti + q + 4 * v) * LP + 16 * tj + rl] = acc[i][v];
    }
  }
}

// LP x LP matrix from global to LDS (stride kSS), optionally transposed or
// negated; fixed trip count, all loads of a thread issued before its stores
template <int LP, int NTH = kThreads>
__device__ __forceinline__ void stage_mat(const GLB double *__restrict__ src, bool trans, bool neg, double *dst) {
  constexpr int IT = (LP * LP + NTH - 1) / NTH;
  double v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NTH;
    const int r = e / LP, c = e % LP;
    v[it] = (e < LP * LP) ? (trans ? src[c * LP + r] : src[e]) : 0.0;
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * NTH;
    if (e < LP * LP) dst[(e / LP) * kSS + (e % LP)] = neg ? -v[it] : v[it];
  }
}

// ---------------------------------------------------------- tall passes
// kTallAlpha: W' = W - Q_{k-1} B_k^T stored in place and its Gram Q_k^T W'
//   (grams = 1, first pass); grams = 0 (second pass): W2 = W' - Q_k P_k
//   with P_k from the history, stored in place (beta's work, fused).
// kTallBeta:  W2 = W' - Q_k P stored in place; Grams Q_k^T W2 and W2^T W2.
// kTallGamma0: Y = W2 R1^-1 - Q_k T (not stored); Gram Y^T Y.
enum { kTallAlpha = 0, kTallBeta = 1, kTallGamma0 = 2 };

// gamma0 (the second Cholesky QR pass); its Gram tiles are staged through
// LDS (ten tiles per panel do not fit the registers of two waves per SIMD
// next to the two panel products)
template <int LP>
__global__ __launch_bounds__(kTallThreads) void bs_gamma0(const BJobDesc *__restrict__ jobs, int njob,
                                                      const int *__restrict__ toff,
                                                      StepClock clock) {
  __shared__ double S1[LP * kSS], S2[LP * kSS];
  __shared__ double Ys[kPanel * kPSMax];
  constexpr int L2 = LP * LP, NT = LP / 16;
  const int g = blockIdx.x;
  const int j = bfind2(toff, njob, g);
  const BJobDesc &J = jobs[j];
  if (J.Lp != LP) return;
  const int k = (int)(sclock(clock) - J.start_clock);
  if (k >= J.Kstop) return;
  if (gp(J.flags)[1]) return;  // one-pass step
  const int vb = g - toff[j];
  const int w = threadIdx.x >> 6;
  const int64_t n = J.n;
  const GLB double *X = gp(J.W);
  const GLB double *Qc = qblock(J, k);
  stage_mat<LP, kTallThreads>(gp(J.scr) + L2, false, false, S1);      // R1^-1
  stage_mat<LP, kTallThreads>(gp(J.scr) + 2 * L2, false, true, S2);  // -T
  __syncthreads();
  constexpr int ntile = NT * (NT + 1) / 2;
  v4d acc[kMaxTiles];
#pragma unroll
  for (int i = 0; i < kMaxTiles; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nch = (int)((n + kTallRows - 1) / kTallRows);
  for (int ch = vb; ch < nch; ch += J.nvb) {
    const int64_t r0 = (int64_t)ch * kTallRows + 16 * w;
    v4d D[4], Qd[4];
    zero4(D);
    zero4(Qd);
    panel_mm<LP>(X, r0, n, S1, D);
    panel_mm<LP>(Qc, r0, n, S2, D);
    gram_chunk<LP>(Qd, D, 0, ntile, Ys, Ys, acc);
  }
  store_gram(J, vb, 0, ntile, acc);
}

// ------------------------------------------------------------------ gamma
// Q_{k+1} = W2 M_k - Q_k N_k
template <int LP>
__global__ __launch_bounds__(kTallThreads) void bs_gamma(const BJobDesc *__restrict__ jobs, int njob,
                                                     const int *__restrict__ toff,
                                                     StepClock clock) {
  __shared__ double S1[LP * kSS], S2[LP * kSS];
  constexpr int L2 = LP * LP;
  const int g = blockIdx.x;
  const int j = bfind2(toff, njob, g);
  const BJobDesc &J = jobs[j];
  if (J.Lp != LP) return;
  const int k = (int)(sclock(clock) - J.start_clock);
  if (k >= J.Kstop) return;
  const int vb = g - toff[j];
  const int w = threadIdx.x >> 6;
  const int64_t n = J.n;
  const GLB double *X = gp(J.W);
  const GLB double *Qc = qblock(J, k);
  GLB double *Qn = qblock(J, k + 1);
  stage_mat<LP, kTallThreads>(gp(J.Mh) + (int64_t)k * L2, false, false, S1);
  stage_mat<LP, kTallThreads>(gp(J.Nh) + (int64_t)k * L2, false, true, S2);
  __syncthreads();
  const int nch = (int)((n + kTallRows - 1) / kTallRows);
  for (int ch = vb; ch < nch; ch += J.nvb) {
    const int64_t r0 = (int64_t)ch * kTallRows + 16 * w;
    v4d D[4];
    zero4(D);
    panel_mm<LP>(X, r0, n, S1, D);
    // keeps the second panel's loads after the first product (hoisted, they
    // exceed the register file at Lp = 64)
    __builtin_amdgcn_sched_barrier(0);
    panel_mm<LP>(Qc, r0, n, S2, D);
    store_dl<LP>(Qn, r0, n, D);
    if (J.store32) store_dl32<LP>(q32block(J, k + 1), r0, n, D);  // mixed precision: FP32 copy
  }
}

// ------------------------------------------------- tall passes, wave-local
// The same passes with the Gram products accumulated per wave from its own
// 16-row panels: lane (rl, q) holds X(row q + 4 v, 16 t + rl) of tile t in
// the MFMA output layout, which is also the A and B operand layout of
// (X^T Y)(16 ti .. , 16 tj ..) = sum_v mfma(X[ti][v], Y[tj][v]), so no LDS
// staging and no barrier is needed inside the loop; the waves run
// independently over the panels w, w + waves, ... of their workgroup's
// share.  At the end the waves' sums are added in a fixed order (wave 0,
// 1, ...) through LDS and stored as the workgroup's partial sums.
template <int LP, int MODE, int NTH>
__global__ __launch_bounds__(NTH, (MODE == kTallBeta && LP == 64) ? 1 : 2) void bs_tall_rg(
    const BJobDesc *__restrict__ jobs, int njob, const int *__restrict__ toff, StepClock clock,
    int grams) {
  static_assert(MODE == kTallAlpha || MODE == kTallBeta, "alpha and beta passes");
  constexpr int NT = LP / 16, L2 = LP * LP, NW = NTH / 64;
  constexpr int NF = NT * NT;                                       // tiles of Q_k^T X
  constexpr int NS = (MODE == kTallAlpha) ? 0 : NT * (NT + 1) / 2;  // upper tiles of X^T X
  constexpr int NA = NF + NS;
  __shared__ double SM[2 * LP * kSS];
  double *S1 = SM, *S2 = SM + LP * kSS;
  const int g = blockIdx.x;
  const int j = bfind2(toff, njob, g);
  const BJobDesc &J = jobs[j];
  if (J.Lp != LP) return;
  const int k = (int)(sclock(clock) - J.start_clock);
  if (k >= J.Kstop) return;
  const int vb = g - toff[j];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const int64_t n = J.n;
  GLB double *X = gp(J.W);
  const GLB double *Qc = qblock(J, k);
  const GLB double *Pv = qblock(J, k > 0 ? k - 1 : k);
  const bool useQ = (MODE != kTallAlpha || k > 0);
  if (MODE == kTallAlpha) {
    if (useQ) stage_mat<LP, NTH>(gp(J.Bh) + (int64_t)k * L2, true, true, S2);  // -B_k^T
    if (!grams) stage_mat<LP, NTH>(gp(J.Ph) + (int64_t)k * L2, false, true, S1);  // -P_k (second pass)
  } else {
    stage_mat<LP, NTH>(gp(J.red), false, true, S2);  // -P
  }
  __syncthreads();
  v4d acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  const int npanel = (int)((n + 15) / 16);
  for (int pn = vb * NW + w; pn < npanel; pn += J.nvb * NW) {
    const int64_t r0 = (int64_t)pn * 16;
    v4d D[4];
    load_dl<LP>(X, r0, n, D);
    if (useQ) panel_mm<LP>(MODE == kTallAlpha ? Pv : Qc, r0, n, S2, D);
    if (MODE == kTallAlpha && !grams) {
      // second pass: W2 = W' - Q_k P_k with the products and their order of
      // beta in the first pass, so the stored W2 is the same bits
      panel_mm<LP>(Qc, r0, n, S1, D);
      store_dl<LP>(X, r0, n, D);
    } else if (MODE == kTallAlpha && useQ) {
      store_dl<LP>(X, r0, n, D);  // W' in place
    }
    if (grams) {
      __builtin_amdgcn_sched_barrier(0);  // Q_k panel loads after the update (register pressure)
      if (NF) {
        v4d Qd[4];
        load_dl<LP>(Qc, r0, n, Qd);
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
          for (int tj = 0; tj < NT; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[ti * NT + tj] = mfma4(Qd[ti][v], D[tj][v], acc[ti * NT + tj]);
      }
      if (NS) {
        int u = NF;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
          for (int tj = ti; tj < NT; ++tj, ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u] = mfma4(D[ti][v], D[tj][v], acc[u]);
      }
    }
    if (MODE == kTallBeta) store_dl<LP>(X, r0, n, D);  // W2 in place
  }
  if (!grams) return;
  // fixed-order sum of the waves' tiles in LDS (the staged matrices are done)
  double *Red = SM;  // NA x 256 doubles
  static_assert(NA * 256 <= 2 * LP * kSS, "reduction buffer");
  __syncthreads();
  for (int ww = 0; ww < NW; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double *r = Red + (i * 4 + v) * 64 + l;
          *r = (ww == 0) ? acc[i][v] : *r + acc[i][v];
        }
    }
    __syncthreads();
  }
  // partial sums of workgroup vb: gpart[(vb * 2 + mat) * L2 + r * Lp + c]
  GLB double *P = gp(J.gpart) + (int64_t)vb * 2 * L2;
  for (int e = t; e < NA * 256; e += NTH) {
    const int i = e >> 8, v = (e >> 6) & 3, ll = e & 63, rr = ll & 15, qq = ll >> 4;
    int mat, ti, tj;
    if (i < NF) {
      mat = 0;
      ti = i / NT;
      tj = i - ti * NT;
    } else {
      mat = 1;
      int u = i - NF;
      ti = 0;
      while (u >= NT - ti) {
        u -= NT - ti;
        ++ti;
      }
      tj = ti + u;
    }
    P[mat * L2 + (16 * ti + qq + 4 * v) * LP + 16 * tj + rr] = Red[e];
  }
}

// ----------------------------------------------------------------- reduce
// red[(d0 + m) L2 + e] = sum over the workgroups vb of gpart[(vb * 2 + m0 +
// m) L2 + e], m < nm, in a fixed order: 8 interleaved partial sums combined
// in order.  Grid (njob, 2 * 64 * 64 / 32); block = 32 outputs x 8 groups.
// The workgroup count of the tall kernels is at most kBlockMaxVB.
__global__ __launch_bounds__(kThreads) void bs_reduce(const BJobDesc *__restrict__ jobs,
                                                      StepClock clock, int m0, int nm, int d0,
                                                      int second) {
  __shared__ double part[8][32];
  const BJobDesc &J = jobs[blockIdx.x];
  const int k = (int)(sclock(clock) - J.start_clock);
  if (k >= J.Kstop) return;
  if (second && gp(J.flags)[1]) return;  // one-pass step: no second Gram
  const int L2 = J.Lp * J.Lp;
  if ((int)blockIdx.y * 32 >= nm * L2) return;
  const int t = threadIdx.x, grp = t >> 5;
  const int o = blockIdx.y * 32 + (t & 31);
  const GLB double *__restrict__ P = gp(J.gpart) + (int64_t)m0 * L2;
  // all of this thread's partials (workgroups grp, grp + 8, ...) are loaded
  // at once, then added in that order (past nvb they are zeros)
  constexpr int kPer = kBlockMaxVB / 8;
  double v[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int vb = grp + 8 * i;
    v[i] = (vb < J.nvb) ? P[(int64_t)vb * 2 * L2 + o] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) s += v[i];
  part[grp][t & 31] = s;
  __syncthreads();
  if (grp == 0) {
    double r = part[0][t];
#pragma unroll
    for (int h = 1; h < 8; ++h) r += part[h][t];
    gp(J.red)[(int64_t)d0 * L2 + o] = r;
  }
}

// ------------------------------------------------------- small matrices
// One workgroup per job.  Lp x Lp matrices live in registers in the MFMA
// output layout (wave w < Lp/16 holds rows 16 w + l/16 + 4 v, columns
// 16 tj + l%16); products run on MFMA from LDS operands; the Cholesky
// factorisation and the triangular inverse advance one row per step with a
// single barrier, the active row broadcast through double-buffered LDS.
// D (+)= sign * A * B or sign * A^T * B with A, B in LDS (stride LP + 1)
// G from the reduced upper tiles: entry (r, c) lives at (r, c) when the tile
// of r is not below the tile of c, else at (c, r)
__device__ __forceinline__ double gram_sym(const GLB double *G, int LP, int r, int c) {
  return ((r >> 4) <= (c >> 4)) ? G[r * LP + c] : G[c * LP + r];
}

template <int LP, bool TA>
__device__ __forceinline__ void mm_lds(const double *A, const double *B, double sign, v4d (&D)[4]) {
  constexpr int NT = LP / 16, KS = LP / 4, SS = LP + 1;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  if (w >= NT) return;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int c = 4 * ks + q;
    const double a = sign * (TA ? A[c * SS + 16 * w + rl] : A[(16 * w + rl) * SS + c]);
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) D[tj] = mfma4(a, B[c * SS + 16 * tj + rl], D[tj]);
  }
}

template <int LP>
__device__ __forceinline__ void regs_to_lds(const v4d (&D)[4], double *X) {
  constexpr int NT = LP / 16, SS = LP + 1;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) X[(16 * w + q + 4 * v) * SS + 16 * tj + rl] = D[tj][v];
}

template <int LP>
__device__ __forceinline__ void regs_to_glb(const v4d (&D)[4], GLB double *X) {
  constexpr int NT = LP / 16;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) X[(16 * w + q + 4 * v) * LP + 16 * tj + rl] = D[tj][v];
}

// LP x LP row-major global -> LDS (stride LP + 1); the trip count is fixed,
// so all loads are issued before the first LDS store
template <int LP>
__device__ __forceinline__ void glb_to_lds(const GLB double *src, double *X, bool neg) {
  constexpr int SS = LP + 1, IT = (LP * LP + kThreads - 1) / kThreads;
  double v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * kThreads;
    v[it] = (e < LP * LP) ? src[e] : 0.0;
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * kThreads;
    if (e < LP * LP) X[(e / LP) * SS + (e % LP)] = neg ? -v[it] : v[it];
  }
}

// element v of a v4d with a runtime index (select chain, no scratch)
__device__ __forceinline__ double pick4(const v4d &x, int v) {
  return v == 0 ? x[0] : (v == 1 ? x[1] : (v == 2 ? x[2] : x[3]));
}
__device__ __forceinline__ void put4(v4d &x, int v, double val) {
  x[0] = v == 0 ? val : x[0];
  x[1] = v == 1 ? val : x[1];
  x[2] = v == 2 ? val : x[2];
  x[3] = v == 3 ? val : x[3];
}

// Right-looking Cholesky (upper factor) of the symmetric matrix in D, in
// place, with deflation: a pivot <= thr[c] zeroes row c of R.  rowb: 2 x LP.
// Each step reads everything it needs from LDS up front and updates its 16
// entries without branches (selects), so the step costs one LDS round trip
// and one barrier.
template <int LP>
__device__ __forceinline__ void chol_regs(v4d (&D)[4], const double *thr, int *dead, double (*rowb)[kBlockMaxLp]) {
  constexpr int NT = LP / 16;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const bool act = w < NT;
  const int i0 = 16 * w + q;  // rows i0 + 4 v
  if (act && w == 0 && q == 0)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) rowb[0][16 * tj + rl] = D[tj][0];
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < LP; ++c) {
    const int cb = c & 1;
    const double d = rowb[cb][c];
    const double th = thr[c];
    double rjv[4], riv[4];
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) rjv[tj] = rowb[cb][16 * tj + rl];
#pragma unroll
    for (int v = 0; v < 4; ++v) riv[v] = rowb[cb][act ? i0 + 4 * v : 0];
    const int dd = !(d > th);
    const double piv = dd ? 0.0 : sqrt(d);
    const double ip = dd ? 0.0 : 1.0 / piv;
    if (act) {
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const int jj = 16 * tj + rl;
        const double rj = rjv[tj] * ip;
        const double rowc = (jj < c) ? 0.0 : (jj == c ? piv : rj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 4 * v;
          const double a = D[tj][v];
          const double upd = a - (riv[v] * ip) * rj;
          D[tj][v] = (i == c) ? rowc : ((i > c && jj > c) ? upd : a);
        }
      }
      const int c1 = c + 1;
      if (c1 < LP && w == c1 / 16 && q == (c1 & 3))
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) rowb[cb ^ 1][16 * tj + rl] = pick4(D[tj], (c1 & 15) >> 2);
    }
    if (t == 0) dead[c] = dd;
    __syncthreads();
  }
}

// X = R^+ of the upper factor R (in LDS Rs, zero rows at deflated columns):
// the inverse on the kept rows and columns, zero elsewhere, in the register
// layout; rows from the bottom up, each finished row broadcast once.
template <int LP>
__device__ __forceinline__ void trinv_regs(const double *Rs, const int *dead, v4d (&X)[4],
                                           double (*rowb)[kBlockMaxLp]) {
  constexpr int NT = LP / 16, SS = LP + 1;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const bool act = w < NT;
  const int i0 = 16 * w + q;
  if (act)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 4 * v, jj = 16 * tj + rl;
        X[tj][v] = (i == jj && !dead[i]) ? 1.0 : 0.0;
      }
#pragma unroll 1
  for (int i = LP - 1; i >= 0; --i) {
    const int cb = i & 1;
    if (act && w == i / 16 && q == (i & 3)) {
      const double di = Rs[i * SS + i];
      const double rdi = dead[i] ? 0.0 : 1.0 / di;
      const int vi = (i & 15) >> 2;
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) {
        const double x = pick4(X[tj], vi) * rdi;
        put4(X[tj], vi, x);
        rowb[cb][16 * tj + rl] = x;
      }
    }
    __syncthreads();
    if (act) {
      double xr[4], rc[4];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) xr[tj] = rowb[cb][16 * tj + rl];
#pragma unroll
      for (int v = 0; v < 4; ++v) rc[v] = Rs[(i0 + 4 * v) * SS + i];
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) X[tj][v] = (i0 + 4 * v < i) ? X[tj][v] - rc[v] * xr[tj] : X[tj][v];
    }
  }
  __syncthreads();
}

// ---------------------------------------------- blocked small factorisations
// Cholesky with deflation and the triangular (pseudo-)inverse of an Lp x Lp
// matrix in LDS (stride Lp + 1), on 16 x 16 tiles: one wave factors and
// inverts each diagonal tile (sixteen steps ordered within the wave, no
// workgroup barrier), the block row and the trailing update run as 16x16x16
// MFMA tile products on all waves.  A deflated column has a zero row in R and
// a zero row and column in R^+ (the inverse on the kept indices).

// Orders this wave's LDS accesses: the LDS unit performs a wave's DS
// operations in issue order, so a write by one lane is seen by a later read
// of another lane of the same wave; only the compiler must not move memory
// operations across this point.
__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// 16x16 tile product on one wave: D (+)= op(A) B, A and B tiles in LDS with
// strides sa, sb; TA: A read transposed
template <bool TA>
__device__ __forceinline__ v4d tile_mm(const double *A, int sa, const double *B, int sb, v4d D) {
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + q;
    const double a = TA ? A[k * sa + rl] : A[rl * sa + k];
    D = mfma4(a, B[k * sb + rl], D);
  }
  return D;
}

__device__ __forceinline__ void tile_store(double *C, int sc, v4d D, double sign) {
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(q + 4 * v) * sc + rl] = sign * D[v];
}

__device__ __forceinline__ v4d tile_load(const double *C, int sc) {
  const int l = threadIdx.x & 63, rl = l & 15, q = l >> 4;
  v4d D;
#pragma unroll
  for (int v = 0; v < 4; ++v) D[v] = C[(q + 4 * v) * sc + rl];
  return D;
}

// one wave: Cholesky of the 16 x 16 diagonal tile at (16 K, 16 K) in place
// (upper factor R, rows scaled), thresholds thr[16 K + c], and the inverse
// of R in the same sweep: the elimination steps applied to the identity
// give R^-T (row c of it final once scaled by the pivot's 1/sqrt), written
// transposed into X's diagonal tile.  Lane l keeps the entries e = l + 64 u
// (u < 4; row e / 16, column e % 16) of both in registers; each step
// broadcasts the active rows through rowb (2 x 16 doubles).  A deflated
// pivot gives a zero row of R and a zero row and column of its inverse.
__device__ void diag_cholinv16(double *A, int SS, int K, const double *thr, int *dead, double *X, double *rowb) {
  const int l = threadIdx.x & 63, j = l & 15;
  double *D = A + 16 * K * SS + 16 * K;
  double *Xd = X + 16 * K * SS + 16 * K;
  double a[4], y[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = l + 64 * u;
    a[u] = D[(e >> 4) * SS + j];
    y[u] = ((e >> 4) == j) ? 1.0 : 0.0;
  }
#pragma unroll 1
  for (int c = 0; c < 16; ++c) {
    // owners of row c publish it (entries 16 c .. 16 c + 15: slot c >> 2)
    const int uc = c >> 2;
    if ((l >> 4) == (c & 3)) {
      rowb[j] = uc == 0 ? a[0] : (uc == 1 ? a[1] : (uc == 2 ? a[2] : a[3]));
      rowb[16 + j] = uc == 0 ? y[0] : (uc == 1 ? y[1] : (uc == 2 ? y[2] : y[3]));
    }
    wave_lds_sync();
    const double d = rowb[c];
    const int dd = !(d > thr[16 * K + c]);
    const double piv = dd ? 0.0 : sqrt(d);
    const double ip = dd ? 0.0 : 1.0 / piv;
    const double rj = rowb[j] * ip, ycj = rowb[16 + j] * ip;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = (l >> 4) + 4 * u;
      const double rci = rowb[i] * ip;
      const double upd = a[u] - rci * rj;
      a[u] = (i == c) ? ((j < c) ? 0.0 : (j == c ? piv : rj)) : ((i > c && j > c) ? upd : a[u]);
      const double yu = y[u] - rci * ycj;
      y[u] = (i == c) ? ycj : ((i > c) ? yu : y[u]);
    }
    if (l == 0) dead[16 * K + c] = dd;
    wave_lds_sync();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = l + 64 * u;
    D[(e >> 4) * SS + j] = a[u];
    Xd[j * SS + (e >> 4)] = y[u];
  }
  wave_lds_sync();
}

template <int LP>
__device__ void chol_inv_blocked(double *A, double *X, const double *thr, int *dead, double *Tmp) {
  constexpr int NB = LP / 16, SS = LP + 1;
  const int t = threadIdx.x, w = t >> 6;
  for (int e = t; e < LP * LP; e += kThreads) X[(e / LP) * SS + (e % LP)] = 0.0;
  __syncthreads();
#pragma unroll 1
  for (int K = 0; K < NB; ++K) {
    if (w == 0) {
      diag_cholinv16(A, SS, K, thr, dead, X, Tmp);
    }
    __syncthreads();
    // block row: R_KJ = X_KK^T A_KJ
    const int J = K + 1 + w;
    if (J < NB) {
      v4d Dm = v4d{0.0, 0.0, 0.0, 0.0};
      Dm = tile_mm<true>(X + 16 * K * SS + 16 * K, SS, A + 16 * K * SS + 16 * J, SS, Dm);
      tile_store(A + 16 * K * SS + 16 * J, SS, Dm, 1.0);
    }
    __syncthreads();
    // trailing update: A_JJ' -= R_KJ^T R_KJ' for K < J <= J'
    const int m = NB - K - 1;
    const int npair = m * (m + 1) / 2;
    for (int pi = w; pi < npair; pi += 4) {
      int u = pi, a = 0;
      while (u >= m - a) {
        u -= m - a;
        ++a;
      }
      const int Jr = K + 1 + a, Jc = Jr + u;
      v4d Dm = tile_load(A + 16 * Jr * SS + 16 * Jc, SS);
      v4d Pm = v4d{0.0, 0.0, 0.0, 0.0};
      Pm = tile_mm<true>(A + 16 * K * SS + 16 * Jr, SS, A + 16 * K * SS + 16 * Jc, SS, Pm);
      tile_store(A + 16 * Jr * SS + 16 * Jc, SS, Dm - Pm, 1.0);
    }
    __syncthreads();
  }
  // inverse by block diagonals: X_KJ = -X_KK sum_{K < L <= J} R_KL X_LJ
  double *Tw = Tmp + w * 16 * 17;
#pragma unroll 1
  for (int d = 1; d < NB; ++d) {
    const int K = w, J = w + d;
    if (J < NB) {
      v4d S = v4d{0.0, 0.0, 0.0, 0.0};
      for (int L = K + 1; L <= J; ++L)
        S = tile_mm<false>(A + 16 * K * SS + 16 * L, SS, X + 16 * L * SS + 16 * J, SS, S);
      tile_store(Tw, 17, S, 1.0);
      wave_lds_sync();
      v4d Y = v4d{0.0, 0.0, 0.0, 0.0};
      Y = tile_mm<false>(X + 16 * K * SS + 16 * K, SS, Tw, 17, Y);
      tile_store(X + 16 * K * SS + 16 * J, SS, Y, -1.0);
    }
    __syncthreads();
  }
}

// reduced slots: red[0] = P, red[1] = C, red[2] = G2 (upper tiles), red[3] =
// G3 (upper tiles); scr = R1, R1^-1, T
template <int LP>
__global__ __launch_bounds__(kThreads) void bs_small1(const BJobDesc *__restrict__ jobs,
                                                      StepClock clock) {
  constexpr int NT = LP / 16, L2 = LP * LP, SS = LP + 1;
  __shared__ double Pm[LP * SS], Cm[LP * SS], As[LP * SS], Xs[LP * SS];
  __shared__ double Tmp[4 * 16 * 17];
  __shared__ int dead[kBlockMaxLp];
  __shared__ double thr[kBlockMaxLp];
  const BJobDesc &J = jobs[blockIdx.x];
  if (J.Lp != LP) return;
  const int k = (int)(sclock(clock) - J.start_clock);
  if (k >= J.Kstop) return;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, rl = l & 15, q = l >> 4;
  const bool act = w < NT;
  const GLB double *red = gp(J.red);
  glb_to_lds<LP>(red, Pm, false);
  glb_to_lds<LP>(red + L2, Cm, false);
  v4d D[4];
  if (act)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) D[tj][v] = gram_sym(red + 2 * L2, LP, 16 * w + q + 4 * v, 16 * tj + rl);
  __syncthreads();
  // Deflation test of column c: its part outside the span of Q_k and of the
  // earlier columns is below kDeflTol times its own norm ||w'_c|| (the norm
  // before the projection, ||P(:, c)||^2 + G2(c, c)), or below 1e-14 ||A^T A||.
  if (t < LP) {
    double own = gram_sym(red + 2 * L2, LP, t, t);
    for (int i = 0; i < LP; ++i) own = fma(Pm[i * SS + t], Pm[i * SS + t], own);
    const double flo = (1e-14 * J.dscale) * (1e-14 * J.dscale);
    thr[t] = fmax(kDeflTol * kDeflTol * own, flo);
  }
  {
    GLB double *Ak = gp(J.Ah) + (int64_t)k * L2, *Pk = gp(J.Ph) + (int64_t)k * L2;
    for (int e = t; e < L2; e += kThreads) {
      const int r = e / LP, c = e - r * LP;
      Ak[e] = 0.5 * (Pm[r * SS + c] + Pm[c * SS + r]);
      Pk[e] = Pm[r * SS + c];  // for beta of the second pass
    }
    mm_lds<LP, true>(Cm, Cm, -1.0, D);  // G2 - C^T C
  }
  regs_to_lds<LP>(D, As);
  __syncthreads();
  chol_inv_blocked<LP>(As, Xs, thr, dead, Tmp);
  // a step marked robust (flags[3], set by the host) leaves the new block to a
  // Householder QR after gamma: M = I, N = C make gamma write W3 = W2 - Q_k C
  const bool robust = gp(J.flags)[3] != 0;
  // one-pass test: rho = ||R1||_F ||R1^-1||_F / Lp, sums in a fixed order
  __shared__ int one_pass;
  {
    double sr = 0.0, sx = 0.0;
    for (int e = t; e < L2; e += kThreads) {
      const int r = e / LP, c = e - r * LP;
      const double a = ((r >> 4) < (c >> 4) || ((r >> 4) == (c >> 4) && c >= r)) ? As[r * SS + c] : 0.0;
      const double x = Xs[r * SS + c];
      sr = fma(a, a, sr);
      sx = fma(x, x, sx);
    }
    Tmp[t] = sr;
    Tmp[kThreads + t] = sx;
    __syncthreads();
    if (w == 0) {
      // four partial sums per lane, then a butterfly over the wave (fixed order)
      double a = (Tmp[l] + Tmp[l + 64]) + (Tmp[l + 128] + Tmp[l + 192]);
      double x = (Tmp[kThreads + l] + Tmp[kThreads + l + 64]) + (Tmp[kThreads + l + 128] + Tmp[kThreads + l + 192]);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        a += __shfl_xor(a, o);
        x += __shfl_xor(x, o);
      }
      const bool anydead = __any(l < LP && dead[l] != 0);
      if (l == 0) {
        const int op = (robust || (!anydead && sqrt(a * x) <= J.onepass_rho * LP)) ? 1 : 0;
        one_pass = op;
        gp(J.flags)[1] = op;
        if (op) gp(J.flags)[0] = 0;
        gp(J.flags)[2] += (op && !robust) ? 1 : 0;  // one-pass Cholesky QR steps of this round
      }
    }
    __syncthreads();
  }
  const bool op = one_pass != 0;
  GLB double *R1 = gp(J.scr), *R1i = R1 + L2, *T = R1 + 2 * L2;
  GLB double *Bn = gp(J.Bh) + (int64_t)(k + 1) * L2, *Mk = gp(J.Mh) + (int64_t)k * L2;
  for (int e = t; e < L2; e += kThreads) {
    const int r = e / LP, c = e - r * LP;
    const double rv = ((r >> 4) < (c >> 4) || ((r >> 4) == (c >> 4) && c >= r)) ? As[r * SS + c] : 0.0;
    R1[e] = rv;
    R1i[e] = Xs[r * SS + c];
    if (op) {
      if (!robust) Bn[e] = rv;
      Mk[e] = robust ? (r == c ? 1.0 : 0.0) : Xs[r * SS + c];
    }
  }
  if (robust) {
    GLB double *Nk = gp(J.Nh) + (int64_t)k * L2;
    for (int e = t; e < L2; e += kThreads) Nk[e] = Cm[(e / LP) * SS + (e % LP)];
  }
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) D[tj] = v4d{0.0, 0.0, 0.0, 0.0};
    mm_lds<LP, false>(Cm, Xs, 1.0, D);  // T = C R1^-1
  }
  regs_to_glb<LP>(D, T);
  if (op && !robust) regs_to_glb<LP>(D, gp(J.Nh) + (int64_t)k * L2);
}

template <int LP>
__global__ __launch_bounds__(kThreads) void bs_small2(const BJobDesc *__restrict__ jobs,
                                                      StepClock clock) {
  constexpr int NT = LP / 16, L2 = LP * LP, SS = LP + 1;
  __shared__ double As[LP * SS], Xs[LP * SS], Os[LP * SS];
  __shared__ double Tmp[4 * 16 * 17];
  __shared__ int dead[kBlockMaxLp];
  __shared__ double thr[kBlockMaxLp];
  const BJobDesc &J = jobs[blockIdx.x];
  if (J.Lp != LP) return;
  const int k = (int)(sclock(clock) - J.start_clock);
  if (k >= J.Kstop) return;
  if (gp(J.flags)[1]) return;  // one-pass step: small1 wrote M, N and B
  const int t = threadIdx.x, w = t >> 6;
  const bool act = w < NT;
  const GLB double *red = gp(J.red);
  const GLB double *R1 = gp(J.scr), *R1i = R1 + L2, *T = R1 + 2 * L2;
  {
    constexpr int IT = (L2 + kThreads - 1) / kThreads;
    double gv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      gv[it] = (e < L2) ? gram_sym(red + 3 * L2, LP, e / LP, e % LP) : 0.0;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = t + it * kThreads;
      if (e < L2) As[(e / LP) * SS + (e % LP)] = gv[it];
    }
  }
  if (t < LP) thr[t] = kDeflTol * kDeflTol * gram_sym(red + 3 * L2, LP, t, t);
  __syncthreads();
  chol_inv_blocked<LP>(As, Xs, thr, dead, Tmp);
  if (t == 0) {
    int nd = 0;
    for (int c = 0; c < LP; ++c) nd += dead[c];
    gp(J.flags)[0] = nd;
  }
  // R2 with zero lower part, for B = R2 R1
  for (int e = t; e < L2; e += kThreads) {
    const int r = e / LP, c = e - r * LP;
    if (!((r >> 4) < (c >> 4) || ((r >> 4) == (c >> 4) && c >= r))) As[r * SS + c] = 0.0;
  }
  glb_to_lds<LP>(R1i, Os, false);
  __syncthreads();
  v4d E[4];
  // M = R1^-1 R2^-1
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) E[tj] = v4d{0.0, 0.0, 0.0, 0.0};
    mm_lds<LP, false>(Os, Xs, 1.0, E);
  }
  regs_to_glb<LP>(E, gp(J.Mh) + (int64_t)k * L2);
  __syncthreads();
  {
    // N = T R2^-1
    glb_to_lds<LP>(T, Os, false);
    __syncthreads();
    if (act) {
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) E[tj] = v4d{0.0, 0.0, 0.0, 0.0};
      mm_lds<LP, false>(Os, Xs, 1.0, E);
    }
    regs_to_glb<LP>(E, gp(J.Nh) + (int64_t)k * L2);
    __syncthreads();
  }
  // B_{k+1} = R2 R1
  glb_to_lds<LP>(R1, Os, false);
  __syncthreads();
  if (act) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) E[tj] = v4d{0.0, 0.0, 0.0, 0.0};
    mm_lds<LP, false>(As, Os, 1.0, E);
  }
  regs_to_glb<LP>(E, gp(J.Bh) + (int64_t)(k + 1) * L2);
}

// ---------------------------------------------------------------- launchers
// one launch per block width present in the batch (blocks of jobs of another
// width return at once)
hipError_t launch_bs_tall(const BBatch &b, int mode, int grams, hipStream_t st) {
  // alpha and beta: wave-local Gram products (beta at Lp = 64 holds 26 Gram
  // tiles per wave: one wave per SIMD); gamma0: panels staged through LDS
#define CSVD_TALL(LPV)                                                                                           \
  if (mode == kTallAlpha)                                                                                        \
    hipLaunchKernelGGL((bs_tall_rg<LPV, kTallAlpha, 512>), dim3(b.totalr), dim3(512), 0, st, b.jobs, b.njob,     \
                       b.toffr, step_clock(b), grams);                                                                 \
  else if (mode == kTallBeta)                                                                                    \
    hipLaunchKernelGGL((bs_tall_rg<LPV, kTallBeta, (LPV == 64 ? 256 : 512)>), dim3(b.totalr),                    \
                       dim3(LPV == 64 ? 256 : 512), 0, st, b.jobs, b.njob, b.toffr, step_clock(b), grams);             \
  else                                                                                                           \
    hipLaunchKernelGGL(bs_gamma0<LPV>, dim3(b.totalr), dim3(kTallThreads), 0, st, b.jobs, b.njob, b.toffr,       \
                       step_clock(b));
  if (b.lpmask & 1) CSVD_TALL(16)
  if (b.lpmask & 2) CSVD_TALL(32)
  if (b.lpmask & 4) CSVD_TALL(64)
#undef CSVD_TALL
  return hipGetLastError();
}

hipError_t launch_bs_gamma(const BBatch &b, hipStream_t st) {
  if (b.lpmask & 1)
    hipLaunchKernelGGL(bs_gamma<16>, dim3(b.totalr), dim3(kTallThreads), 0, st, b.jobs, b.njob, b.toffr, step_clock(b));
  if (b.lpmask & 2)
    hipLaunchKernelGGL(bs_gamma<32>, dim3(b.totalr), dim3(kTallThreads), 0, st, b.jobs, b.njob, b.toffr, step_clock(b));
  if (b.lpmask & 4)
    hipLaunchKernelGGL(bs_gamma<64>, dim3(b.totalr), dim3(kTallThreads), 0, st, b.jobs, b.njob, b.toffr, step_clock(b));
  return hipGetLastError();
}

hipError_t launch_bs_reduce(const BBatch &b, int m0, int nm, int d0, int second, hipStream_t st) {
  hipLaunchKernelGGL(bs_reduce, dim3(b.njob, 2 * kBlockMaxLp * kBlockMaxLp / 32), dim3(kThreads), 0, st, b.jobs,
                     step_clock(b), m0, nm, d0, second);
  return hipGetLastError();
}

hipError_t launch_bs_small1(const BBatch &b, hipStream_t st) {
  if (b.lpmask & 1) hipLaunchKernelGGL(bs_small1<16>, dim3(b.njob), dim3(kThreads), 0, st, b.jobs, step_clock(b));
  if (b.lpmask & 2) hipLaunchKernelGGL(bs_small1<32>, dim3(b.njob), dim3(kThreads), 0, st, b.jobs, step_clock(b));
  if (b.lpmask & 4) hipLaunchKernelGGL(bs_small1<64>, dim3(b.njob), dim3(kThreads), 0, st, b.jobs, step_clock(b));
  return hipGetLastError();
}

hipError_t launch_bs_small2(const BBatch &b, hipStream_t st) {
  if (b.lpmask & 1) hipLaunchKernelGGL(bs_small2<16>, dim3(b.njob), dim3(kThreads), 0, st, b.jobs, step_clock(b));
  if (b.lpmask & 2) hipLaunchKernelGGL(bs_small2<32>, dim3(b.njob), dim3(kThreads), 0, st, b.jobs, step_clock(b));
  if (b.lpmask & 4) hipLaunchKernelGGL(bs_small2<64>, dim3(b.njob), dim3(kThreads), 0, st, b.jobs, step_clock(b));
  return hipGetLastError();
}

}  // namespace csvd
