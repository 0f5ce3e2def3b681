// Internal declarations shared by the host orchestration (csvd.cpp,
// engine.cpp) and the gfx950 kernels (k_*.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/csvd.h"

namespace csvd {

// ----------------------------------------------------------------------------
// Launch-shape constants
constexpr int kThreads = 256;        // threads per block for the vector kernels
constexpr int kMaxLp = 256;          // widest Lanczos block (padded L)
constexpr int kMaxWindow = 64;       // longest basis window
constexpr int kMaxShifts = 64;       // N/2 upper bound (N <= 128)
constexpr int kRowPad = 64;          // column-major arrays pad rows to this

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Pointers loaded from a descriptor in memory are generic (flat) to the
// compiler; casting them to the global address space lets it emit global
// loads/stores (no LDS-aperture checks, no lgkmcnt coupling of the waits).
#if defined(__HIP_DEVICE_COMPILE__)
#define GLB __attribute__((address_space(1)))
#else
#define GLB
#endif
template <class T>
__host__ __device__ __forceinline__ GLB T *gp(T *p) {
  return (GLB T *)p;
}

// ----------------------------------------------------------------------------
// A device Lanczos job: one problem (matrix + block of L right-hand sides)
// advanced by the batched kernels.  All pointers are device pointers.  The
// descriptor is immutable while the job runs; the mutable per-step state
// lives in the arrays it points to.
struct JobDesc {
  // matrix A (m x n) and its transpose, CSR
  const int *rp, *ci;
  const double *va;
  const int *rpT, *ciT;
  const double *vaT;
  int m, n, Lp, lgLp, L, S, W, npad;
  int tiles1, tiles2;       // tiles of the A product (m rows) and A^T product (n rows)
  int G1, lgG1, E1, rpt1;   // A product: nnz split per row, slots per thread, rows per tile
  int G2, lgG2, E2, rpt2;   // A^T product: same
  int Sg, nsg;              // window update: shifts per block, shift groups
  int start_clock;          // engine clock value at which the job's step 0 runs
  double tol;               // per (shift, column) relative residual target
  // vectors
  double *u;                // m x Lp row-major: A v_k
  double *wring;            // 3 x (n x Lp) row-major: unnormalised Lanczos vectors
  double *win;              // W slots x Lp columns x npad rows: normalised v_i
  double2 *X, *P;           // S x Lp x npad complex: solutions and search vectors
  float2 *Xf, *Pf;          // FP32 variants (mixed precision), or null
  float *winf;              // FP32 window (mixed precision), or null
  double *part1, *part2;    // Lp x tiles partial sums (column-major over tiles)
  // per column state (Lp entries)
  double *beta0;            // ||V_in col||
  double *alpha;            // alpha_k of the current step
  double *coup;             // beta_k: coupling of v_k to v_{k-1} (0 at k = 0)
  double *inv_cur;          // 1 / ||w_k||  (0 for dead columns)
  double *inv_prev;         // 1 / ||w_{k-1}||
  double *nrm_hist;         // first kHist (alpha, beta) pairs of column 0 (norm estimate)
  // per (shift, column) state (S x Lp, index s * Lp + l)
  const double2 *shift;     // S shifts
  double2 *eta, *zeta;      // D-Lanczos pivots and solution coefficients
  int *done;                // 1 once the pair met tol
  int *conv_iter;           // step at which it did
  double *res;              // last residual estimate
  // window scalars: slot i (0..W-1): eta/zeta per pair, e per column
  double2 *w_eta, *w_zeta;  // W x S x Lp
  double *w_e;              // W x Lp
  int *skip_pair;           // S x Lp: pair finished before the current window
  // window coefficients (per window): index (l * S + s)
  double2 *cA, *cC;         // S*Lp
  double2 *cE, *cD;         // S*Lp*W
  int *active;              // [2] active pair counters (parity of the window)
};

constexpr int kHist = 128;

// ----------------------------------------------------------------------------
// A device block-Lanczos job.  One real block Lanczos process on A^T A of
// width Lp (the L right-hand sides plus seeded padding columns) serves every
// shift; the per-shift block LU of (z I - T_k) monitors convergence, and a
// second pass regenerates the basis to accumulate the moments.
struct BJobDesc {
  const int *rp, *ci;
  const double *va;
  const int *rpT, *ciT;
  const double *vaT;
  int m, n, Lp, lgLp, L, S, npad;
  int G1, lgG1, E1, rpt1, tiles1;  // tiling of the A product (m rows)
  int G2, lgG2, E2, rpt2, tiles2;  // tiling of the A^T product (n rows)
  int nchunk;                      // 64-row chunks of the tall kernels
  int nvb;                         // workgroups per tall kernel (each walks chunks vb, vb + nvb, ...)
  int nring;                       // slots of the basis ring
  int qC, qT;                      // basis table: Q_k at Qtab[(k / qC) mod qT] + (k mod qC) n Lp
  double *const *Qtab;             // qT block pointers (ring: one entry, the ring, qC = nring)
  int Kcap;                        // capacity of the per-step histories
  int Kstop;                       // steps of the current pass that do work (later steps are no-ops)
  int start_clock;                 // engine clock of step 0 of the current pass
  int Kmom;                        // moments accumulated in pass 2
  int cstride;                     // row stride of cmom (M + 1)
  double tol;
  double dscale;                   // ||A||^2 estimate: scale of the deflation test
  double onepass_rho;              // one Cholesky QR pass when rho <= this (0: always two)
  double *U;                       // m x Lp
  double *Q;                       // the ring: nring x (n x Lp)
  double *W;                       // n x Lp work block
  double *Vpad;                    // n x Lp: the padded starting block
  double *gpart;                   // nvb x 2 x Lp x Lp partial Gram matrices
  double *red;                     // 4 x Lp x Lp reduced Gram matrices (P, C, G2, G3)
  double *scr;                     // 3 x Lp x Lp: R1, R1^-1, T of the current step
  double *Ah, *Bh, *Mh, *Nh;       // (Kcap + 1) x Lp x Lp step histories
  double *Ph;                      // (Kcap + 1) x Lp x Lp: P = Q_k^T W' of each step (second pass)
  double2 *Hinv, *Zh;              // S x (Kcap + 1) x Lp x Lp
  double2 *ctmp;                   // S x 2 x Lp x Lp complex scratch
  double *res;                     // S x Lp residual estimates
  int *active;                     // unconverged (shift, column) pairs after the last step
  int *flags;                      // [0] deflated columns of the newest basis block
  const double2 *shift;            // S shifts
  const double2 *cmom;             // S x Kmom moment coefficients
  double *beta0;                   // Lp column norms of Vpad
  double *F;                       // Kcap x (Kmom L) x Lp moment coefficients (column-major per step)
  double *Sout;                    // npad x (Kmom L) column-major moments
  // mixed precision (CSVD_MIXED): the basis blocks for the moments are kept
  // as FP32 copies, block k at Q32tab[k / kStoreChunk] + (k mod kStoreChunk)
  // n Lp, while the recurrence reads its FP64 blocks from the ring
  float *const *Q32tab;
  int store32;                     // 1: gamma also writes the FP32 copy of Q_{k+1}
  // rows with more than tlong nonzeros (A product: side 1, A^T product:
  // side 2) are left out of the row tiles and split into segments of at
  // most tlong nonzeros [sgb, sge); each segment's partial row goes to sgp
  // (nseg x Lp) and the long row lrow[r] is the sum of its segments
  // lseg[r] .. lseg[r+1]-1 added in order
  int tlong;
  const int *sgb1, *sge1, *lrow1, *lseg1;
  const int *sgb2, *sge2, *lrow2, *lseg2;
  int nseg1, nlong1, nseg2, nlong2;
  double *sgp1, *sgp2;
  // column group of a wider right-hand side (L > kBlockMaxLp, solved as
  // independent groups of at most kBlockMaxLp columns): moment k of the
  // group's column l is column k sL + soff + l of Sout (sL = L, soff = 0
  // for a job that holds every column)
  int sL, soff;
};

constexpr int kStoreChunk = 64;  // basis blocks per allocation of a stored basis

// Q_k of a block job (ring slot, or the stored basis)
__device__ __forceinline__ GLB double *qblock(const BJobDesc &J, int k) {
  typedef GLB double *gptr;
  const GLB gptr *tab = (const GLB gptr *)(J.Qtab);
  return tab[(k / J.qC) % J.qT] + (int64_t)(k % J.qC) * J.n * J.Lp;
}

// FP32 copy of Q_k (mixed-precision stored basis)
__device__ __forceinline__ GLB float *q32block(const BJobDesc &J, int k) {
  typedef GLB float *gptr;
  const GLB gptr *tab = (const GLB gptr *)(J.Q32tab);
  return tab[k / kStoreChunk] + (int64_t)(k % kStoreChunk) * J.n * J.Lp;
}

struct BBatch {
  const BJobDesc *jobs;
  int njob;
  const int *toff1, *toff2, *toffr, *toffs;  // tiles of A, A^T, row chunks, shifts
  int total1, total2, totalr, totals;
  int lpmask;  // block widths present: bit 0 -> 16, bit 1 -> 32, bit 2 -> 64
  int64_t clock;  // engine step clock of the launches (step k of a job: clock - start_clock)
  // non-null: the step kernels read the clock from this device word instead
  // (a captured step graph, replayed at successive clocks; a tick kernel at
  // the end of the step advances it)
  const int64_t *clkp;
};

// The step clock a step kernel runs at: by value, or from device memory.
struct StepClock {
  int64_t value;
  const int64_t *ptr;
};
__device__ __forceinline__ int64_t sclock(const StepClock &c) { return c.ptr ? *c.ptr : c.value; }
inline StepClock step_clock(const BBatch &b) { return StepClock{b.clock, b.clkp}; }

constexpr int kBlockMaxLp = 64;   // widest block of the block Lanczos engine
constexpr int kBlockMinLp = 16;   // narrowest (MFMA tile width)
constexpr int kBlockPanel = 64;   // rows per chunk of the tall kernels
constexpr int kBlockMaxVB = 256;  // workgroups per job in the tall kernels
constexpr int kBlockPollSteps = 8;  // block steps between convergence polls
constexpr int kMomWindow = 16;   // second-pass steps per moment accumulation (basis ring = window + 2)
constexpr double kDeflTol = 1e-10;  // relative size below which a new basis direction is deflated
constexpr int kRobustSteps = 2;      // Householder-orthonormalised steps at the start of a round (rounds after
                                     // the first, a rank-deficient or nearly invariant starting block)
constexpr double kRankTol = 1e-6;    // min |R_ii| <= kRankTol max |R_ii| of the starting block: rank deficient
constexpr double kInvTol = 1e-4;     // first new block: a direction below kInvTol of its product (nearly invariant
                                     // start) or cond above 1 / kInvTol takes Householder steps
constexpr double kOnePassRho = 1.5;  // one Cholesky pass when ||R1||_F ||R1^-1||_F <= 1.5 Lp

hipError_t launch_b_spmm_a(const BBatch &b, hipStream_t st);
hipError_t launch_b_spmm_at(const BBatch &b, hipStream_t st);
// the long rows of one job's product at step k (side 1: U = A Q_k, side 2:
// W = A^T U): segment partial rows, then their sums in order
hipError_t launch_b_spmm_long(const BJobDesc &hj, int side, int k, hipStream_t st);
constexpr int kLongRow = 128;  // rows with more nonzeros are split into segments of this many
// S += sum_{b < T} Q_{k0+b} F_{k0+b} for one job: the basis blocks are read
// from the ring or the stored basis (its FP32 copies when hj.store32), F from
// the coefficient history
hipError_t launch_b_moments(const BJobDesc &hj, int k0, int T, hipStream_t st);
// FP32 copy of block kb of the basis (qblock -> q32block) of one job
hipError_t launch_b_store32(const BJobDesc &hj, int kb, hipStream_t st);
// Tall kernels of one block step (see k_bstep.hip).  mode 0 (alpha): W' =
// W - Q_{k-1} B_k^T and (grams = 1) the partial Gram matrix Q_k^T W'; mode 1
// (beta): partial Gram matrices of W2 = W' - Q_k P; mode 2 (gamma0): partial
// Gram matrix of Y = W' R1^-1 - Q_k T (skipped on one-pass steps).
// gamma: Q_{k+1} = W' M_k - Q_k N_k.
hipError_t launch_bs_tall(const BBatch &b, int mode, int grams, hipStream_t st);
hipError_t launch_bs_gamma(const BBatch &b, hipStream_t st);
// reduction of nm partial Gram matrices from slot m0 into red slots d0.. (fixed order)
hipError_t launch_bs_reduce(const BBatch &b, int m0, int nm, int d0, int second, hipStream_t st);
// small1: A_k, first Cholesky, R1^-1, T (and M_k, N_k, B_{k+1} on one-pass
// steps).  small2: second Cholesky, M_k, N_k, B_{k+1}
hipError_t launch_bs_small1(const BBatch &b, hipStream_t st);
hipError_t launch_bs_small2(const BBatch &b, hipStream_t st);
hipError_t launch_b_shift(const BBatch &b, int init, hipStream_t st);
hipError_t launch_b_backsolve(const BJobDesc &hj, int K, hipStream_t st);
hipError_t launch_b_fcoef(const BJobDesc &hj, int K, hipStream_t st);
// counters of every job of the batch after its newest step into pinned host
// memory (part 0: active count, on the stream of the shift recurrences;
// part 1: flags[0..2], on the step stream)
hipError_t launch_b_snap(const BBatch &b, int part, int *host, hipStream_t st);
hipError_t launch_b_r0(const double *X, int64_t ld, int Lp, double *B, hipStream_t st);
// device step clock of captured steps: set to a value / advance by one
hipError_t launch_b_setclock(int64_t *clk, int64_t value, hipStream_t st);
hipError_t launch_b_tick(int64_t *clk, hipStream_t st);
hipError_t launch_b_eye(double *Z, int64_t ld, int64_t rows, int cols, hipStream_t st);

struct Ctx;  // defined in csvd.cpp

// ----------------------------------------------------------------------------
// Launchers (k_sparse.hip)
hipError_t launch_csr_transpose(int m, int n, int nnz, const int *rp, const int *ci, const double *va,
                                int *rpT, int *ciT, double *vaT, int *work, hipStream_t st);
hipError_t launch_spmm_rowmajor(int rows, int64_t k, const int *rp, const int *ci, const double *va,
                                const double *x, double *y, hipStream_t st);
hipError_t launch_col_to_row(int rows, int cols, const double *src, int64_t ld, double *dst,
                             int64_t dst_cols, hipStream_t st);
hipError_t launch_row_to_col(int rows, int cols, const double *src, int64_t src_cols, double *dst,
                             int64_t ld, hipStream_t st);
hipError_t launch_check_csr(int m, int n, const int *rp, const int *ci, const double *va, int nnz,
                            int *flags, hipStream_t st);

// Batched Lanczos stages (k_krylov.hip).  `jobs` is a device array of njob
// descriptors; `toff1`/`toff2`/`toffw` are device prefix offsets of the tiles
// of each job (njob + 1 entries) for the A product, the A^T product and the
// window update.
struct BatchLaunch {
  const JobDesc *jobs;
  int njob;
  const int *toff1, *toff2, *toffw, *toffc, *toffp;  // tile prefix tables
  int total1, total2, totalw, totalc, totalp;        // totals (host copies)
  const int64_t *clock;                      // device engine clock
  int *ticket;                               // device ticket counter for the clock
  int64_t *clock_mut;
  int Wmax;                                  // largest window of the batch
  int mixed;                                 // FP32 window / X / P
};

hipError_t launch_k1_spmm_alpha(const BatchLaunch &b, hipStream_t st);
hipError_t launch_r1_alpha(const BatchLaunch &b, hipStream_t st);
hipError_t launch_k2_spmm_lanczos(const BatchLaunch &b, hipStream_t st);
hipError_t launch_s2_step(const BatchLaunch &b, hipStream_t st);
hipError_t launch_window_coef(const BatchLaunch &b, int wlen, int parity, hipStream_t st);
hipError_t launch_window_apply(const BatchLaunch &b, int wlen, hipStream_t st);
// Job initialisation: ring[0] <- V (column-major n x L, ld n), norms, state.
hipError_t launch_job_init(const JobDesc &hj, const double *Vcol, int64_t ldv, hipStream_t st);
// Moments S_k (k = 0..K-1) of one job, column-major n x (K*L), ld npad.
hipError_t launch_moments(const JobDesc &hj, const double2 *coef, int K, double *out, hipStream_t st);
// Copy shift solution j of a job into column-major re/im arrays (n x L, ld n).
hipError_t launch_get_solution(const JobDesc &hj, int j, double *re, double *im, hipStream_t st);
hipError_t launch_zero(double *p, int64_t count, hipStream_t st);

// Dense FP64 kernels (k_dense.hip).  Column-major storage.
hipError_t launch_hh_make(double *X, int64_t ld, int rows, int j, double *tau, hipStream_t st);
hipError_t launch_hh_step(double *X, int64_t ld, int rows, int cols, int j, double *tau, hipStream_t st);
hipError_t launch_hh_apply(const double *Xr, int64_t ldr, int rows, int j, const double *tau, double *Z,
                           int64_t ldz, int zcols, hipStream_t st);
hipError_t launch_jacobi_step(double *A, int64_t lda, int rows, int cols_even, double *V, int64_t ldv,
                              int vrows, int step, double tol, double floor2, int *counter, hipStream_t st);
// Block-pair Jacobi (k_dense.hip): columns in blocks of jacobi_block_width(n)
// (0: use the per-column kernel); ncol must be jacobi_padded_cols(n), rows
// and vrows at most 4096 / width; one sweep is steps 0 .. ncol / width - 2.
int jacobi_block_width(int n);
int jacobi_padded_cols(int n);
hipError_t launch_jacobi_blk(double *A, int64_t lda, int rows, int ncol, double *V, int64_t ldv, int vrows, int step,
                             double tol, double floor2, int *counter, hipStream_t st);
constexpr int kHB = 32;  // panel width of the blocked Householder QR
// workspace (doubles) of the blocked QR of a rows x cols matrix: partial sums,
// W, V^T V and the T factors of every panel (kept for hh_apply_blocked)
size_t hh_blocked_ws_doubles(int cols);
// blocked Householder QR in place (R on and above the diagonal, reflectors
// below, tau); ws: hh_blocked_ws_doubles(cols) doubles, keeps the T factors
hipError_t hh_qr_blocked(double *X, int64_t ld, int rows, int cols, double *tau, double *ws, hipStream_t st);
// Z <- Q Z with the reflectors and T factors of hh_qr_blocked (ws of the QR,
// read only); ws_rw: hh_blocked_ws_doubles(ncols) doubles of scratch
hipError_t hh_apply_blocked(const double *X, int64_t ld, int rows, int nref, const double *ws, double *Z,
                            int64_t ldz, int ncols, double *ws_rw, hipStream_t st);
hipError_t launch_col_norms(const double *A, int64_t lda, int rows, int cols, double *out, hipStream_t st);
hipError_t launch_copy_block(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows, int cols,
                             hipStream_t st);
hipError_t launch_gemm(int R, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double beta, double *C, int64_t ldc, hipStream_t st);
// same with A stored transposed (element (r, k) at A[r * lda + k])
hipError_t launch_gemm_ta(int R, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                          int64_t ldb, double beta, double *C, int64_t ldc, hipStream_t st);
hipError_t launch_scale_cols(double *A, int64_t lda, int rows, int cols, const double *s, hipStream_t st);
hipError_t launch_sign_fix(double *U, int64_t ldu, int urows, double *V, int64_t ldv, int vrows, int cols,
                           hipStream_t st);
// Per-column sum of squares of (X - Y diag(s)), X row-major (rows x cols),
// Y column-major (ld).  Writes one value per column (deterministic order).
hipError_t launch_resid_cols(const double *X, const double *Y, int64_t ldy, const double *s, int rows,
                             int cols, double *out, hipStream_t st);

}  // namespace csvd
