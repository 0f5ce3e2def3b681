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
                              int vrows, int step, double tol, int *counter, hipStream_t st);
hipError_t launch_col_norms(const double *A, int64_t lda, int rows, int cols, double *out, hipStream_t st);
hipError_t launch_gemm(int R, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double beta, double *C, int64_t ldc, hipStream_t st);
hipError_t launch_scale_cols(double *A, int64_t lda, int rows, int cols, const double *s, hipStream_t st);
hipError_t launch_sign_fix(double *U, int64_t ldu, int urows, double *V, int64_t ldv, int vrows, int cols,
                           hipStream_t st);
// Per-column sum of squares of (X - Y diag(s)), X row-major (rows x cols),
// Y column-major (ld).  Writes one value per column (deterministic order).
hipError_t launch_resid_cols(const double *X, const double *Y, int64_t ldy, const double *s, int rows,
                             int cols, double *out, hipStream_t st);

}  // namespace csvd
