/*
 * csvd.h -- C ABI of the MI355X interior singular triplet solver.
 *
 * Problem (Imakura & Sakurai, Sec. 1, eq. psvd): given a real sparse
 * A (m x n, m >= n) and an interval [a, b] with 0 <= a < b, compute the
 * singular triplets (sigma_i, u_i, v_i) with a <= sigma_i <= b.
 *
 * Method: the block SS-SVD method (Algorithm 1) and its variant with the
 * nonlinear transformation g(t) = exp(t) (Algorithm 2):
 *   steps 1-2  shifted block solves (shift_j I - A^T A) Y_j = V, j = 1..N/2,
 *              and moment sums S_k = 2 sum_j Re(c_jk Y_j)   (Sec. 3.1)
 *   step 3     low-rank approximation of S-hat = [S_0 .. S_{M-1}], V~ = U_S1
 *   step 4     [U~, B] = qr(A V~)
 *   step 5     SVD of B = P Phi Q^T, triplets (phi_i, U~ p_i, V~ q_i)
 * with the ellipse quadrature of Sec. 4 and the spurious index of Sec. 3.4.2.
 *
 * Conventions for every call:
 *   - returns an int status: CSVD_OK (0) or a negative CSVD_E* code;
 *   - no exception crosses the ABI; after an error the context stays usable
 *     and csvd_last_error() describes the failure;
 *   - dense host arrays are column-major (Fortran order) float64;
 *   - one context is used by one host thread at a time, and holds one solve at
 *     a time: while a server request on it is queued or running, or a batch
 *     runs it, every other call that solves on it or reads its results
 *     returns CSVD_ESTATE (a batch rejects a context listed twice with
 *     CSVD_EINVAL);
 *   - all device work runs on the HIP stream given at csvd_create (NULL means
 *     the default stream); calls return after that work has completed.
 */
#ifndef CSVD_H
#define CSVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csvd_ctx csvd_ctx;

enum {
  CSVD_OK = 0,
  CSVD_EINVAL = -1,     /* invalid argument (message says which)                 */
  CSVD_ENOMEM = -2,     /* device or host allocation failed                      */
  CSVD_ENOTCONV = -3,   /* shifted solves hit max_iters before solve_rtol, or a   */
                        /* dense SVD of step 3 or 5 reached its sweep limit;      */
                        /* triplets were still extracted and can be read          */
  CSVD_EDEVICE = -4,    /* a HIP runtime call failed                             */
  CSVD_ESTATE = -5,     /* call out of order (e.g. triplets before a solve)      */
  CSVD_ENUMERIC = -6    /* non-finite value met in the input or the computation  */
};

enum { CSVD_PLAIN = 0, CSVD_EXP = 1 };      /* Algorithm 1 / Algorithm 2 (g = exp)   */
enum { CSVD_FP64 = 0, CSVD_MIXED = 1 };     /* see csvd_params.precision             */

/* Parameters of Algorithms 1 and 2 (inputs listed in both algorithms) plus
 * the solver controls of this implementation. */
typedef struct {
  int32_t L;              /* columns of V_in, 1..256                                    */
  int32_t M;              /* number of moments, >= 1, with L*M <= n                     */
  int32_t N;              /* quadrature points on the full contour, even, >= 2          */
  int32_t ell;            /* iteration count of eq. iter1/iter2, >= 1 (paper: 1)         */
  double  delta;          /* low-rank threshold of step 3, relative to the largest      */
                          /* singular value of S-hat (paper: 1e-20)                     */
  double  alpha;          /* ellipse aspect ratio (paper: 0.1)                          */
  int32_t transform;      /* CSVD_PLAIN or CSVD_EXP (EXP requires a > 0)                */
  int32_t precision;      /* CSVD_FP64: everything in FP64.  CSVD_MIXED: the Krylov      */
                          /* bulk is stored in FP32 while the recurrence, the sparse    */
                          /* products, the block orthogonalisation and steps 3-5 stay   */
                          /* FP64.  Block solver: the basis kept for the moments holds  */
                          /* FP32 copies of the blocks (half the memory of keep_basis,  */
                          /* so larger problems avoid the second pass); a solve whose   */
                          /* triplets miss 1e-6 is refined by accumulating the moments  */
                          /* again from the basis regenerated in FP64 (csvd_info.       */
                          /* mixed_refined); csvd_solve_batch and served block solves   */
                          /* keep FP64 bases.                                           */
                          /* Per-column solver: the per-shift solution/search vectors   */
                          /* and the window basis are FP32.  Target residual 1e-6       */
  double  solve_rtol;     /* per (shift, column) stop: ||V - (z I - A^T A) Y|| / ||V||     */
  int32_t max_iters;      /* Lanczos step cap per round; reaching it -> CSVD_ENOTCONV     */
  double  spurious_eps;   /* drop a triplet when tau_i < eps * sigma_S,1 (Sec. 3.4.2)   */
  uint64_t seed;          /* V_in ~ N(0,1) from this seed when V_in == NULL              */
  double  norm_a;         /* ||A||_2 if known (> 0); 0 -> estimated from the Lanczos     */
                          /* tridiagonal; used to make residuals relative                */
  int32_t window;         /* Lanczos steps per basis window, 1..64 (0 -> automatic)      */
  int32_t check_solves;   /* 1: compute the true FP64 residual of every shifted solve    */
                          /* (per-column solver; the block solver keeps no per-shift    */
                          /* solutions and reports NaN)                                  */
  int32_t solver;         /* CSVD_SOLVER_BLOCK: one block Lanczos basis of width L (padded */
                          /* to a power of two <= 64) for all shifts; a wider L runs as   */
                          /* independent groups of <= 64 columns stepped together        */
                          /* (csvd_solve_interval only; batches and servers need L <= 64) */
                          /* CSVD_SOLVER_SINGLE: one Lanczos basis per column with        */
                          /* windowed per-shift updates (any L <= 256);                    */
                          /* CSVD_SOLVER_AUTO: BLOCK when it applies and n >= 64 x padded  */
                          /* L (smaller matrices exhaust the block space in a few steps), */
                          /* else SINGLE                                                  */
  int32_t keep_basis;     /* block solver: 1 keeps the whole basis in device memory while */
                          /* it fits (leaving 8 GB free), so the moments need no second   */
                          /* pass; 0 always regenerates it in a second pass; k >= 2 keeps */
                          /* at most k blocks and, past them, goes on with the ring and a */
                          /* second pass (memory is taken in chunks of 64 blocks, so up   */
                          /* to k rounded up to 64).  All give the same bits.  A served   */
                          /* request keeps it only when its largest size also fits the   */
                          /* server's budget                                              */
  int32_t cholqr_passes;  /* block solver: 0 (default) orthonormalises a new basis block  */
                          /* with one Cholesky QR pass when the first factor R1 is well   */
                          /* conditioned (||R1||_F ||R1^-1||_F <= 1.5 Lp, no deflated    */
                          /* column) and with two otherwise; 2 always uses two passes     */
  double  resid_target;   /* > 0: triplets whose relative residual exceeds this are not   */
                          /* returned; csvd_info.dropped counts them and the solve        */
                          /* returns CSVD_ENOTCONV.  0 (default): every triplet in [a, b] */
                          /* that passes the spurious test is returned (Algorithm 1)     */
  int32_t ell_adaptive;   /* 1: steps 3-5 run after every round of eq. iter1/iter2, and a */
                          /* further round (from that round's S_0, at most ell rounds in  */
                          /* all) runs only while some triplet's relative residual       */
                          /* exceeds resid_target, which must then be > 0; every round   */
                          /* accumulates all M+1 moments.  0 (default): exactly ell      */
                          /* rounds, steps 3-5 after the last                            */
} csvd_params;

enum { CSVD_SOLVER_AUTO = 0, CSVD_SOLVER_BLOCK = 1, CSVD_SOLVER_SINGLE = 2 };

/* Fills *p with the paper's defaults: L=16, M=8, N=32, ell=1, delta=1e-20,
 * alpha=0.1, PLAIN, FP64, solve_rtol=1e-10, max_iters=1000000,
 * spurious_eps=1e-12, seed=2109, norm_a=0, window=0, check_solves=0,
 * solver=CSVD_SOLVER_AUTO, keep_basis=1, cholqr_passes=0, resid_target=0,
 * ell_adaptive=0. */
int csvd_params_default(csvd_params *p);

/* Creates a context holding a device copy of A in CSR form (and of A^T,
 * built on the device).
 *   rowptr [m+1], colidx [nnz] (sorted within each row), vals [nnz].
 *   on_device = 0: the three arrays are host memory; 1: device memory.
 *   The caller keeps ownership of its arrays and may free them on return.
 *   hip_stream: a hipStream_t (or NULL for the default stream).
 * Errors: CSVD_EINVAL for m < n, n < 1, malformed CSR (non-monotone rowptr,
 * column out of range or unsorted, nnz >= 2^31); CSVD_ENUMERIC for a
 * non-finite value; CSVD_ENOMEM / CSVD_EDEVICE from the runtime. */
int csvd_create(csvd_ctx **ctx, int64_t m, int64_t n, int64_t nnz,
                const int32_t *rowptr, const int32_t *colidx, const double *vals,
                int32_t on_device, void *hip_stream);

/* Runs Algorithm 1 (PLAIN) or Algorithm 2 (EXP) for the interval [a, b].
 *   V_in: n x L column-major host array, or NULL to draw N(0,1) from p->seed.
 * The context keeps the triplets and the moments until the next solve.
 * Returns CSVD_OK, CSVD_ENOTCONV (triplets still available), or an error. */
int csvd_solve_interval(csvd_ctx *ctx, double a, double b, const csvd_params *p,
                        const double *V_in);

/* Copies the triplets of the last solve, ascending sigma.  Call with
 * capacity = 0 to query *t_hat.  capacity < t_hat -> CSVD_EINVAL (t_hat
 * set).  Any of sigma/U/V/resid may be NULL.  U: m x capacity column-major,
 * V: n x capacity, resid: max(||A v - s u||, ||A^T u - s v||) / ||A||_2.
 * Sign convention: the largest-magnitude entry of each v is positive. */
int csvd_get_triplets(csvd_ctx *ctx, int64_t *t_hat, int64_t capacity,
                      double *sigma, double *U, double *V, double *resid);

/* Residual estimates of the last solve (Sec. 3.4.1), one per triplet in the
 * order of csvd_get_triplets, relative to ||A||_2 like its resid: the norm
 * ||A^T u_i - s_i v_i|| computed from the moments without a product with A,
 *   CSVD_PLAIN (eq. residual):  || S_+ W_S1 Sigma_S1^-1 q_i - s_i^2 U_S1 q_i || / s_i,
 *     S_+ = [S_1 .. S_M], U_S1, Sigma_S1, W_S1 from the low-rank step, q_i the
 *     i-th right singular vector of B (step 5);
 *   CSVD_EXP (eq. res_nonlinear): the same with log(s_i^2) in place of s_i^2,
 *     times mu = ||r_i'|| / ||r~_i'|| taken from the triplet i' with the
 *     largest computed residual ||A^T u - s v||.
 * capacity >= t_hat (CSVD_EINVAL otherwise); CSVD_ESTATE before a solve. */
int csvd_get_residual_estimates(csvd_ctx *ctx, int64_t capacity, double *est);

/* Summary of the last solve. */
typedef struct {
  int64_t iterations;        /* Lanczos steps of the last round                      */
  int64_t iterations_total;  /* over all ell rounds                                  */
  int32_t rank;              /* r kept by the low-rank step                           */
  int32_t t_hat;             /* triplets returned                                     */
  int32_t converged;         /* 1 if every (shift, column) met solve_rtol              */
  int32_t n_shift;           /* N/2                                                   */
  double  max_solve_resid_est;  /* largest Lanczos residual estimate at exit          */
  double  max_solve_resid_true; /* largest true FP64 solve residual (check_solves)    */
  double  max_triplet_resid;    /* largest relative triplet residual                  */
  double  norm_a;            /* ||A||_2 used (given or estimated)                      */
  double  sigma_s1;          /* largest singular value of S-hat                        */
  double  t_solve_ms;        /* steps 1-2 (solves + moments)                           */
  double  t_lowrank_ms;      /* step 3                                                */
  double  t_qr_ms;           /* step 4                                                */
  double  t_extract_ms;      /* step 5 + residuals                                    */
  double  t_total_ms;
  double  spmm_a_ms;         /* average duration of one A-product launch (sampled)     */
  double  spmm_at_ms;        /* average duration of one A^T-product launch (sampled)   */
  double  window_ms;         /* average duration of one window-apply launch (sampled)  */
  int64_t spmm_samples;      /* launches behind the averages                           */
  double  spmm_a_bytes;      /* algorithmic bytes of one A-product launch              */
  double  spmm_at_bytes;     /* algorithmic bytes of one A^T-product launch            */
  double  window_bytes;      /* algorithmic bytes of one window-apply launch           */
  int32_t window;            /* Lanczos steps per window used (0: block solver)        */
  int32_t L_padded;          /* block width used on the device                         */
  int32_t solver;            /* solver that ran                                        */
  int32_t deflated;          /* basis directions dropped from the newest block (block solver) */
  double  rest_ms;           /* average duration of the rest of a block step (sampled) */
  int32_t basis_stored;      /* 1: the block basis was kept in device memory (no second */
                             /* pass); 0: regenerated, or the per-column solver          */
  int32_t one_pass_steps;    /* block steps of the last round whose basis block took one */
                             /* Cholesky QR pass (see csvd_params.cholqr_passes)         */
  double  moments_ms;        /* block solver: average duration of one moment launch     */
                             /* over 16 basis blocks (sampled)                          */
  int32_t svd_sweeps_exhausted; /* 1 if a one-sided Jacobi SVD of step 3 or 5 stopped at */
                             /* its limit of 60 sweeps (the solve returns CSVD_ENOTCONV) */
  int32_t column_groups;     /* block solver: independent column groups of at most 64     */
                             /* columns that L was split into (1 when L <= 64)            */
  int32_t mixed_refined;     /* CSVD_MIXED, block solver: 1 if the triplets from the FP32  */
                             /* stored basis missed the 1e-6 residual target and the      */
                             /* moments were accumulated again from the basis regenerated */
                             /* in FP64 (steps 3-5 then ran again)                         */
  int32_t dropped;           /* triplets not returned because their residual exceeded     */
                             /* csvd_params.resid_target                                   */
  double  mixed_resid_fp32;  /* CSVD_MIXED with an FP32 stored basis: the largest relative */
                             /* triplet residual of the result from the FP32 basis (before */
                             /* any refinement); 0 otherwise                               */
  int32_t rounds;            /* rounds of eq. iter1/iter2 that ran: ell, or fewer with    */
                             /* csvd_params.ell_adaptive                                  */
} csvd_info;

int csvd_get_info(csvd_ctx *ctx, csvd_info *info);

/* Copies moment k (0 <= k <= M) of the last solve, S_k (n x L, column-major).
 * S_M is the extra moment of Sec. 3.4.1 (also used to check Prop. 1). */
int csvd_get_moment(csvd_ctx *ctx, int32_t k, double *S_k);

/* Copies the solution of shift j (0 <= j < N/2) of the last round,
 * Y_j ~ (z_j I - A^T A)^{-1} V (n x L, real and imaginary parts). */
int csvd_get_solution(csvd_ctx *ctx, int32_t j, double *Y_re, double *Y_im);

/* Quadrature of Sec. 4 as used by the solver (upper-half points j = 1..N/2):
 * shifts (z_j or exp(t_j)), weights (omega_j or psi_j) and moment
 * coefficients c_jk = weight_j * point_j^k, k = 0..M, stored c[j*(M+1)+k].
 * Pure host computation; no context needed. */
int csvd_quadrature(double a, double b, const csvd_params *p,
                    double *shift_re, double *shift_im, double *w_re, double *w_im,
                    double *c_re, double *c_im);

/* Device sparse products with the context's matrix (host in, host out):
 *   transpose = 0: Y (m x k) = A X (n x k);  1: Y (n x k) = A^T X (m x k).
 * Column-major host arrays.  Used by tests and by callers that want the
 * operator alone. */
int csvd_spmm(csvd_ctx *ctx, int32_t transpose, int64_t k, const double *X, double *Y);

/* csvd_spmm for callers that cannot allocate device memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid
 * it): the same product with the same arguments and results, bit for bit,
 * but its staging blocks (X and Y in column- and row-major order) live in a
 * fixed device array of 32 MiB per GPU, held from the first call on that GPU
 * until the process ends.  Calls no hipMalloc/hipFree.
 * Limit: 2 k (rows of X + rows of Y) <= 4194304 doubles, else CSVD_EINVAL
 * with a message (the context stays usable).  The array is shared by every
 * call on the same GPU, so calls that overlap in time on one GPU (other host
 * threads, other contexts) race: serialise them. */
int csvd_spmm_noalloc(csvd_ctx *ctx, int32_t transpose, int64_t k, const double *X, double *Y);

/* Dense FP64 product on the matrix cores: C (R x N) = A (R x K) B (K x N),
 * column-major host arrays, computed on the device (the kernel that forms
 * V-hat = V~ Q_sel in step 5).  Needs no context. */
int csvd_dense_gemm(int64_t R, int64_t N, int64_t K, const double *A, const double *B, double *C);

/* Copies the device-built CSR of A^T (rowptr [n+1], colidx/vals [nnz]). */
int csvd_get_transpose(csvd_ctx *ctx, int32_t *rowptr, int32_t *colidx, double *vals);

/* Error text of the last failing call on ctx (never NULL). */
const char *csvd_last_error(const csvd_ctx *ctx);

/* Frees everything the context owns.  NULL is accepted. */
void csvd_destroy(csvd_ctx *ctx);

/* Frees the device memory kept between solves on the context's device: the
 * idle chunks of stored block bases (csvd_params.keep_basis), which the next
 * solve of the same size would reuse (a solve that needs room frees idle
 * chunks of other sizes by itself), and the context's workspace of the dense
 * steps 3-5.  Waits for the context's stream first.
 * Returns CSVD_OK, CSVD_EINVAL (NULL) or CSVD_EDEVICE. */
int csvd_trim(csvd_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Batched solves.  Runs independent (context, interval) problems together:
 * every Lanczos step of every problem is done by the same kernel launches
 * (one launch per stage covers all problems' rows and columns), so small
 * problems share the GPU instead of each being launch-latency bound.  Each
 * problem's arithmetic is the same as in a solo csvd_solve_interval call.
 *   ctxs[i], a[i], b[i], params[i], V_in[i] (V_in may be NULL or hold NULLs).
 *   status[i] receives the per-problem status; the call returns CSVD_OK when
 *   the batch ran (per-problem failures are in status[]).
 * All contexts must share the stream of ctxs[0]. */
int csvd_solve_batch(int32_t count, csvd_ctx *const *ctxs, const double *a, const double *b,
                     const csvd_params *params, const double *const *V_in, int32_t *status);

/* ---------------------------------------------------------------------------
 * Serving.  A server owns a continuous-batching loop: submitted requests are
 * admitted while their device footprint fits the HBM budget, join the
 * running batch at the next window boundary, and leave it when their solves
 * converge; their dense steps then run and the request is marked done.
 */
typedef struct csvd_server csvd_server;

/* budget_bytes: device memory the server may use for request state (the
 * matrices themselves live in their contexts).  max_batch: cap on
 * concurrently running requests.  The results a finished request leaves in
 * its context (moments, triplet vectors, epilogue buffers) are outside the
 * budget until csvd_trim or csvd_destroy; while other requests run, a
 * request is also admitted only when the device's free memory holds its
 * footprint and 2 GiB more, and a request that cannot get its memory ends
 * with CSVD_ENOMEM without stopping the others. */
int csvd_server_create(csvd_server **srv, int64_t budget_bytes, int32_t max_batch, void *hip_stream);

/* Queues a request.  The context must stay alive until the request is done.
 * V_in may be NULL (seeded).  Returns a request id >= 0 in *req.  A request
 * whose footprint alone exceeds the budget is rejected with CSVD_ENOMEM; a
 * context that already has a queued or running request, with CSVD_ESTATE. */
int csvd_server_submit(csvd_server *srv, csvd_ctx *ctx, double a, double b,
                       const csvd_params *p, const double *V_in, int64_t *req);

/* Advances the loop by up to `steps` Lanczos steps of the running batch
 * (admitting and retiring requests at window boundaries).  *n_active
 * receives running + queued requests after the call. */
int csvd_server_step(csvd_server *srv, int32_t steps, int32_t *n_active);

/* *done = 1 when the request finished (its triplets are then in its
 * context, readable with csvd_get_triplets), 0 otherwise; *status is the
 * request's solve status once done. */
int csvd_server_poll(csvd_server *srv, int64_t req, int32_t *done, int32_t *status);

/* Removes a queued or running request; others are unaffected. */
int csvd_server_cancel(csvd_server *srv, int64_t req);

const char *csvd_server_last_error(const csvd_server *srv);
void csvd_server_destroy(csvd_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* CSVD_H */
