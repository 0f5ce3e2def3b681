// Host side of the batched Lanczos engine: device buffers of one job, the
// engine that advances a set of jobs with one launch per stage, and the
// context / server objects behind the C ABI.
#pragma once

#include <cstdlib>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "csvd_impl.h"

namespace csvd {

// Frees the idle chunks of stored bases kept for reuse (block.cpp).
void release_idle_chunks();

// Device allocation helper: frees on destruction.  When the device is out of
// memory, the idle stored-basis chunks are released and the allocation tried
// once more (reclaim = false for callers that hold the chunk pool's lock).  A
// failed hipMalloc's error is consumed here, so that a later launch check
// (hipGetLastError) does not report it.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  hipError_t alloc(size_t b, bool reclaim = true) {
    release();
    if (b == 0) b = 256;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipErrorOutOfMemory && reclaim) {
      (void)hipGetLastError();
      release_idle_chunks();
      e = hipMalloc(&p, b);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return e;
    }
    bytes = b;
    if (poison_allocs()) return hipMemset(p, 0xFF, b);  // all-ones bytes: NaN doubles
    return hipSuccess;
  }
  // CSVD_POISON_ALLOC=1 fills every new buffer with NaN bytes so that a read
  // of memory no kernel has written shows up in the results (debug aid)
  static bool poison_allocs() {
    static const bool on = [] {
      const char *v = std::getenv("CSVD_POISON_ALLOC");
      return v && v[0] == '1';
    }();
    return on;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

inline int ilog2i(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// Sparse-product tiling of one job side (rows of A or of A^T): G lane
// groups split each row's nonzeros (about 16 nonzeros per lane group), E
// thread slots per thread, rpt = 256 E / (Lp G) rows per tile; E shrinks
// until there are enough tiles to fill the chip.
struct Tiling {
  int G, lgG, E, rpt, tiles;
};

inline Tiling tiling_for(int64_t rows, int64_t nnz, int Lp) {
  Tiling t{};
  const double avg = rows > 0 ? (double)nnz / rows : 0.0;
  t.G = 1;
  while (t.G * Lp < kThreads && avg / t.G > 16.0) t.G *= 2;
  t.lgG = ilog2i(t.G);
  t.E = 8;
  while (t.E > 1 && rows * Lp * t.G / (kThreads * t.E) < 2048) t.E /= 2;
  t.rpt = kThreads * t.E / (Lp * t.G);
  t.tiles = (int)((rows + t.rpt - 1) / t.rpt);
  return t;
}



// Rows of one side of the block products (A or A^T) with more than
// kLongRow nonzeros, cut into segments of at most kLongRow nonzeros:
// segment s covers nonzeros [sgb_s, sge_s); long row r is row lrow_r with
// segments lseg_r .. lseg_{r+1} - 1.  Built once per matrix.
struct LongRows {
  DevBuf sgb, sge, lrow, lseg;
  int nseg = 0, nlong = 0;
  int64_t nnz_long = 0;
  hipError_t build(const std::vector<int> &rowptr, hipStream_t st);
};

struct SolveSpec {
  double a = 0, b = 0;
  csvd_params p{};
  int S = 0, Lp = 0, W = 0;
  std::vector<double> shift_re, shift_im;  // S
  std::vector<double> c_re, c_im;          // S x (M+1)
};

// One job: the Lanczos block of one (matrix, right-hand sides) pair.
struct Job {
  JobDesc h{};          // host copy of the descriptor
  DevBuf mem;           // all per-job device arrays in one allocation
  DevBuf d_shift;       // S shifts (double2)
  int64_t iters = 0;    // steps run so far
  int64_t max_iters = 0;
  bool finished = false;
  bool converged = false;
  double max_res = 0;   // largest residual estimate at exit
  std::vector<double> hist;  // (alpha, beta) of column 0, first kHist steps
  static size_t bytes_needed(int64_t m, int64_t n, int64_t nnz, int Lp, int S, int W, bool mixed);
  hipError_t create(const int *rp, const int *ci, const double *va, const int *rpT, const int *ciT,
                    const double *vaT, int64_t m, int64_t n, int64_t nnz, int L, int Lp, int S, int W, bool mixed,
                    double tol,
                    const std::vector<double> &sre, const std::vector<double> &sim, hipStream_t st);
};

// Sampled HIP-event timings of the hot kernels.
struct KernelTimer {
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<int> kind;       // 0 = A product, 1 = A^T product, 2 = window apply / rest of a
                               // block step, 3 = moment window (block solver)
  size_t used = 0;
  ~KernelTimer();
  void reset() { used = 0; kind.clear(); }
  hipError_t begin(int k, hipStream_t st);
  hipError_t end(hipStream_t st);
  static constexpr int kKinds = 4;
  // averages in ms per kind; count of samples
  void summarize(double out[kKinds], int64_t cnt[kKinds]);
};

class Engine {
 public:
  explicit Engine(hipStream_t st, int W, bool mixed) : st_(st), W_(W), mixed_(mixed) {}
  ~Engine();
  hipError_t init();
  // add a job; its step 0 runs at the current clock (a multiple of W)
  hipError_t add(Job *j);
  // drop a job (cancellation); the others keep running
  void remove(Job *j);
  // run one window (W Lanczos steps of every job) and apply the window
  hipError_t run_window(KernelTimer *timer, int sample_every);
  // read active counts after a window; fills finished flags of jobs
  hipError_t collect(std::vector<Job *> *finished_jobs);
  size_t active() const { return jobs_.size(); }
  int64_t clock() const { return clock_; }
  int W() const { return W_; }
  bool mixed() const { return mixed_; }

 private:
  hipError_t rebuild();
  hipStream_t st_;
  int W_;
  bool mixed_;
  int64_t clock_ = 0;
  int parity_ = 0;
  bool dirty_ = true;
  std::vector<Job *> jobs_;
  DevBuf d_clock_, d_ticket_, d_jobs_, d_toff_;
  BatchLaunch bl_{};
  int64_t step_count_ = 0;
};

}  // namespace csvd

// ABI objects
struct csvd_ctx {
  int64_t m = 0, n = 0, nnz = 0;
  hipStream_t st = nullptr;
  csvd::DevBuf rp, ci, va, rpT, ciT, vaT, work;
  std::string err;
  // last solve
  bool solved = false;
  int last_status = CSVD_OK;
  int L = 0, M = 0, N = 0, S = 0;
  int64_t npad = 0, mpad = 0;
  csvd::DevBuf d_S;                  // moments, npad x (M+1)L
  csvd::DevBuf d_U, d_V;             // triplet vectors, mpad x t / npad x t
  std::vector<double> sigma, resid;  // t_hat
  std::vector<double> resid_est;     // t_hat: residual estimates of Sec. 3.4.1
  double resid_all_max = 0.0;        // largest residual before resid_target drops
  csvd::DevBuf ws[32];               // epilogue workspace (steps 3-5), kept between solves
  csvd_info info{};
  std::unique_ptr<csvd::Job> job;    // last round's job (solutions), single-vector solver
  double norm_est = 0.0;             // cached ||A||_2 estimate
  csvd::SolveSpec spec;
  // a server request (queued or running) or a batch holds the context: its
  // moments, triplets and info belong to that solve until it is done
  bool busy = false;
  csvd::LongRows lr[2];              // long rows of A (0) and of A^T (1)
};

struct csvd_server;
