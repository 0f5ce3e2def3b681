// Host side of the block Lanczos engine (see k_block.hip for the method).
#pragma once

#include <memory>
#include <vector>

#include "engine.h"

namespace csvd {

// device memory left free when the stored basis grows (bytes)
constexpr size_t kStoreReserve = (size_t)8 << 30;

// Frees the idle stored-basis chunks of the current device.
void release_idle_chunks();

// One block Lanczos problem: device histories, work blocks and the pass
// state.  Pass 1 builds the block tridiagonal matrix and monitors every
// (shift, column) residual.  If the whole basis fits in device memory it is
// kept (store mode) and the moments are accumulated from it right after
// pass 1; otherwise pass 2 regenerates the basis in a ring of kMomWindow + 2
// blocks and accumulates the moments as it goes.
struct BlockJob {
  BJobDesc h{};
  DevBuf mem, d_shift, d_cmom, d_desc, d_toff, d_qtab, d_q32tab;
  DevBuf seg_part;  // partial rows of the long-row segments (both products)
  // work buffers of the Householder QR of one block (inside `mem`)
  double *orth_x = nullptr, *orth_z = nullptr, *orth_tau = nullptr, *orth_ws = nullptr, *orth_ws2 = nullptr;
  BBatch solo{};
  std::vector<double *> qtab;                  // host copy of the basis table
  std::vector<float *> q32tab;                 // host copy of the FP32 basis table (mixed precision)
  std::vector<std::unique_ptr<DevBuf>> chunks;  // stored basis, kStoreChunk blocks each
  bool mixed = false;      // CSVD_MIXED: the stored basis holds FP32 copies (h.store32) and the
                           // recurrence keeps its FP64 blocks in the ring
  bool want_store = true;  // try store mode (the server keeps the ring: its budget covers the job only)
  int store_cap = 0;       // most basis blocks to store (0: as device memory allows)
  bool store = false;      // store mode active for the current pass 1
  bool stored_last = false;  // the last round's moments came from a stored basis
  int pass = 0;            // 0 idle, 1 building the basis, 2 accumulating moments, 3 done
  int K = 0;               // block steps used by the solution
  int Kcap = 0;
  bool converged = false;
  int64_t steps_total = 0; // over all passes and rounds
  int64_t steps_last = 0;  // pass-1 steps of the last round
  int mflushed = 0;        // second-pass steps whose moments are already in Sout
  int deflated_last = 0;   // deflated columns and one-pass steps at step K - 1 of the last pass 1
  int one_pass_last = 0;
  int robust_steps = 0;    // steps 0 .. robust_steps - 1 of each pass orthonormalise the new block by
                           // Householder QR (a filtered or otherwise nearly invariant starting block
                           // makes the first Krylov blocks tiny and numerically rank deficient)
  double *block_ptr(int k) const {  // Q_k in the basis storage (host view of the basis table)
    return qtab[(k / h.qC) % h.qT] + (size_t)(k % h.qC) * h.n * h.Lp;
  }
  static size_t bytes_needed(int64_t m, int64_t n, int64_t nnz, int Lp, int S, int Kcap, int L, int Kmom);
  hipError_t create(const int *rp, const int *ci, const double *va, const int *rpT, const int *ciT,
                    const double *vaT, int64_t m, int64_t n, int64_t nnz, int L, int Lp, int S, int Kcap, int Kmom,
                    double tol, const std::vector<double> &sre, const std::vector<double> &sim,
                    const std::vector<double> &cre, const std::vector<double> &cim, int cstride, hipStream_t st,
                    const LongRows *lr = nullptr);
  // copies the host descriptor to the device copy used by solo launches
  hipError_t sync_desc(hipStream_t st);
  // basis table: ring mode (no stored basis, FP64 or FP32), or store mode
  // with chunks covering blocks 0 .. kneed (false: memory did not allow it);
  // chunks hold FP64 blocks (qtab) or, for a mixed-precision job, FP32 ones
  // (q32tab)
  hipError_t set_ring(hipStream_t st);
  bool grow_store(int kneed, hipStream_t st);
  // keep: the chunks go to the device's pool of idle chunks; else they are freed
  void free_store(bool keep);
};

// The per-shift recurrences (b_shift) of step k depend only on A_k, B_k and
// B_{k+1}, so they run on a second stream and overlap the next steps.  The
// step clock is the host's: every launch of a step takes it by value.
class BEngine {
 public:
  explicit BEngine(hipStream_t st) : st_(st) {}
  ~BEngine();
  BEngine(const BEngine &) = delete;
  BEngine &operator=(const BEngine &) = delete;
  hipError_t init();
  // starts pass 1 of a job whose Vpad and Sout are ready (runs its set-up)
  hipError_t start(BlockJob *j);
  // one block step of every running job
  hipError_t step(KernelTimer *timer, bool sample);
  // after a few steps: moves converged pass-1 jobs to pass 2 and reports
  // jobs whose pass 2 is complete
  hipError_t poll(std::vector<BlockJob *> *finished);
  void remove(BlockJob *j);
  // a finished job whose moments came from a stored basis runs the second
  // pass (regenerating its basis in FP64) and accumulates its moments again
  // from the coefficients it already has (the backward solution works in
  // place on the histories and runs once)
  hipError_t regenerate(BlockJob *j) { return enter_pass2(j, false); }
  size_t active() const { return p1_.size() + p2_.size(); }
  int64_t clock() const { return clock_; }

 private:
  hipError_t rebuild(std::vector<BlockJob *> &jobs, DevBuf &dj, DevBuf &dt, BBatch &b);
  hipError_t enter_pass2(BlockJob *j, bool coefficients = true);
  hipError_t finish_stored(BlockJob *j);
  hipError_t clear_moments(const BJobDesc &J);
  hipError_t start_block(BlockJob *j, bool first);
  // Householder QR of the row-major n x Lp block src: Q into dst (may be src),
  // optionally R (row-major Lp x Lp, zero below) and the column norms of src
  hipError_t orth_block(BlockJob *j, const double *src, double *dst, double *R, double *norms);
  // robust steps of the jobs in v after their gamma (Q_{k+1} from W3)
  hipError_t robust_finish(std::vector<BlockJob *> &v, bool first_pass);
  hipError_t launch_shift(const BBatch &b, int init);
  // step 0 of a round without Householder steps: takes them when the
  // starting block is close to an invariant subspace
  hipError_t check_first_block(BlockJob *j);
  // long rows of the jobs in v for one product (side 1: A, side 2: A^T)
  hipError_t long_rows(const std::vector<BlockJob *> &v, int side);
  // The shift recurrences of the steps since the last poll, launched together
  // behind one event (they read only history entries of their own steps).
  hipError_t flush_shifts();
  int npend_ = 0;
  // Convergence snapshot: each poll writes the counters of every pass-1 job
  // (after its last enqueued step) into pinned host memory without waiting,
  // and decides from the snapshot of the poll before, so the device always
  // has the steps of one poll interval queued.  A job whose snapshot shows
  // convergence after `steps` steps ends with K = steps, as if it had been
  // polled at once; the steps it ran meanwhile only wrote history entries
  // and basis blocks past K.
  struct Snap {
    BlockJob *j;
    int steps;
  };
  hipError_t take_snapshot();
  std::vector<Snap> snap_;
  int *snap_host_ = nullptr;  // pinned, 4 ints per entry: active count, flags[0..2]
  size_t snap_cap_ = 0;
  hipEvent_t snap_main_ = nullptr, snap_side_ = nullptr;
  KernelTimer *timer_ = nullptr;  // the timer of the last step() call (moment launches are sampled)
  hipStream_t st_;
  hipStream_t side_ = nullptr;
  hipEvent_t ev_ = nullptr;
  // Step graph: the kernels of one pass-1 step of the current batch tables,
  // captured once (on a private stream) and replayed at successive clocks;
  // the kernels read the clock from clk_ and a tick kernel at the end of the
  // graph advances it.  Steps with host-side work (robust steps, long-row
  // segments, sampled timings) or second-pass jobs run as eager launches.
  // Opt-in: CSVD_STEP_GRAPH=1 in the environment (eager launches otherwise).
  hipError_t step_kernels(const BBatch &b, hipStream_t st);
  hipError_t capture_step();
  bool graph_step_ok() const;
  bool graphs_ = true;
  hipStream_t cap_ = nullptr;
  DevBuf clk_;
  hipGraphExec_t gexec_ = nullptr;
  bool clk_synced_ = false;
  int64_t graph_steps_ = 0, eager_steps_ = 0;

 public:
  int64_t graph_steps() const { return graph_steps_; }
  int64_t eager_steps() const { return eager_steps_; }

 private:
  int64_t clock_ = 0;
  std::vector<BlockJob *> p1_, p2_;
  DevBuf dj1_, dt1_, dj2_, dt2_;
  BBatch b1_{}, b2_{};
  bool dirty1_ = true, dirty2_ = true;
};

}  // namespace csvd
