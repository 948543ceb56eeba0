// Batch solver: device state of a batch of restarts and the orchestration of
// one time step of Algorithm 2.2 (heat solve, node step, normalisation),
// energies and labels.
#pragma once

#include <array>
#include <utility>
#include <functional>
#include <string>
#include <vector>

#include "autotune.h"
#include "kernels.h"

namespace sp {

struct BatchSpec {
  std::vector<int> m;       // components per restart
  std::vector<double> eps;  // eps per restart
};

void validate_params(const sp_params& p);
void validate_batch(int32_t nres, const int32_t* m, const double* eps);

// Kernel classes of the CG profile (sp_state_kernel_time): matrix product,
// x/r update, p update, polynomial preconditioner pass.
constexpr int kKernelClasses = 4;
// Device counters of a batch (StepArgs::stat).
constexpr int kStats = 4;

class Solver {
 public:
  // stream == nullptr: the solver creates and owns a stream; otherwise it
  // uses *stream (which may be the legacy default stream 0).  min_columns /
  // min_restarts reserve extra column and restart slots (server batches
  // start with an empty spec and fill slots later).  arena (nullable): every
  // device buffer, K = M + tau A of this tau included, is taken from it
  // instead of allocated, and nothing else allocates device or pinned host
  // memory (no tiling search, no graph replays, pageable host polls); the
  // host-pointer upload/download helpers are not available then.
  Solver(Mesh* mesh, const sp_params& prm, const BatchSpec& spec, const hipStream_t* stream,
         int min_columns = 0, int min_restarts = 0, Arena* arena = nullptr);
  ~Solver();
  Solver(const Solver&) = delete;
  Solver& operator=(const Solver&) = delete;

  // Initial state [R][n] (caller numbering) from host or device memory;
  // normalise = scale every live component to unit L2 norm.
  void upload_host(const double* u0, bool normalise);
  void upload_device(const double* d_u0, bool normalise, bool check_norms);
  void download_host(double* u);      // [R][n] host
  void download_device(double* d_u);  // [R][n] device

  // Algorithm 2.2: k full steps (energies at the prm.energy_every cadence,
  // recorded in the history).
  void step(int64_t k);
  // Run until every restart met the stop rule (n_steps == 0) or max_steps.
  void run_to_stop();
  void stage_heat();
  void stage_node();
  void stage_norm();
  // Energies of the current state into device arrays (lam [rp], seps/E [nres]).
  void energy();
  void energy_to_host(double* lam, double* seps, double* E);
  // Lagrange multipliers lambda^eps [R] of the current state (host)
  void multipliers_to_host(double* lam_eps);
  void labels_device(int32_t* d_lab, int32_t* d_lab_am);
  void labels_host(int32_t* lab, int32_t* lab_am);
  // Partition post-processing (partition.cpp).  Restrict every column to its
  // region: labels [nres][n] (caller order), column lo_r + i of restart r
  // keeps the vertices labelled i (interior: and not on the region's
  // boundary, i.e. without a mesh neighbour labelled otherwise); the state
  // is masked, columns with an empty region stop being live.  Float64 only.
  void set_region_mask(const int32_t* labels, bool interior);
  // Inverse iteration u <- (M + tau A)^{-1} M u on the regions, normalised,
  // until every live column's Rayleigh quotient changes by <= tol relative;
  // lam [R] host (NaN where not live).  Returns the iterations taken.
  int region_eigen(double tol, int max_iter, double* lam);

  // column/restart activity (continuous batching, stop rule)
  void set_restart_live(int r, bool live);
  void sync();
  hipStream_t stream() const { return s_; }

  int R() const { return R_; }
  int rp() const { return rp_; }
  int nres() const { return int(spec_.m.size()); }
  int64_t n() const { return mesh_->n; }
  int64_t steps_done() const { return steps_done_; }
  void set_steps_done(int64_t k) { steps_done_ = k; }
  const std::vector<std::vector<std::pair<int64_t, double>>>& history() const { return hist_; }
  sp_stats stats();
  bool converged();
  // sum over columns [c_lo, c_lo + cnt) of the CG iterations each has taken
  // (cumulative since the solver was made; synchronous)
  int64_t column_iters(int c_lo, int cnt);

  // event timing of the three large CG kernels (0 matrix product, 1 x/r
  // update, 2 p update) on the solver's stream
  void profile(bool on);
  void kernel_time(int which, int64_t* launches, double* ms, double* bytes_per_launch);

  const double* d_lam() const { return lam_.p; }
  const double* d_seps() const { return seps_.p; }
  const double* d_energy() const { return energy_.p; }
  double* d_u() {
    flush_scale();
    return u_.p;
  }
  const Tile& tile() const { return args_.t; }
  const Tile& gather_tile() const { return args_.tm; }
  double tuned_us() const { return tuned_.us; }
  const sp_params& params() const { return prm_; }
  Mesh* mesh() const { return mesh_; }

  // Re-seat a restart's columns (server slots): new m/eps tables must keep
  // the column layout; used by the server which owns one solver per batch.
  void set_columns(const std::vector<int>& seg_lo, const std::vector<int>& seg_len,
                   const std::vector<double>& coef, const std::vector<int>& live,
                   const std::vector<int>& res_lo, const std::vector<int>& res_len,
                   const std::vector<double>& res_ieps2);
  void normalise_columns();  // normalise live columns of the current state in place

  // Column range [c_lo, c_lo + Rq) of the state from/to caller layout [Rq][n]
  // on the device (server slots).
  void pack_range(int c_lo, int Rq, const double* d_src);
  void unpack_range(int c_lo, int Rq, double* d_dst);
  // Normalise only columns [c_lo, c_lo + Rq); throws SP_EINVAL on a zero norm.
  void normalise_range(int c_lo, int Rq);
  // Skip the stream synchronisation in the destructor (work already done).
  void detach() { detached_ = true; }
  // Forget the previous heat increments of every column (the next step
  // starts from x0 = u).
  void reset_guess() {
    forget_history(0, rp_);
    aw_fresh_ = false;
  }
  // Graph replay of the inner CG blocks (on by default; off for batches whose
  // stream shares the device with other threads' launches, e.g. the server's).
  void set_graphs(bool on) { graph_on_ = on && graph_on_; }

  // Checkpoint of the whole device state (checkpoint.cpp): its size in bytes,
  // the image written to a host buffer, and its restore into a solver of the
  // same batch (mesh size, columns, precision, extrapolation depth, tau, m,
  // eps), after which the run continues exactly as the one that wrote it.
  int64_t checkpoint_size();
  void checkpoint(void* buf, int64_t bytes);
  void restore(const void* buf, int64_t bytes);

  bool record_history = true;          // copy energies to the host at the cadence
  std::vector<int64_t> restart_steps;  // per restart: steps taken (stop mode)

 private:
  void heat();  // heat solve; its result is left in heat_x_
  void step_small(int64_t k);
  void heat_fp64();
  void heat_mixed();
  void node_to_r();
  void norm_dot_scale(const double* v, bool defer);
  void flush_scale();
  int poll(const int* dev_counter);
  void push_tables();
  // algorithmic HBM bytes (sp_stats.hbm_bytes): per_elem x n x live columns
  // + extra, for a pass over the live columns (kernels that skip converged
  // columns are counted in full: an upper bound); the CG iterations are
  // counted exactly in stats() from the device's active-column counter
  void acct(double per_elem, double extra = 0.0);
  double mat_bytes(double value_bytes, int n_mats) const;  // ELL pattern + n_mats value arrays
  double fixed_bytes_ = 0.0;
  int live_cols_ = 0;
  std::vector<Tile> tile_candidates() const;
  TuneChoice tune_tiling(const std::string& key, Tile StepArgs::*field,
                         const std::function<void()>& launch);
  void autotune();
  TuneChoice tuned_{};

  Mesh* mesh_;
  TauMats* km_;
  Arena* arena_ = nullptr;
  TauMats own_km_;      // this tau's matrices taken from the arena
  int poll_host_[16] = {};  // poll target without pinned memory (arena mode)
  template <class T>
  void get(DevBuf<T>& b, size_t count) {
    if (arena_)
      b.adopt(arena_->take<T>(count), count);
    else
      b.alloc(count);
  }
  sp_params prm_;
  BatchSpec spec_;
  int R_ = 0, rp_ = 0, nres_p_ = 0;
  hipStream_t s_ = nullptr;
  bool own_stream_ = false;
  bool detached_ = false;

  DevBuf<double> u_, r64_, p64_, q64_;
  DevBuf<float> d32_, r32_, q32_;
  DevBuf<bf16_t> p16_;  // direction ring slot 0 (bf16, like the whole ring)
  DevBuf<double> z64_;  // polynomial preconditioner's output (float64 CG)
  DevBuf<bf16_t> z16_;  // (float32 inner CG: bf16)
  DevBuf<bf16_t> pbuf_[kPRing];       // direction ring slots 1.. (slot 0 is p16_)
  bf16_t* pring_[kPRing] = {};
  DevBuf<double> ah_;                 // [kPRing][rp] alpha of each ring slot
  // heat increments of the last prm_.extrapolate steps (extrapolated start):
  // dh_[0] the latest, dh_[q-1] the oldest; a solve overwrites the oldest
  // with its start guess g and accumulates its own increment on top of it,
  // then the ring rotates so that buffer becomes dh_[0]
  DevBuf<float> dbuf_[kMaxExtrap];
  float* dh_[kMaxExtrap] = {};
  int n_prev_ = 0;  // increments available to some column (0 .. prm_.extrapolate)
  std::vector<int> h_hlen_;  // host copy of the per-column history lengths (args_.hlen)
  // columns [c_lo, c_lo + cnt) have no previous increment (all columns: n_prev_ = 0)
  void forget_history(int c_lo, int cnt);
  DevBuf<double> xg_;          // iterate of a solve started from u + g (u stays b's source)
  DevBuf<float> d0buf_;        // sweep 0's correction while the iterate is deferred
  double* heat_x_ = nullptr;   // where the last heat solve left its result (u_ or xg_)
  bool small_ = false;         // whole steps in one workgroup (small batches)
  // refinement sweeps the last mixed heat solve took: sweep o's update also
  // writes sweep o + 1's inner start when o + 1 < last_sweeps_
  int last_sweeps_ = 0;
  static constexpr int kSmallChunk = 128;  // steps per launch of the small path
  DevBuf<double> small_hist_;  // [kSmallChunk][nres_p] energies at the cadence
  bool aw_fresh_ = false;      // xg_ holds A v of the norm pass that produced u (and
                               // cg.bb_next its ||M u||^2): the next solve can start
                               // without gathering u
  // Deferred normalisation: in a mixed-precision step the node step writes
  // v straight into u_ and the norm pass leaves 1/||v||_M in cg.isc instead
  // of scaling; the next solve's first update and the S_eps kernels apply the
  // factor as they read u_.  Anything else that reads u_ or changes the live
  // masks calls flush_scale() first.
  // The float32 inner CG in blocks of kPRing iterations (the polling period)
  // replayed from a captured HIP graph: one launch instead of 5 kPRing.
  // Variant [f]: f = 1 once the direction ring has been folded before (the
  // block's last iteration folds it again, accumulating).  Re-captured when
  // args_ has changed since the capture (the kernels take it by value).
  // SEGPART_GRAPH=0 turns this off; never used while profiling, on the
  // legacy default stream, or with another polling period.
  void cg_block(int flushed);
  void precond_start();
  double class_bytes(int which, bool f64) const;
  bool graph_on_ = true;
  hipGraphExec_t cg_graph_[2] = {nullptr, nullptr};
  StepArgs cg_graph_args_[2];
  bool u_pending_ = false;
  DevBuf<uint8_t> mask_;  // [n][rp] region mask (set_region_mask)
  double* node_out_ = nullptr;  // where the last node step wrote (u_ or r64_)
  bool lam_fresh_ = false;  // lam holds the Rayleigh quotients of the current state
  bool all_live_ = true;    // every real column is live
  DevBuf<double> part_, part_s_;
  DevBuf<double> part2_;  // preconditioner pass partials [nblk][rp]
  DevBuf<double> colf_;  // 8 x rp column doubles + nres_p restart doubles
  DevBuf<int> coli_;     // 7 x rp column ints + 3 x nres_p restart ints
  DevBuf<int> ring_;     // 2 x kRing
  DevBuf<long long> stat_;
  DevBuf<double> lam_, seps_, energy_;
  int* h_poll_ = nullptr;

  std::vector<int> h_seg_lo_, h_seg_len_, h_live_, h_res_lo_, h_res_len_, h_res_live_;
  std::vector<double> h_coef_, h_res_ieps2_;

  StepArgs args_{};
  SepsPlan sp_{};
  DevBuf<int4> seps_tiles_;
  int64_t steps_done_ = 0;
  std::vector<std::vector<std::pair<int64_t, double>>> hist_;

  bool prof_ = false;
  std::vector<std::array<hipEvent_t, 8>> ev_;
  size_t ev_used_ = 0;
  int64_t prof_launches_[kKernelClasses] = {};
  double prof_ms_[kKernelClasses] = {};
  long long prof_stat0_[kStats] = {};
  void prof_flush();
  const hipEvent_t* prof_events();
  void read_stat(long long* st);
};

// Solvers whose work was enqueued asynchronously are freed later, from an
// ordinary API call (never from inside a stream callback).
void defer_delete(Solver* s);
void reap_deferred();

}  // namespace sp
