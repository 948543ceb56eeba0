// Continuous-batching request loop on one GPU.
//
// Requests of the same (mesh, tau, precision, solver tolerances) share a
// batch: one Solver whose columns are slots.  An admission thread places
// queued requests into free column ranges of a compatible batch, or opens a
// new batch when the HBM budget allows.  Each batch has a worker thread and a
// stream of its own; at every step boundary it takes in newly placed
// requests (upload + normalisation of their columns only), advances all
// resident requests one time step in the same launches, and retires requests
// that reached their step count (energies, labels and state copied out, their
// columns freed).  Batches of different meshes run concurrently on their own
// streams.
#pragma once

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "engine.h"

namespace sp {

// Host array of doubles left uninitialised on allocation: a request's input
// and output state (up to gigabytes) is first touched by the parallel copies
// of the server, not by a serial zero fill.
struct HostBuf {
  std::unique_ptr<double[]> p;
  size_t n = 0;
  void alloc(size_t k) {
    p.reset(new double[k]);
    n = k;
  }
  void clear() {
    p.reset();
    n = 0;
  }
  double* data() { return p.get(); }
};

class Server {
 public:
  Server(int64_t budget_bytes, int max_cols);
  ~Server();
  int64_t submit(Mesh* mesh, const sp_params& prm, const BatchSpec& spec, const double* u0);
  bool poll(int64_t ticket);
  bool wait(int64_t ticket, double timeout_s);
  int fetch(int64_t ticket, double* u_out, int32_t* labels, double* lambda, double* seps,
            double* energy, double* latency_s);
  void stats(double* p50, double* p99, double* cdof_per_s, int64_t* completed);
  // CG iterations summed over a finished request's columns, and its steps
  void request_stats(int64_t ticket, int64_t* col_iters, int64_t* steps);

 private:
  struct Batch;
  struct Request {
    int64_t id = 0;
    Mesh* mesh = nullptr;
    sp_params prm{};
    BatchSpec spec;
    HostBuf u0;
    int R = 0;
    double t_submit = 0, t_done = 0;
    bool placed = false, admitted = false, done = false;
    int error = SP_OK;
    std::string error_msg;
    Batch* batch = nullptr;
    int c_lo = 0, r_lo = 0;
    int64_t steps = 0;
    int64_t iters0 = 0, col_iters = 0;  // column CG iterations at admission / taken
    HostBuf u_out;
    std::vector<double> lam, seps, energy;
    std::vector<int32_t> labels;
  };
  struct Batch {
    Mesh* mesh = nullptr;
    sp_params prm{};
    int cap = 0, rcap = 0;
    int64_t bytes = 0;
    std::unique_ptr<Solver> solver;
    DevBuf<double> stage;             // [cap][n] request state in caller layout
    DevBuf<int32_t> lab;              // [rcap][n] labels of the restart slots
    std::vector<Request*> col_owner;  // per column slot
    std::vector<Request*> res_owner;  // per restart slot
    std::vector<Request*> pending;    // placed, waiting for the step boundary
    std::vector<Request*> resident;
    std::thread th;
    std::condition_variable cv;
    bool quit = false;
    bool exited = false;
  };
  struct Tables {
    std::vector<int> seg_lo, seg_len, live, res_lo, res_len;
    std::vector<double> coef, ieps2;
  };

  static bool compatible(const sp_params& a, const sp_params& b);
  static int64_t batch_bytes(const Mesh* m, const sp_params& p, int cap, int rcap);
  bool try_place(Request* q);           // under mu_
  bool find_slots(Batch* b, int R, int nres, int* c_lo, int* r_lo);
  void admission_loop();
  void batch_loop(Batch* b);
  void retire(Batch* b, Request* q);
  void admit(Batch* b, Request* q);
  Tables build_tables(Batch* b);        // under mu_
  void apply_tables(Batch* b, const Tables& t);  // batch thread, without mu_

  int64_t budget_, used_ = 0;
  int max_cols_;
  std::mutex mu_;
  std::condition_variable cv_;       // admission thread wake-up
  std::condition_variable done_cv_;  // request completion
  bool stop_ = false;
  int64_t next_id_ = 1;
  std::deque<Request*> queue_;
  std::map<int64_t, std::unique_ptr<Request>> reqs_;
  std::vector<std::unique_ptr<Batch>> batches_;
  std::vector<double> latencies_;
  double t_first_ = -1, t_last_ = 0, cdof_done_ = 0;
  int64_t completed_ = 0;
  std::thread adm_;
};

}  // namespace sp
