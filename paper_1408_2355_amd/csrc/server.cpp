// Continuous-batching request loop (see server.h).
#include "server.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

namespace sp {

namespace {
// f(lo, hi) over [0, n) in contiguous slices on up to 16 threads (the
// calling thread takes the first), one slice per 64 MB of doubles at least;
// for the request-sized host copies, whose cost is mostly first-touch page
// faults that a single thread takes one by one.
template <class F>
void par_for(size_t n, F&& f) {
  constexpr size_t kMin = size_t(1) << 23;
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t T = std::max<size_t>(1, std::min<size_t>(std::min<size_t>(hw, 16), n / kMin));
  if (T <= 1) {
    f(size_t(0), n);
    return;
  }
  const size_t step = (n + T - 1) / T;
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (size_t t = 1; t < T; ++t) {
    const size_t lo = t * step, hi = std::min(n, lo + step);
    if (lo < hi) th.emplace_back([&f, lo, hi] { f(lo, hi); });
  }
  f(size_t(0), std::min(n, step));
  for (auto& x : th) x.join();
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

Server::Server(int64_t budget_bytes, int max_cols) : budget_(budget_bytes), max_cols_(max_cols) {
  SP_REQUIRE(max_cols_ >= 4, SP_EINVAL, "server: max_batch_columns must be >= 4");
  adm_ = std::thread([this] { admission_loop(); });
}

Server::~Server() {
  // Stop the admission thread first: after it has exited no batch is opened
  // or reaped any more, so batches_ is this thread's alone.
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (adm_.joinable()) adm_.join();
  {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& b : batches_) b->quit = true;
  }
  for (auto& b : batches_) b->cv.notify_all();
  for (auto& b : batches_)
    if (b->th.joinable()) b->th.join();
  batches_.clear();
}

bool Server::compatible(const sp_params& a, const sp_params& b) {
  return a.tau == b.tau && a.precision == b.precision && a.cg_rtol == b.cg_rtol &&
         a.cg_max_iter == b.cg_max_iter && a.check_every == b.check_every &&
         a.extrapolate == b.extrapolate && a.precond == b.precond &&
         (a.precision == SP_FP64 || (a.inner_rtol == b.inner_rtol && a.max_outer == b.max_outer));
}

int64_t Server::batch_bytes(const Mesh* m, const sp_params& p, int cap, int rcap) {
  // state u and outer residual (float64) + CG vectors (float64 pair or
  // float32 quad, plus the rest of the float32 direction ring) and, for the
  // extrapolated start, the float32 increments, a float64 iterate and a
  // float32 deferred correction per element, the polynomial preconditioner's
  // output, the float64/float32 K copies of this tau, the mesh matrices,
  // partial sums and tables
  const double n = double(m->n);
  const bool poly = p.precond == SP_PRECOND_CHEB1;
  // (float32 CG: d, r, q float32, the kPRing ring directions and z bf16)
  const bool mixed = p.precision != SP_FP64;
  const double per_col =
      16.0 + (mixed ? 12.0 + 2.0 * kPRing : 16.0) +
      (mixed && p.extrapolate ? 12.0 + 4.0 * p.extrapolate : 0.0) +
      (poly ? (mixed ? 2.0 : 8.0) : 0.0);
  const double mats = double(m->W) * n * (4 + 8 + 8 + 8 + 4 + (poly ? 12 : 0)) + n * 28.0 +
                      double(m->nt) * 20.0;
  // partial sums: 3 slots (5 with the extrapolation's order control), +1 for
  // the polynomial preconditioner's pass
  const double part = ((mixed && p.extrapolate >= 2 ? 5.0 : 3.0) + (poly ? 1.0 : 0.0)) * 8.0 * cap *
                      (n / 64.0 + 1.0);
  // staging of request state (admission and retirement) and of labels
  const double stage = 8.0 * n * cap + 4.0 * n * rcap;
  return int64_t(n * cap * per_col + mats + part + stage + 64.0 * (cap + rcap) + (1 << 20));
}

int64_t Server::submit(Mesh* mesh, const sp_params& prm, const BatchSpec& spec, const double* u0) {
  SP_REQUIRE(u0 != nullptr, SP_EINVAL, "NULL u0");
  std::unique_ptr<Request> q(new Request());
  q->mesh = mesh;
  q->prm = prm;
  q->spec = spec;
  for (int x : spec.m) q->R += x;
  SP_REQUIRE(q->R <= max_cols_, SP_EINVAL, "server: request has more components than a batch holds");
  const size_t cnt = size_t(q->R) * mesh->n;
  q->u0.alloc(cnt);
  std::atomic<bool> finite{true};
  par_for(cnt, [&](size_t lo, size_t hi) {
    double* dst = q->u0.data();
    bool ok = true;
    for (size_t i = lo; i < hi; ++i) {
      dst[i] = u0[i];
      ok = ok && std::isfinite(u0[i]);
    }
    if (!ok) finite = false;
  });
  SP_REQUIRE(finite.load(), SP_EINVAL, "u0 holds a non-finite value");
  const int cap = (q->R + 3) / 4 * 4;
  SP_REQUIRE(batch_bytes(mesh, prm, cap, int(spec.m.size())) <= budget_, SP_ENOMEM,
             "server: request does not fit in the HBM budget");
  std::lock_guard<std::mutex> g(mu_);
  SP_REQUIRE(!stop_, SP_EINVAL, "server stopped");
  q->id = next_id_++;
  q->t_submit = now_s();
  if (t_first_ < 0) t_first_ = q->t_submit;
  const int64_t id = q->id;
  queue_.push_back(q.get());
  reqs_[id] = std::move(q);
  cv_.notify_one();
  return id;
}

bool Server::find_slots(Batch* b, int R, int nres, int* c_lo, int* r_lo) {
  auto first_fit = [](const std::vector<Request*>& own, int need, int* lo) {
    int run = 0;
    for (int i = 0; i < int(own.size()); ++i) {
      run = own[i] ? 0 : run + 1;
      if (run == need) {
        *lo = i - need + 1;
        return true;
      }
    }
    return false;
  };
  return first_fit(b->col_owner, R, c_lo) && first_fit(b->res_owner, nres, r_lo);
}

bool Server::try_place(Request* q) {
  const int nres = int(q->spec.m.size());
  for (auto& bp : batches_) {
    Batch* b = bp.get();
    if (b->quit || b->mesh != q->mesh || !compatible(b->prm, q->prm)) continue;
    int c_lo, r_lo;
    if (!find_slots(b, q->R, nres, &c_lo, &r_lo)) continue;
    for (int c = 0; c < q->R; ++c) b->col_owner[c_lo + c] = q;
    for (int r = 0; r < nres; ++r) b->res_owner[r_lo + r] = q;
    q->batch = b;
    q->c_lo = c_lo;
    q->r_lo = r_lo;
    q->placed = true;
    b->pending.push_back(q);
    b->cv.notify_one();
    return true;
  }
  // open a new batch sized for a few requests like this one
  int cap = std::min(max_cols_, std::max(4 * ((q->R + 3) / 4 * 4), 64));
  cap = std::max(cap, (q->R + 3) / 4 * 4);
  int64_t bytes = batch_bytes(q->mesh, q->prm, cap, cap);
  while (used_ + bytes > budget_ && cap > (q->R + 3) / 4 * 4) {
    cap = std::max((q->R + 3) / 4 * 4, cap / 2 / 4 * 4);
    bytes = batch_bytes(q->mesh, q->prm, cap, cap);
  }
  if (used_ + bytes > budget_) return false;
  std::unique_ptr<Batch> b(new Batch());
  b->mesh = q->mesh;
  b->prm = q->prm;
  b->prm.n_steps = 1;
  b->prm.energy_every = 0;
  b->cap = cap;
  b->rcap = cap;
  b->bytes = bytes;
  b->col_owner.assign(cap, nullptr);
  b->res_owner.assign(cap, nullptr);
  used_ += bytes;
  for (int c = 0; c < q->R; ++c) b->col_owner[c] = q;
  for (int r = 0; r < nres; ++r) b->res_owner[r] = q;
  q->batch = b.get();
  q->c_lo = 0;
  q->r_lo = 0;
  q->placed = true;
  b->pending.push_back(q);
  Batch* raw = b.get();
  batches_.push_back(std::move(b));
  raw->th = std::thread([this, raw] { batch_loop(raw); });
  return true;
}

void Server::admission_loop() {
  std::unique_lock<std::mutex> lk(mu_);
  while (!stop_) {
    // reap batches whose worker exited
    for (auto it = batches_.begin(); it != batches_.end();) {
      Batch* b = it->get();
      if (b->exited && b->th.joinable()) {
        std::thread th = std::move(b->th);
        lk.unlock();
        th.join();
        lk.lock();
        it = batches_.erase(it);
      } else {
        ++it;
      }
    }
    if (stop_) break;  // set while a batch was being reaped
    for (auto it = queue_.begin(); it != queue_.end();) {
      if (try_place(*it))
        it = queue_.erase(it);
      else
        ++it;
    }
    cv_.wait_for(lk, std::chrono::milliseconds(20));
  }
}

Server::Tables Server::build_tables(Batch* b) {
  Tables t;
  const int rp = (b->cap + 3) / 4 * 4;
  t.seg_lo.assign(rp, 0);
  t.seg_len.assign(rp, 0);
  t.live.assign(rp, 0);
  t.coef.assign(rp, 0.0);
  int nres_used = 0;
  for (Request* q : b->resident)
    nres_used = std::max(nres_used, q->r_lo + int(q->spec.m.size()));
  t.res_lo.assign(nres_used, 0);
  t.res_len.assign(nres_used, 0);
  t.ieps2.assign(nres_used, 0.0);
  for (Request* q : b->resident) {
    int lo = q->c_lo;
    for (size_t j = 0; j < q->spec.m.size(); ++j) {
      const int m = q->spec.m[j];
      const double e = q->spec.eps[j];
      for (int i = 0; i < m; ++i) {
        t.seg_lo[lo + i] = lo;
        t.seg_len[lo + i] = m;
        t.live[lo + i] = 1;
        t.coef[lo + i] = 2.0 * b->prm.tau / (e * e);
      }
      const int rs = q->r_lo + int(j);
      t.res_lo[rs] = lo;
      t.res_len[rs] = m;
      t.ieps2[rs] = 1.0 / (e * e);
      lo += m;
    }
  }
  return t;
}

void Server::apply_tables(Batch* b, const Tables& t) {
  b->solver->set_columns(t.seg_lo, t.seg_len, t.coef, t.live, t.res_lo, t.res_len, t.ieps2);
}

void Server::admit(Batch* b, Request* q) {
  const size_t cnt = size_t(q->R) * b->mesh->n;
  SP_REQUIRE(cnt <= b->stage.n, SP_EINVAL, "server: request larger than its batch");
  SP_HIP(hipMemcpyAsync(b->stage.p, q->u0.data(), cnt * sizeof(double), hipMemcpyHostToDevice,
                        b->solver->stream()));
  b->solver->pack_range(q->c_lo, q->R, b->stage.p);
  b->solver->normalise_range(q->c_lo, q->R);
  b->solver->sync();
  q->iters0 = b->solver->column_iters(q->c_lo, q->R);
  q->u0.clear();
}

void Server::retire(Batch* b, Request* q) {
  Solver& S = *b->solver;
  const int nres = int(q->spec.m.size());
  const int64_t n = b->mesh->n;
  q->lam.resize(q->R);
  q->seps.resize(nres);
  q->energy.resize(nres);
  SP_HIP(hipMemcpyAsync(q->lam.data(), S.d_lam() + q->c_lo, q->R * sizeof(double),
                        hipMemcpyDeviceToHost, S.stream()));
  SP_HIP(hipMemcpyAsync(q->seps.data(), S.d_seps() + q->r_lo, nres * sizeof(double),
                        hipMemcpyDeviceToHost, S.stream()));
  SP_HIP(hipMemcpyAsync(q->energy.data(), S.d_energy() + q->r_lo, nres * sizeof(double),
                        hipMemcpyDeviceToHost, S.stream()));
  const size_t cnt = size_t(q->R) * n;
  q->col_iters = S.column_iters(q->c_lo, q->R) - q->iters0;
  S.unpack_range(q->c_lo, q->R, b->stage.p);
  // first touch of the output pages on many threads, then the copy
  q->u_out.alloc(cnt);
  par_for(q->u_out.n, [&](size_t lo, size_t hi) {
    std::memset(q->u_out.data() + lo, 0, (hi - lo) * sizeof(double));
  });
  SP_HIP(hipMemcpyAsync(q->u_out.data(), b->stage.p, cnt * sizeof(double), hipMemcpyDeviceToHost,
                        S.stream()));
  S.sync();
}

void Server::batch_loop(Batch* b) {
  auto fail_all = [&](const std::vector<Request*>& v, int code, const std::string& msg) {
    std::lock_guard<std::mutex> g(mu_);
    for (Request* q : v) {
      q->error = code;
      q->error_msg = msg;
      q->done = true;
      q->t_done = now_s();
      for (auto& o : b->col_owner)
        if (o == q) o = nullptr;
      for (auto& o : b->res_owner)
        if (o == q) o = nullptr;
    }
    done_cv_.notify_all();
    cv_.notify_all();
  };
  try {
    b->solver.reset(new Solver(b->mesh, b->prm, BatchSpec{}, nullptr, b->cap, b->rcap));
    b->solver->record_history = false;
    // Batch threads share the device: no graph capture on them (a capture
    // on one thread would run beside other threads' launches and device
    // allocations), and no device allocation after set-up: request state and
    // labels go through staging buffers sized for the batch.
    b->solver->set_graphs(false);
    b->stage.alloc(size_t(b->cap) * size_t(b->mesh->n));
    b->lab.alloc(size_t(b->rcap) * size_t(b->mesh->n));
  } catch (const Error& e) {
    std::vector<Request*> v;
    {
      std::lock_guard<std::mutex> g(mu_);
      v.swap(b->pending);
      b->quit = true;
    }
    fail_all(v, e.code, e.what());
    std::lock_guard<std::mutex> g(mu_);
    used_ -= b->bytes;
    b->exited = true;
    return;
  }
  std::vector<int32_t> lab_dev_host;
  for (;;) {
    std::vector<Request*> newly;
    {
      std::unique_lock<std::mutex> lk(mu_);
      while (!b->quit && b->pending.empty() && b->resident.empty()) {
        if (b->cv.wait_for(lk, std::chrono::milliseconds(300)) == std::cv_status::timeout &&
            b->pending.empty() && b->resident.empty())
          b->quit = true;
      }
      if (b->quit) break;
      newly.swap(b->pending);
      for (Request* q : newly) {
        q->admitted = true;
        b->resident.push_back(q);
      }
    }
    try {
      if (!newly.empty()) {
        Tables tb;
        {
          std::lock_guard<std::mutex> g(mu_);
          tb = build_tables(b);
        }
        apply_tables(b, tb);
        for (Request* q : newly) {
          try {
            admit(b, q);
          } catch (const Error& e) {
            {
              std::lock_guard<std::mutex> g(mu_);
              b->resident.erase(std::find(b->resident.begin(), b->resident.end(), q));
              q->admitted = false;
            }
            fail_all({q}, e.code, e.what());
            {
              std::lock_guard<std::mutex> g(mu_);
              tb = build_tables(b);
            }
            apply_tables(b, tb);
          }
        }
      }
      std::vector<Request*> res;
      {
        std::lock_guard<std::mutex> g(mu_);
        res = b->resident;
      }
      if (res.empty()) continue;
      b->solver->step(1);
      std::vector<Request*> fin;
      for (Request* q : res)
        if (++q->steps >= q->prm.n_steps) fin.push_back(q);
      if (!fin.empty()) {
        b->solver->energy();
        // labels of every restart slot in use, then each request takes its rows
        int nres_used = 0;
        {
          std::lock_guard<std::mutex> g(mu_);
          for (Request* q : b->resident)
            nres_used = std::max(nres_used, q->r_lo + int(q->spec.m.size()));
        }
        const int64_t n = b->mesh->n;
        const size_t nlab = size_t(std::max(nres_used, 1)) * n;
        SP_REQUIRE(nlab <= b->lab.n, SP_EINVAL, "server: restart slots beyond the batch");
        b->solver->labels_device(b->lab.p, nullptr);
        lab_dev_host.resize(nlab);
        SP_HIP(hipMemcpyAsync(lab_dev_host.data(), b->lab.p, nlab * sizeof(int32_t),
                              hipMemcpyDeviceToHost, b->solver->stream()));
        for (Request* q : fin) {
          retire(b, q);  // synchronises the stream
          const int nres = int(q->spec.m.size());
          q->labels.assign(lab_dev_host.begin() + size_t(q->r_lo) * n,
                           lab_dev_host.begin() + size_t(q->r_lo + nres) * n);
        }
        Tables tb;
        {
        std::lock_guard<std::mutex> g(mu_);
        const double t = now_s();
        for (Request* q : fin) {
          q->done = true;
          q->t_done = t;
          latencies_.push_back(t - q->t_submit);
          cdof_done_ += double(q->R) * double(n) * double(q->prm.n_steps);
          t_last_ = t;
          ++completed_;
          for (auto& o : b->col_owner)
            if (o == q) o = nullptr;
          for (auto& o : b->res_owner)
            if (o == q) o = nullptr;
          b->resident.erase(std::find(b->resident.begin(), b->resident.end(), q));
        }
        tb = build_tables(b);
        done_cv_.notify_all();
        cv_.notify_all();
        }
        apply_tables(b, tb);
      }
    } catch (const Error& e) {
      std::vector<Request*> v;
      {
        std::lock_guard<std::mutex> g(mu_);
        v = b->resident;
        b->resident.clear();
        v.insert(v.end(), b->pending.begin(), b->pending.end());
        b->pending.clear();
        b->quit = true;
      }
      fail_all(v, e.code, e.what());
      break;
    }
  }
  // abandon whatever is left (server stop) and release the batch
  std::vector<Request*> left;
  {
    std::lock_guard<std::mutex> g(mu_);
    left = b->resident;
    left.insert(left.end(), b->pending.begin(), b->pending.end());
    b->resident.clear();
    b->pending.clear();
  }
  if (!left.empty()) fail_all(left, SP_EAGAIN, "server stopped before the request finished");
  b->solver.reset();
  b->stage.release();
  b->lab.release();
  std::lock_guard<std::mutex> g(mu_);
  used_ -= b->bytes;
  b->exited = true;
  cv_.notify_all();
}

bool Server::poll(int64_t ticket) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = reqs_.find(ticket);
  SP_REQUIRE(it != reqs_.end(), SP_ENOTFOUND, "unknown ticket");
  return it->second->done;
}

bool Server::wait(int64_t ticket, double timeout_s) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = reqs_.find(ticket);
  SP_REQUIRE(it != reqs_.end(), SP_ENOTFOUND, "unknown ticket");
  Request* q = it->second.get();
  return done_cv_.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return q->done; });
}

int Server::fetch(int64_t ticket, double* u_out, int32_t* labels, double* lambda, double* seps,
                  double* energy, double* latency_s) {
  std::unique_ptr<Request> q;
  {
    std::lock_guard<std::mutex> g(mu_);
    auto it = reqs_.find(ticket);
    SP_REQUIRE(it != reqs_.end(), SP_ENOTFOUND, "unknown ticket");
    if (!it->second->done) return SP_EAGAIN;
    q = std::move(it->second);
    reqs_.erase(it);
  }
  if (q->error != SP_OK) throw Error(q->error, q->error_msg);
  if (u_out) {
    const double* src = q->u_out.data();
    par_for(q->u_out.n, [&](size_t lo, size_t hi) { std::copy(src + lo, src + hi, u_out + lo); });
  }
  if (labels) std::copy(q->labels.begin(), q->labels.end(), labels);
  if (lambda) std::copy(q->lam.begin(), q->lam.end(), lambda);
  if (seps) std::copy(q->seps.begin(), q->seps.end(), seps);
  if (energy) std::copy(q->energy.begin(), q->energy.end(), energy);
  if (latency_s) *latency_s = q->t_done - q->t_submit;
  return SP_OK;
}

void Server::request_stats(int64_t ticket, int64_t* col_iters, int64_t* steps) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = reqs_.find(ticket);
  SP_REQUIRE(it != reqs_.end(), SP_ENOTFOUND, "unknown ticket");
  const Request& q = *it->second;
  SP_REQUIRE(q.done, SP_EAGAIN, "request not finished");
  if (col_iters) *col_iters = q.col_iters;
  if (steps) *steps = q.steps;
}

void Server::stats(double* p50, double* p99, double* cdof_per_s, int64_t* completed) {
  std::lock_guard<std::mutex> g(mu_);
  std::vector<double> v = latencies_;
  std::sort(v.begin(), v.end());
  auto pct = [&](double p) {
    if (v.empty()) return 0.0;
    size_t k = size_t(std::ceil(p * double(v.size()))) ;
    k = std::min(std::max<size_t>(k, 1), v.size());
    return v[k - 1];
  };
  if (p50) *p50 = pct(0.50);
  if (p99) *p99 = pct(0.99);
  if (cdof_per_s) *cdof_per_s = (t_last_ > t_first_ && t_first_ >= 0) ? cdof_done_ / (t_last_ - t_first_) : 0.0;
  if (completed) *completed = completed_;
}

}  // namespace sp
