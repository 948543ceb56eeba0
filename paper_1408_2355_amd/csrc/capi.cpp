// extern "C" entry points of libsegpart (declared in include/segpart.h).
// Every call catches all exceptions and turns them into a status code plus a
// thread-local message.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "continuation.h"
#include "partition.h"
#include "engine.h"
#include "server.h"

struct sp_mesh {
  std::unique_ptr<sp::Mesh> m;
};

struct sp_state {
  sp::Mesh* mesh = nullptr;
  std::unique_ptr<sp::Solver> solver;
};

struct sp_server {
  std::unique_ptr<sp::Server> srv;
};

namespace {

thread_local std::string g_err;

template <class F>
int guard(F&& f) {
  try {
    g_err.clear();
    sp::reap_deferred();
    return f();
  } catch (const sp::Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return SP_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return SP_EDEVICE;
  } catch (...) {
    g_err = "unknown error";
    return SP_EDEVICE;
  }
}

sp::BatchSpec make_spec(int32_t nres, const int32_t* m, const double* eps) {
  sp::validate_batch(nres, m, eps);
  sp::BatchSpec s;
  s.m.assign(m, m + nres);
  s.eps.assign(eps, eps + nres);
  return s;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

const char* sp_last_error(void) { return g_err.c_str(); }

int sp_version(int* major, int* minor) {
  if (major) *major = SP_VERSION_MAJOR;
  if (minor) *minor = SP_VERSION_MINOR;
  return SP_OK;
}

void sp_params_default(sp_params* p, double tau) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tau = tau;
  p->n_steps = 100;
  p->stop_tol = 1e-6;
  p->max_steps = 1000000;
  p->energy_every = tau > 0 ? std::max<int64_t>(1, std::llround(0.1 / tau)) : 1;
  p->precision = SP_MIXED;
  p->cg_rtol = 1e-10;
  p->cg_max_iter = 500;
  p->inner_rtol = 1e-5;
  p->max_outer = 8;
  p->check_every = 8;
  p->extrapolate = 5;
  p->precond = SP_PRECOND_CHEB1;
}

int sp_mesh_create(int64_t n_vert, const double* xyz, int64_t n_tri, const int32_t* tri,
                   sp_mesh** out) {
  return guard([&] {
    SP_REQUIRE(out != nullptr, SP_EINVAL, "NULL out");
    *out = nullptr;
    std::unique_ptr<sp_mesh> h(new sp_mesh());
    h->m.reset(sp::mesh_create(n_vert, xyz, n_tri, tri));
    *out = h.release();
    return SP_OK;
  });
}

int sp_mesh_info(const sp_mesh* mesh, int64_t* n_vert, int64_t* n_tri, int64_t* nnz,
                 double* area) {
  return guard([&] {
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    if (n_vert) *n_vert = mesh->m->n;
    if (n_tri) *n_tri = mesh->m->nt;
    if (nnz) *nnz = mesh->m->nnz;
    if (area) *area = mesh->m->area;
    return SP_OK;
  });
}

int sp_mesh_export(const sp_mesh* mesh, int32_t which, int64_t* row_ptr, int32_t* col,
                   double* val) {
  return guard([&] {
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    SP_REQUIRE(which == SP_MAT_M || which == SP_MAT_A, SP_EINVAL, "which must be SP_MAT_M or SP_MAT_A");
    SP_REQUIRE(row_ptr && col && val, SP_EINVAL, "NULL output");
    const sp::Mesh& m = *mesh->m;
    const size_t cnt = size_t(m.W) * m.n;
    std::vector<double> v(cnt);
    const sp::DevBuf<double>& src = which == SP_MAT_M ? m.M64 : m.A64;
    SP_HIP(hipMemcpy(v.data(), src.p, cnt * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<std::pair<int32_t, double>> row;
    int64_t pos = 0;
    row_ptr[0] = 0;
    for (int64_t r = 0; r < m.n; ++r) {
      const int64_t i = m.iperm[r];
      row.clear();
      for (int k = 0; k < m.W; ++k) {
        const int32_t c = m.h_cols[size_t(k) * m.n + i];
        if (k > 0 && c == i) continue;  // padding slot
        row.push_back({m.perm[c], v[size_t(k) * m.n + i]});
      }
      std::sort(row.begin(), row.end());
      for (auto& e : row) {
        col[pos] = e.first;
        val[pos] = e.second;
        ++pos;
      }
      row_ptr[r + 1] = pos;
    }
    return SP_OK;
  });
}

void sp_mesh_destroy(sp_mesh* mesh) { delete mesh; }

int sp_solve(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts, const int32_t* m,
             const double* eps, const double* u0, double* u_out, int32_t* labels,
             int32_t* labels_argmax, double* lambda, double* s_eps, double* energy,
             sp_stats* stats) {
  return guard([&] {
    const double t0 = now_s();
    SP_REQUIRE(prm, SP_EINVAL, "NULL params");
    sp::validate_params(*prm);
    sp::BatchSpec spec = make_spec(n_restarts, m, eps);
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    sp::Solver S(mesh->m.get(), *prm, spec, nullptr);  // private stream
    S.upload_host(u0, true);
    if (prm->n_steps > 0)
      S.step(prm->n_steps);
    else
      S.run_to_stop();
    S.energy_to_host(lambda, s_eps, energy);
    if (labels || labels_argmax) S.labels_host(labels, labels_argmax);
    if (u_out) S.download_host(u_out);
    sp_stats st = S.stats();
    st.seconds = now_s() - t0;
    if (stats) *stats = st;
    return st.converged ? SP_OK : SP_ENOCONV;
  });
}

int sp_solve_async(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts,
                   const int32_t* m, const double* eps, const double* d_u0, double* d_u_out,
                   int32_t* d_labels, int32_t* d_labels_argmax, double* d_lambda,
                   double* d_s_eps, double* d_energy, void* hip_stream) {
  return guard([&] {
    SP_REQUIRE(prm, SP_EINVAL, "NULL params");
    sp::validate_params(*prm);
    SP_REQUIRE(prm->n_steps > 0, SP_EINVAL, "sp_solve_async needs n_steps > 0");
    sp::BatchSpec spec = make_spec(n_restarts, m, eps);
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);  // NULL = default stream
    auto* S = new sp::Solver(mesh->m.get(), *prm, spec, &s);
    int rc = SP_OK;
    try {
      S->record_history = false;
      S->upload_device(d_u0, true, false);
      S->step(prm->n_steps);
      S->energy();
      const int R = S->R(), nres = S->nres();
      if (d_lambda)
        SP_HIP(hipMemcpyAsync(d_lambda, S->d_lam(), R * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (d_s_eps)
        SP_HIP(hipMemcpyAsync(d_s_eps, S->d_seps(), nres * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (d_energy)
        SP_HIP(hipMemcpyAsync(d_energy, S->d_energy(), nres * sizeof(double), hipMemcpyDeviceToDevice,
                              s));
      if (d_labels || d_labels_argmax) S->labels_device(d_labels, d_labels_argmax);
      if (d_u_out) S->download_device(d_u_out);
    } catch (...) {
      delete S;
      throw;
    }
    // The solver's buffers must outlive the enqueued work: free them from a
    // host callback once the stream reaches this point.
    S->detach();
    hipError_t e = hipLaunchHostFunc(
        s, [](void* p) { sp::defer_delete(static_cast<sp::Solver*>(p)); }, S);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);
      delete S;
      throw sp::Error(SP_EDEVICE, std::string("hipLaunchHostFunc: ") + hipGetErrorString(e));
    }
    return rc;
  });
}

int sp_solve_async_noalloc(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts,
                           const int32_t* m, const double* eps, const double* d_u0,
                           double* d_u_out, int32_t* d_labels, int32_t* d_labels_argmax,
                           double* d_lambda, double* d_s_eps, double* d_energy,
                           void* hip_stream) {
  return guard([&] {
    SP_REQUIRE(prm, SP_EINVAL, "NULL params");
    sp::validate_params(*prm);
    SP_REQUIRE(prm->n_steps > 0, SP_EINVAL, "sp_solve_async_noalloc needs n_steps > 0");
    sp::BatchSpec spec = make_spec(n_restarts, m, eps);
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);  // NULL = default stream
    // the current device's scratch (located once per device); every work
    // buffer of the batch comes from it, so a batch that does not fit is
    // rejected (SP_ENOMEM) before any work is enqueued
    sp::Arena ar = sp::noalloc_scratch();
    sp::Solver S(mesh->m.get(), *prm, spec, &s, 0, 0, &ar);
    S.record_history = false;
    S.upload_device(d_u0, true, false);
    S.step(prm->n_steps);
    S.energy();
    const int R = S.R(), nres = S.nres();
    if (d_lambda)
      SP_HIP(hipMemcpyAsync(d_lambda, S.d_lam(), R * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_s_eps)
      SP_HIP(hipMemcpyAsync(d_s_eps, S.d_seps(), nres * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_energy)
      SP_HIP(hipMemcpyAsync(d_energy, S.d_energy(), nres * sizeof(double), hipMemcpyDeviceToDevice,
                            s));
    if (d_labels || d_labels_argmax) S.labels_device(d_labels, d_labels_argmax);
    if (d_u_out) S.download_device(d_u_out);
    // the work stays enqueued: the solver's host object goes, its buffers
    // (the scratch) stay in use until the stream passes this point
    S.detach();
    return SP_OK;
  });
}

int sp_state_create(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts,
                    const int32_t* m, const double* eps, const double* u0, void* hip_stream,
                    sp_state** out) {
  return guard([&] {
    SP_REQUIRE(out != nullptr, SP_EINVAL, "NULL out");
    *out = nullptr;
    SP_REQUIRE(prm, SP_EINVAL, "NULL params");
    sp::validate_params(*prm);
    sp::BatchSpec spec = make_spec(n_restarts, m, eps);
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    std::unique_ptr<sp_state> st(new sp_state());
    st->mesh = mesh->m.get();
    hipStream_t hs = reinterpret_cast<hipStream_t>(hip_stream);
    st->solver.reset(new sp::Solver(mesh->m.get(), *prm, spec, hs ? &hs : nullptr));
    st->solver->upload_host(u0, true);
    *out = st.release();
    return SP_OK;
  });
}

int sp_state_step(sp_state* st, int64_t k) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    SP_REQUIRE(k >= 1, SP_EINVAL, "k must be >= 1");
    st->solver->step(k);
    st->solver->sync();
    return st->solver->converged() ? SP_OK : SP_ENOCONV;
  });
}

int sp_state_stage(sp_state* st, int32_t stage) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    switch (stage) {
      case SP_STAGE_HEAT: st->solver->stage_heat(); break;
      case SP_STAGE_NODE: st->solver->stage_node(); break;
      case SP_STAGE_NORM: st->solver->stage_norm(); break;
      default: throw sp::Error(SP_EINVAL, "unknown stage");
    }
    st->solver->sync();
    return SP_OK;
  });
}

int sp_state_energy(sp_state* st, double* lambda, double* s_eps, double* energy) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    st->solver->energy_to_host(lambda, s_eps, energy);
    return SP_OK;
  });
}

int sp_state_multipliers(sp_state* st, double* lambda_eps) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    st->solver->multipliers_to_host(lambda_eps);
    return SP_OK;
  });
}

int sp_state_read(sp_state* st, double* u, int64_t* step) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    if (u) st->solver->download_host(u);
    if (step) *step = st->solver->steps_done();
    return SP_OK;
  });
}

int sp_state_write(sp_state* st, const double* u, int64_t step, int32_t normalise) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    SP_REQUIRE(step >= 0, SP_EINVAL, "step must be >= 0");
    st->solver->upload_host(u, normalise != 0);
    st->solver->set_steps_done(step);
    return SP_OK;
  });
}

int sp_state_checkpoint_size(sp_state* st, int64_t* bytes) {
  return guard([&] {
    SP_REQUIRE(st && st->solver && bytes, SP_EINVAL, "NULL state or output");
    *bytes = st->solver->checkpoint_size();
    return SP_OK;
  });
}

int sp_state_checkpoint(sp_state* st, void* buf, int64_t bytes) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    st->solver->checkpoint(buf, bytes);
    return SP_OK;
  });
}

int sp_state_restore(sp_state* st, const void* buf, int64_t bytes) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    st->solver->restore(buf, bytes);
    return SP_OK;
  });
}

int sp_state_labels(sp_state* st, int32_t* labels, int32_t* labels_argmax) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    st->solver->labels_host(labels, labels_argmax);
    return SP_OK;
  });
}

int sp_state_history(sp_state* st, int32_t r, int64_t cap, int64_t* steps, double* energies,
                     int64_t* count) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    const auto& h = st->solver->history();
    SP_REQUIRE(r >= 0 && r < int32_t(h.size()), SP_EINVAL, "restart index out of range");
    const auto& v = h[r];
    if (count) *count = int64_t(v.size());
    for (int64_t i = 0; i < cap && i < int64_t(v.size()); ++i) {
      if (steps) steps[i] = v[i].first;
      if (energies) energies[i] = v[i].second;
    }
    return SP_OK;
  });
}

int sp_state_stats(sp_state* st, sp_stats* stats) {
  return guard([&] {
    SP_REQUIRE(st && st->solver && stats, SP_EINVAL, "NULL state or stats");
    *stats = st->solver->stats();
    return SP_OK;
  });
}

int sp_state_profile(sp_state* st, int32_t enable) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    st->solver->profile(enable != 0);
    return SP_OK;
  });
}

int sp_state_kernel_time(sp_state* st, int32_t which, int64_t* launches, double* total_ms,
                         double* bytes_per_launch) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    st->solver->kernel_time(which, launches, total_ms, bytes_per_launch);
    return SP_OK;
  });
}

int sp_state_tiling(sp_state* st, int32_t* lanes_per_row, int32_t* rows_per_chunk,
                    int32_t* groups_per_xcd, double* matvec_us) {
  return guard([&] {
    SP_REQUIRE(st && st->solver, SP_EINVAL, "NULL state");
    const sp::Tile& t = st->solver->gather_tile();
    if (lanes_per_row) *lanes_per_row = t.tg;
    if (rows_per_chunk) *rows_per_chunk = t.ch;
    if (groups_per_xcd) *groups_per_xcd = t.nper;
    if (matvec_us) *matvec_us = st->solver->tuned_us();
    return SP_OK;
  });
}

void sp_state_destroy(sp_state* st) { delete st; }

int sp_server_create(int64_t hbm_budget_bytes, int32_t max_batch_columns, sp_server** out) {
  return guard([&] {
    SP_REQUIRE(out != nullptr, SP_EINVAL, "NULL out");
    *out = nullptr;
    SP_REQUIRE(hbm_budget_bytes > 0, SP_EINVAL, "hbm budget must be > 0");
    SP_REQUIRE(max_batch_columns >= 0, SP_EINVAL, "max_batch_columns must be >= 0");
    std::unique_ptr<sp_server> h(new sp_server());
    h->srv.reset(new sp::Server(hbm_budget_bytes, max_batch_columns ? max_batch_columns : 4096));
    *out = h.release();
    return SP_OK;
  });
}

int sp_server_submit(sp_server* srv, const sp_mesh* mesh, const sp_params* prm,
                     int32_t n_restarts, const int32_t* m, const double* eps, const double* u0,
                     int64_t* ticket) {
  return guard([&] {
    SP_REQUIRE(srv && srv->srv && prm && ticket, SP_EINVAL, "NULL argument");
    sp::validate_params(*prm);
    SP_REQUIRE(prm->n_steps > 0, SP_EINVAL, "server requests need n_steps > 0");
    sp::BatchSpec spec = make_spec(n_restarts, m, eps);
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    *ticket = srv->srv->submit(mesh->m.get(), *prm, spec, u0);
    return SP_OK;
  });
}

int sp_server_poll(sp_server* srv, int64_t ticket, int32_t* done) {
  return guard([&] {
    SP_REQUIRE(srv && srv->srv && done, SP_EINVAL, "NULL argument");
    *done = srv->srv->poll(ticket) ? 1 : 0;
    return SP_OK;
  });
}

int sp_server_wait(sp_server* srv, int64_t ticket, double timeout_s) {
  return guard([&] {
    SP_REQUIRE(srv && srv->srv, SP_EINVAL, "NULL server");
    return srv->srv->wait(ticket, timeout_s) ? SP_OK : SP_EAGAIN;
  });
}

int sp_server_fetch(sp_server* srv, int64_t ticket, double* u_out, int32_t* labels,
                    double* lambda, double* s_eps, double* energy, double* latency_s) {
  return guard([&] {
    SP_REQUIRE(srv && srv->srv, SP_EINVAL, "NULL server");
    return srv->srv->fetch(ticket, u_out, labels, lambda, s_eps, energy, latency_s);
  });
}

int sp_server_stats(sp_server* srv, double* p50_s, double* p99_s, double* cdof_per_s,
                    int64_t* completed) {
  return guard([&] {
    SP_REQUIRE(srv && srv->srv, SP_EINVAL, "NULL server");
    srv->srv->stats(p50_s, p99_s, cdof_per_s, completed);
    return SP_OK;
  });
}

int sp_server_request_stats(sp_server* srv, int64_t ticket, int64_t* col_iters, int64_t* steps) {
  return guard([&] {
    SP_REQUIRE(srv && srv->srv, SP_EINVAL, "NULL server");
    srv->srv->request_stats(ticket, col_iters, steps);
    return SP_OK;
  });
}

void sp_server_destroy(sp_server* srv) { delete srv; }

}  // extern "C"

int sp_mesh_refine(const sp_mesh* coarse, sp_project_fn project, void* ctx, sp_mesh** fine) {
  return guard([&] {
    SP_REQUIRE(fine != nullptr, SP_EINVAL, "NULL fine");
    *fine = nullptr;
    SP_REQUIRE(coarse && coarse->m, SP_EINVAL, "NULL mesh");
    std::unique_ptr<sp_mesh> h(new sp_mesh());
    h->m.reset(sp::mesh_refine(*coarse->m, project, ctx));
    *fine = h.release();
    return SP_OK;
  });
}

int sp_mesh_parents(const sp_mesh* fine, int32_t* parents, int64_t* n_coarse) {
  return guard([&] {
    SP_REQUIRE(fine && fine->m, SP_EINVAL, "NULL mesh");
    SP_REQUIRE(fine->m->n_coarse > 0, SP_EINVAL, "mesh was not made by sp_mesh_refine");
    if (parents) std::memcpy(parents, fine->m->parents.data(), fine->m->parents.size() * sizeof(int32_t));
    if (n_coarse) *n_coarse = fine->m->n_coarse;
    return SP_OK;
  });
}

int sp_prolong(const sp_mesh* fine, int32_t n_cols, const double* u_coarse, double* u_fine) {
  return guard([&] {
    SP_REQUIRE(fine && fine->m, SP_EINVAL, "NULL mesh");
    SP_REQUIRE(fine->m->n_coarse > 0, SP_EINVAL, "mesh was not made by sp_mesh_refine");
    SP_REQUIRE(n_cols >= 0, SP_EINVAL, "n_cols must be >= 0");
    SP_REQUIRE(n_cols == 0 || (u_coarse && u_fine), SP_EINVAL, "NULL state");
    const sp::Mesh& F = *fine->m;
    if (n_cols == 0) return SP_OK;
    sp::DevBuf<double> c(size_t(n_cols) * F.n_coarse), f(size_t(n_cols) * F.n);
    SP_HIP(hipMemcpy(c.p, u_coarse, c.bytes(), hipMemcpyHostToDevice));
    sp::k::prolong(F, n_cols, c.p, f.p, nullptr);
    SP_HIP(hipMemcpy(u_fine, f.p, f.bytes(), hipMemcpyDeviceToHost));
    return SP_OK;
  });
}

int sp_continue(const sp_mesh* mesh0, const sp_params* prm, int32_t n_restarts, int32_t m,
                const double* u0, int32_t n_levels, const sp_level* levels,
                sp_project_fn project, void* ctx, sp_level_result* results, double* lambda,
                sp_mesh** final_mesh, double* u_final, sp_level_fn on_level,
                void* level_ctx) {
  return guard([&] {
    if (final_mesh) *final_mesh = nullptr;
    SP_REQUIRE(mesh0 && mesh0->m && prm, SP_EINVAL, "NULL mesh or params");
    sp::ContinuationOut o =
        sp::run_continuation(mesh0->m.get(), *prm, n_restarts, m, u0, n_levels, levels, project,
                             ctx, results, lambda, u_final, on_level, level_ctx);
    if (final_mesh && o.mesh) {
      std::unique_ptr<sp_mesh> h(new sp_mesh());
      h->m = std::move(o.mesh);
      *final_mesh = h.release();
    }
    return o.converged ? SP_OK : SP_ENOCONV;
  });
}

int sp_region_eigen(const sp_mesh* mesh, int32_t n_restarts, const int32_t* m,
                    const int32_t* labels, int32_t interior, const double* u0, double shift,
                    double tol, int32_t max_iter, double* lambda, double* u_out,
                    int32_t* iterations) {
  return guard([&] {
    SP_REQUIRE(mesh && mesh->m && labels && lambda, SP_EINVAL, "NULL argument");
    SP_REQUIRE(std::isfinite(shift) && shift > 0, SP_EINVAL, "shift must be > 0");
    SP_REQUIRE(n_restarts >= 1 && m, SP_EINVAL, "need n_restarts >= 1");
    std::vector<double> eps(n_restarts, 1.0);  // unused by the restricted solve
    sp::BatchSpec spec = make_spec(n_restarts, m, eps.data());
    sp_params p;
    sp_params_default(&p, shift);
    p.precision = SP_FP64;
    p.cg_rtol = 1e-12;
    p.cg_max_iter = 100000;
    p.n_steps = 1;
    p.energy_every = 0;
    sp::Solver S(mesh->m.get(), p, spec, nullptr);
    const int R = S.R();
    const int64_t n = mesh->m->n;
    std::vector<double> ones;
    if (!u0) {
      ones.assign(size_t(R) * n, 1.0);
      u0 = ones.data();
    }
    S.upload_host(u0, false);
    S.set_region_mask(labels, interior != 0);
    const int it = S.region_eigen(tol, max_iter, lambda);
    if (iterations) *iterations = it < 0 ? -it : it;
    if (u_out) S.download_host(u_out);
    return it > 0 ? SP_OK : SP_ENOCONV;
  });
}

int sp_region_graph(const sp_mesh* mesh, int32_t n_restarts, const int32_t* m,
                    const int32_t* labels, uint8_t* adjacency, int32_t* sides) {
  return guard([&] {
    SP_REQUIRE(mesh && mesh->m, SP_EINVAL, "NULL mesh");
    sp::region_graph(*mesh->m, n_restarts, m, labels, adjacency, sides);
    return SP_OK;
  });
}

