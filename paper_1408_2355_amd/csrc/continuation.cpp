// Mesh refinement and the level loop of the convergence study in eps
// (Section 3.1): refine, carry the minimiser over, shrink eps and tau, run to
// the stopping rule of Section 2.2, repeat.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "continuation.h"
#include "engine.h"
#include "internal.h"

namespace sp {

Mesh* mesh_refine(const Mesh& c, ProjectFn project, void* ctx) {
  const int64_t n = c.n, nt = c.nt;
  SP_REQUIRE(int64_t(c.h_tri.size()) == 3 * nt && int64_t(c.h_xyz.size()) == 3 * n, SP_EINVAL,
             "refine: mesh has no host geometry");
  // unique edges (a, b), a < b, in lexicographic order: new vertex n + j
  std::vector<uint64_t> e(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      uint64_t a = uint32_t(c.h_tri[3 * t + k]), b = uint32_t(c.h_tri[3 * t + (k + 1) % 3]);
      if (a > b) std::swap(a, b);
      e[3 * t + k] = (a << 32) | b;
    }
  std::sort(e.begin(), e.end());
  e.erase(std::unique(e.begin(), e.end()), e.end());
  const int64_t ne = int64_t(e.size());
  const int64_t nf = n + ne;
  SP_REQUIRE(nf < (int64_t(1) << 31) && 4 * nt < (int64_t(1) << 29), SP_EINVAL,
             "refine: refined mesh too large");
  std::vector<double> xyz(3 * nf);
  std::copy(c.h_xyz.begin(), c.h_xyz.end(), xyz.begin());
  std::vector<int32_t> parents(2 * ne);
  for (int64_t j = 0; j < ne; ++j) {
    const int32_t a = int32_t(e[j] >> 32), b = int32_t(e[j] & 0xffffffffu);
    parents[2 * j] = a;
    parents[2 * j + 1] = b;
    for (int k = 0; k < 3; ++k)
      xyz[3 * (n + j) + k] = 0.5 * (c.h_xyz[3 * a + k] + c.h_xyz[3 * b + k]);
  }
  if (project && ne > 0) project(xyz.data() + 3 * n, ne, ctx);
  auto mid = [&](int32_t a, int32_t b) {
    const uint64_t key = a < b ? (uint64_t(uint32_t(a)) << 32) | uint32_t(b)
                               : (uint64_t(uint32_t(b)) << 32) | uint32_t(a);
    return int32_t(n + (std::lower_bound(e.begin(), e.end(), key) - e.begin()));
  };
  std::vector<int32_t> tri(12 * nt);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t a = c.h_tri[3 * t], b = c.h_tri[3 * t + 1], cc = c.h_tri[3 * t + 2];
    const int32_t ab = mid(a, b), bc = mid(b, cc), ca = mid(cc, a);
    const int32_t f[12] = {a, ab, ca, b, bc, ab, cc, ca, bc, ab, bc, ca};
    std::copy(f, f + 12, tri.begin() + 12 * t);
  }
  std::unique_ptr<Mesh> F(mesh_create(nf, xyz.data(), 4 * nt, tri.data()));
  F->n_coarse = n;
  F->parents = std::move(parents);
  F->parents_d.alloc(F->parents.size());
  SP_HIP(hipMemcpy(F->parents_d.p, F->parents.data(), F->parents_d.bytes(), hipMemcpyHostToDevice));
  return F.release();
}

namespace {
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

ContinuationOut run_continuation(Mesh* mesh0, const sp_params& prm, int nres, int m,
                                 const double* u0, int nlev, const sp_level* levels,
                                 ProjectFn project, void* ctx, sp_level_result* results,
                                 double* lambda, double* u_final, sp_level_fn on_level,
                                 void* level_ctx) {
  SP_REQUIRE(mesh0 && u0 && levels && results, SP_EINVAL, "continue: NULL argument");
  SP_REQUIRE(m >= 1 && nres >= 1 && nlev >= 1, SP_EINVAL,
             "continue: need m >= 1, n_restarts >= 1 and n_levels >= 1");
  SP_REQUIRE(int64_t(nres) * m <= (int64_t(1) << 24), SP_EINVAL, "continue: too many columns");
  const int R = nres * m;
  SP_REQUIRE(levels[0].refine == 0, SP_EINVAL, "continue: level 0 cannot refine");
  for (int l = 0; l < nlev; ++l)
    SP_REQUIRE(std::isfinite(levels[l].eps) && levels[l].eps > 0 && std::isfinite(levels[l].tau) &&
                   levels[l].tau > 0,
               SP_EINVAL, "continue: level " + std::to_string(l) + " needs eps > 0 and tau > 0");
  ContinuationOut out;
  Mesh* mesh = mesh0;
  hipStream_t s;
  SP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  } guard{s};
  DevBuf<double> u(size_t(R) * mesh->n);
  SP_HIP(hipMemcpyAsync(u.p, u0, u.bytes(), hipMemcpyHostToDevice, s));
  for (int l = 0; l < nlev; ++l) {
    const double t0 = now_s();
    if (levels[l].refine) {
      std::unique_ptr<Mesh> fine(mesh_refine(*mesh, project, ctx));
      DevBuf<double> uf(size_t(R) * fine->n);
      k::prolong(*fine, R, u.p, uf.p, s);
      SP_HIP(hipStreamSynchronize(s));
      u = std::move(uf);
      out.mesh = std::move(fine);  // frees the previous refined mesh
      mesh = out.mesh.get();
    }
    sp_params p = prm;
    p.tau = levels[l].tau;
    p.energy_every = std::max<int64_t>(1, std::llround(0.1 / p.tau));
    BatchSpec spec;
    spec.m.assign(nres, m);
    spec.eps.assign(nres, levels[l].eps);
    Solver S(mesh, p, spec, &s);
    S.record_history = p.n_steps == 0;  // the stopping rule reads the energies
    S.upload_device(u.p, true, true);
    if (p.n_steps > 0)
      S.step(p.n_steps);
    else
      S.run_to_stop();
    std::vector<double> lam(R), seps(nres), E(nres);
    S.energy_to_host(lam.data(), seps.data(), E.data());
    S.download_device(u.p);
    SP_HIP(hipStreamSynchronize(s));
    const sp_stats st = S.stats();
    const double secs = now_s() - t0;
    for (int r = 0; r < nres; ++r) {
      sp_level_result& o = results[size_t(l) * nres + r];
      o.n_vert = mesh->n;
      o.steps = p.n_steps > 0 ? p.n_steps : S.restart_steps[r];
      o.energy = E[r];
      o.s_eps = seps[r];
      o.converged = st.converged;
      o.reserved = 0;
      o.seconds = secs;
    }
    if (lambda) std::copy(lam.begin(), lam.end(), lambda + size_t(l) * R);
    out.converged = out.converged && st.converged;
    if (on_level) on_level(l, results + size_t(l) * nres, level_ctx);
  }
  if (u_final) {
    SP_HIP(hipMemcpyAsync(u_final, u.p, u.bytes(), hipMemcpyDeviceToHost, s));
    SP_HIP(hipStreamSynchronize(s));
  }
  return out;
}

}  // namespace sp
