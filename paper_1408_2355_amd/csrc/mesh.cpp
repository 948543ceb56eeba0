// Mesh set-up: validation of the triangulated surface, vertex renumbering for
// locality, the ELL sparsity pattern, and the GPU assembly of M and A.
//
// Section 2.1 of the paper: Gamma_h is a closed surface made of flat
// triangles whose vertices lie on Gamma; S_h is the continuous piecewise
// affine space on it.  Validation enforces "closed": every edge belongs to
// exactly two triangles.  The numeric assembly runs on the GPU (kernels.hip);
// this file builds only index structures.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>

#include "internal.h"

namespace sp {

namespace {

// Reverse Cuthill-McKee order of the vertex graph: breadth-first layers
// from a pseudo-peripheral start, neighbours visited by increasing degree,
// the whole order reversed.  Neighbouring vertices end up at nearby indices,
// so the rows an ELL row gathers from stay close in memory (and in cache).
std::vector<int32_t> rcm_order(int64_t n, const std::vector<int64_t>& ptr,
                               const std::vector<int32_t>& adj) {
  std::vector<int32_t> deg(n);
  for (int64_t i = 0; i < n; ++i) deg[i] = int32_t(ptr[i + 1] - ptr[i]);
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int32_t> level(n, -1);

  auto bfs_far = [&](int32_t s) {
    // returns a vertex of the last BFS layer with the smallest degree
    std::fill(level.begin(), level.end(), -1);
    std::queue<int32_t> q;
    q.push(s);
    level[s] = 0;
    int32_t best = s;
    while (!q.empty()) {
      int32_t v = q.front();
      q.pop();
      if (level[v] > level[best] || (level[v] == level[best] && deg[v] < deg[best])) best = v;
      for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) {
        int32_t w = adj[e];
        if (level[w] < 0) { level[w] = level[v] + 1; q.push(w); }
      }
    }
    return best;
  };

  std::vector<int32_t> nb;
  for (int64_t root = 0; root < n; ++root) {
    if (seen[root]) continue;
    int32_t s = bfs_far(bfs_far(int32_t(root)));
    std::queue<int32_t> q;
    q.push(s);
    seen[s] = 1;
    while (!q.empty()) {
      int32_t v = q.front();
      q.pop();
      order.push_back(v);
      nb.clear();
      for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e)
        if (!seen[adj[e]]) nb.push_back(adj[e]);
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
        return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
      });
      for (int32_t w : nb) { seen[w] = 1; q.push(w); }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

}  // namespace

Mesh* mesh_create(int64_t n, const double* xyz, int64_t nt, const int32_t* tri) {
  SP_REQUIRE(xyz && tri, SP_EINVAL, "mesh: NULL xyz or tri");
  SP_REQUIRE(n >= 3 && nt >= 1, SP_EINVAL, "mesh: need n_vert >= 3 and n_tri >= 1");
  SP_REQUIRE(n < (int64_t(1) << 31) && nt < (int64_t(1) << 29), SP_EINVAL, "mesh: too large");
  for (int64_t i = 0; i < 3 * n; ++i)
    SP_REQUIRE(std::isfinite(xyz[i]), SP_EINVAL, "mesh: non-finite coordinate");

  // --- validation: indices, distinct corners, nonzero area, closedness ------
  std::vector<char> used(n, 0);
  double area = 0.0;
  for (int64_t t = 0; t < nt; ++t) {
    int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    SP_REQUIRE(a >= 0 && a < n && b >= 0 && b < n && c >= 0 && c < n, SP_EMESH,
               "mesh: triangle " + std::to_string(t) + " has an index out of range");
    SP_REQUIRE(a != b && b != c && a != c, SP_EMESH,
               "mesh: triangle " + std::to_string(t) + " repeats a vertex");
    used[a] = used[b] = used[c] = 1;
    const double* p = xyz + 3 * a;
    const double* q = xyz + 3 * b;
    const double* r = xyz + 3 * c;
    double u[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    double v[3] = {r[0] - p[0], r[1] - p[1], r[2] - p[2]};
    double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
           cz = u[0] * v[1] - u[1] * v[0];
    double twice = std::sqrt(cx * cx + cy * cy + cz * cz);
    double scale = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    SP_REQUIRE(twice > 1e-14 * scale, SP_EMESH,
               "mesh: triangle " + std::to_string(t) + " has (near) zero area");
    area += 0.5 * twice;
  }
  for (int64_t i = 0; i < n; ++i)
    SP_REQUIRE(used[i], SP_EMESH, "mesh: vertex " + std::to_string(i) + " is in no triangle");

  std::vector<uint64_t> edges(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      uint64_t a = uint32_t(tri[3 * t + k]), b = uint32_t(tri[3 * t + (k + 1) % 3]);
      if (a > b) std::swap(a, b);
      edges[3 * t + k] = (a << 32) | b;
    }
  std::sort(edges.begin(), edges.end());
  std::vector<uint64_t> uedge;
  uedge.reserve(edges.size() / 2);
  for (size_t i = 0; i < edges.size();) {
    size_t j = i;
    while (j < edges.size() && edges[j] == edges[i]) ++j;
    SP_REQUIRE(j - i == 2, SP_EMESH,
               "mesh: edge (" + std::to_string(edges[i] >> 32) + "," +
                   std::to_string(edges[i] & 0xffffffffu) + ") belongs to " + std::to_string(j - i) +
                   " triangles; a closed surface needs exactly 2");
    uedge.push_back(edges[i]);
    i = j;
  }

  // --- vertex graph and renumbering ----------------------------------------
  std::vector<int64_t> ptr(n + 1, 0);
  for (uint64_t e : uedge) { ptr[(e >> 32) + 1]++; ptr[(e & 0xffffffffu) + 1]++; }
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  std::vector<int32_t> adj(ptr[n]);
  {
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (uint64_t e : uedge) {
      int32_t a = int32_t(e >> 32), b = int32_t(e & 0xffffffffu);
      adj[fill[a]++] = b;
      adj[fill[b]++] = a;
    }
  }
  std::unique_ptr<Mesh> M(new Mesh());
  M->n = n;
  M->nt = nt;
  M->area = area;
  M->h_xyz.assign(xyz, xyz + 3 * n);
  M->h_tri.assign(tri, tri + 3 * nt);
  M->perm = rcm_order(n, ptr, adj);
  M->iperm.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) M->iperm[M->perm[i]] = int32_t(i);

  int W = 0;
  for (int64_t i = 0; i < n; ++i) W = std::max<int>(W, int(ptr[i + 1] - ptr[i]) + 1);
  SP_REQUIRE(W <= 64, SP_EMESH, "mesh: a vertex has more than 63 neighbours");
  // The row kernels walk slots in unrolled groups of 8; pad the width to a
  // multiple of 8 (padding slots point at the row itself with value 0).
  W = (W + 7) / 8 * 8;
  M->W = W;
  M->nnz = n + int64_t(uedge.size()) * 2;

  // ELL pattern in the new numbering: slot 0 = diagonal, then neighbours by
  // increasing new index; unused slots repeat the row (value stays 0).
  M->h_cols.assign(size_t(W) * n, 0);
  std::vector<int32_t> nb;
  for (int64_t i = 0; i < n; ++i) {
    int32_t old = M->perm[i];
    nb.clear();
    for (int64_t e = ptr[old]; e < ptr[old + 1]; ++e) nb.push_back(M->iperm[adj[e]]);
    std::sort(nb.begin(), nb.end());
    M->h_cols[i] = int32_t(i);
    int k = 1;
    for (int32_t c : nb) M->h_cols[size_t(k++) * n + i] = c;
    for (; k < W; ++k) M->h_cols[size_t(k) * n + i] = int32_t(i);
  }

  // Triangles in the new numbering, sorted by their smallest vertex (the
  // energy kernel walks them in this order), orientation kept.
  std::vector<int32_t> tnew(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) tnew[3 * t + k] = M->iperm[tri[3 * t + k]];
  std::vector<int64_t> tord(nt);
  std::iota(tord.begin(), tord.end(), 0);
  auto tkey = [&](int64_t t) {
    int32_t a = tnew[3 * t], b = tnew[3 * t + 1], c = tnew[3 * t + 2];
    return std::min(a, std::min(b, c));
  };
  std::stable_sort(tord.begin(), tord.end(), [&](int64_t x, int64_t y) { return tkey(x) < tkey(y); });
  std::vector<int32_t> tsorted(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) tsorted[3 * t + k] = tnew[3 * tord[t] + k];

  // Incident (triangle, corner) list per row, in triangle order: the assembly
  // kernel sums element contributions of a row in this fixed order.
  std::vector<int32_t> inc_ptr(n + 1, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) inc_ptr[tsorted[3 * t + k] + 1]++;
  for (int64_t i = 0; i < n; ++i) inc_ptr[i + 1] += inc_ptr[i];
  std::vector<int32_t> inc(inc_ptr[n]);
  {
    std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int64_t t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k) inc[fill[tsorted[3 * t + k]]++] = int32_t(3 * t + k);
  }
  std::vector<double> xnew(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) xnew[3 * i + k] = xyz[3 * M->perm[i] + k];

  SP_HIP(hipGetDevice(&M->device));
  hipStream_t s;
  SP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  try {
    M->cols.alloc(size_t(W) * n);
    M->M64.alloc(size_t(W) * n);
    M->A64.alloc(size_t(W) * n);
    M->tri.alloc(3 * nt);
    M->tarea.alloc(nt);
    M->perm_d.alloc(n);
    M->iperm_d.alloc(n);
    DevBuf<double> xd(3 * n);
    DevBuf<int32_t> incp(n + 1), incd(inc.size());
    SP_HIP(hipMemcpyAsync(M->cols.p, M->h_cols.data(), M->cols.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(M->tri.p, tsorted.data(), M->tri.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(M->perm_d.p, M->perm.data(), M->perm_d.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(M->iperm_d.p, M->iperm.data(), M->iperm_d.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(xd.p, xnew.data(), xd.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(incp.p, inc_ptr.data(), incp.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(incd.p, inc.data(), incd.bytes(), hipMemcpyHostToDevice, s));
    k::assemble(*M, xd.p, incp.p, incd.p, s);
    SP_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    throw;
  }
  SP_HIP(hipStreamDestroy(s));
  return M.release();
}

// K = M + tau A and its Jacobi diagonal, built once per (mesh, tau) on a
// private stream and cached; callers on any stream may use the result.  The
// polynomial preconditioner's matrix is added the first time a caller asks.
TauMats* Mesh::tau_mats(double tau, bool with_precond) {
  double c0 = 0, c1 = 0;
  if (with_precond) cheb_coefs(tau, &c0, &c1);  // host work, outside mu
  std::lock_guard<std::mutex> g(mu);
  TauMats* t = nullptr;
  for (auto& e : kcache)
    if (e->tau == tau) t = e.get();
  if (t && (!with_precond || t->P64.p)) return t;
  std::unique_ptr<TauMats> fresh;
  if (!t) {
    fresh.reset(new TauMats());
    t = fresh.get();
    t->tau = tau;
    t->K64.alloc(size_t(W) * n);
    t->K32.alloc(size_t(W) * n);
    t->dinv64.alloc(n);
    t->dinv32.alloc(n);
  }
  if (with_precond) {
    t->pc0 = c0;
    t->pc1 = c1;
    t->P64.alloc(size_t(W) * n);
    t->P32.alloc(size_t(W) * n);
  }
  hipStream_t s;
  SP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (fresh) k::tau_mats(*this, *t, s);
  if (with_precond) k::precond_mats(*this, *t, s);
  hipError_t e = hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  SP_HIP(e);
  if (fresh) kcache.push_back(std::move(fresh));
  return t;
}

}  // namespace sp
