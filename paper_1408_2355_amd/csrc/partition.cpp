// Post-processing of a computed partition: the first Dirichlet eigenvalue of
// every region (the partition problem's energy, Problem 1.1, is their sum)
// by inverse iteration on the region-restricted float64 heat solve, and the
// adjacency of the regions (their numbers of sides, for the identity the
// paper derives from Euler's formula).
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <vector>

#include "engine.h"
#include "partition.h"

namespace sp {

void Solver::set_region_mask(const int32_t* labels, bool interior) {
  SP_REQUIRE(labels != nullptr, SP_EINVAL, "NULL labels");
  SP_REQUIRE(prm_.precision == SP_FP64, SP_EINVAL, "region restriction needs SP_FP64");
  flush_scale();
  const int64_t n = mesh_->n;
  const int nres = int(spec_.m.size());
  std::vector<uint8_t> mk(size_t(n) * rp_, 0);
  std::vector<int64_t> count(rp_, 0);
  const int W = mesh_->W;
  const std::vector<int32_t>& cols = mesh_->h_cols;  // [W][n], new numbering
  std::vector<int32_t> lnew(n);
  for (int r = 0; r < nres; ++r) {
    const int lo = h_res_lo_[r], m = h_res_len_[r];
    const int32_t* lr = labels + size_t(r) * n;
    for (int64_t v = 0; v < n; ++v) lnew[v] = lr[mesh_->perm[v]];
    for (int64_t v = 0; v < n; ++v) {
      const int32_t l = lnew[v];
      bool in = l >= 0 && l < m;
      if (in && interior)  // padding slots repeat the row, which has label l
        for (int k = 1; k < W && in; ++k) in = lnew[cols[size_t(k) * n + v]] == l;
      if (in) {
        mk[size_t(v) * rp_ + lo + l] = 1;
        ++count[lo + l];
      }
    }
  }
  mask_.alloc(mk.size());
  SP_HIP(hipMemcpyAsync(mask_.p, mk.data(), mk.size(), hipMemcpyHostToDevice, s_));
  args_.mask = mask_.p;
  small_ = false;  // the one-workgroup path has no restriction
  forget_history(0, rp_);
  aw_fresh_ = false;
  lam_fresh_ = false;
  k::apply_mask(args_, u_.p, s_);
  for (int c = 0; c < rp_; ++c)
    if (h_live_[c] && count[c] == 0) h_live_[c] = 0;
  push_tables();
  SP_HIP(hipStreamSynchronize(s_));  // mk is freed on return
}

int Solver::region_eigen(double tol, int max_iter, double* lam) {
  SP_REQUIRE(args_.mask != nullptr, SP_EINVAL, "region_eigen: no region mask");
  SP_REQUIRE(std::isfinite(tol) && tol > 0 && max_iter >= 1, SP_EINVAL,
             "region_eigen: need tol > 0 and max_iter >= 1");
  std::vector<double> prev(rp_), cur(rp_);
  auto quotients = [&](std::vector<double>& out) {
    norm_dot_scale(u_.p, false);  // normalise; lam_ = Rayleigh quotients
    SP_HIP(hipMemcpyAsync(out.data(), lam_.p, rp_ * sizeof(double), hipMemcpyDeviceToHost, s_));
    SP_HIP(hipStreamSynchronize(s_));
  };
  quotients(prev);
  int it = 0;
  bool done = false;
  while (!done && it < max_iter) {
    heat_fp64();
    quotients(cur);
    ++it;
    done = true;
    for (int c = 0; c < R_; ++c)
      if (h_live_[c] && !(std::fabs(cur[c] - prev[c]) <= tol * std::fabs(cur[c]))) done = false;
    prev.swap(cur);
  }
  for (int c = 0; c < R_; ++c)
    lam[c] = h_live_[c] ? prev[c] : std::numeric_limits<double>::quiet_NaN();
  return done ? it : -it;
}

void region_graph(const Mesh& mesh, int nres, const int* m, const int32_t* labels, uint8_t* adj,
                  int32_t* sides) {
  SP_REQUIRE(nres >= 1 && m && labels && adj, SP_EINVAL, "region_graph: NULL argument");
  const int64_t n = mesh.n;
  std::vector<int> off(nres + 1, 0);
  int64_t total = 0;
  for (int r = 0; r < nres; ++r) {
    SP_REQUIRE(m[r] >= 1 && m[r] <= 4096, SP_EINVAL, "region_graph: m must be in 1..4096");
    total += int64_t(m[r]) * m[r];
    SP_REQUIRE(total < (int64_t(1) << 31), SP_EINVAL,
               "region_graph: adjacency too large (sum of m^2 must stay below 2^31)");
    off[r + 1] = int(total);
  }
  // labels in the renumbered vertex order
  std::vector<int32_t> lab(size_t(n) * nres);
  for (int r = 0; r < nres; ++r)
    for (int64_t v = 0; v < n; ++v) lab[size_t(r) * n + v] = labels[size_t(r) * n + mesh.perm[v]];
  hipStream_t s;
  SP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  try {
    DevBuf<int32_t> dl(lab.size());
    DevBuf<int> doff(nres), dm(nres);
    DevBuf<uint8_t> dadj(off[nres]);
    SP_HIP(hipMemcpyAsync(dl.p, lab.data(), dl.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(doff.p, off.data(), doff.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemcpyAsync(dm.p, m, dm.bytes(), hipMemcpyHostToDevice, s));
    SP_HIP(hipMemsetAsync(dadj.p, 0, dadj.bytes(), s));
    StepArgs a;
    a.t.n = int(n);
    a.W = mesh.W;
    a.cols = mesh.cols.p;
    k::region_graph(a, dl.p, doff.p, dm.p, nres, dadj.p, s);
    SP_HIP(hipMemcpyAsync(adj, dadj.p, dadj.bytes(), hipMemcpyDeviceToHost, s));
    SP_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    throw;
  }
  SP_HIP(hipStreamDestroy(s));
  if (sides) {
    int c = 0;
    for (int r = 0; r < nres; ++r)
      for (int i = 0; i < m[r]; ++i, ++c) {
        int k = 0;
        for (int j = 0; j < m[r]; ++j) k += adj[off[r] + i * m[r] + j];
        sides[c] = k;
      }
  }
}

}  // namespace sp
