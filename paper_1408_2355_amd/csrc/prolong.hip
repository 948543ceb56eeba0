// Prolongation of a state to a refined mesh (the continuation of Section 3.1):
// the coarse P1 function evaluated at the fine vertices.  Coarse vertices keep
// their value; a new vertex, the midpoint of a coarse edge (a, b), takes
// (u_a + u_b) / 2.  Caller layout [cols][n] on both sides, float64, one
// thread per fine value; bound by HBM (read 8 B per coarse value plus two
// neighbouring reads per new vertex, write 8 B per fine value).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace sp {
namespace {

constexpr int kProlongBlock = 256;

__global__ __launch_bounds__(kProlongBlock) void k_prolong(int64_t nc, int64_t nf, int64_t total,
                                                           const int32_t* __restrict__ parents,
                                                           const double* __restrict__ uc,
                                                           double* __restrict__ uf) {
  for (int64_t i = blockIdx.x * int64_t(kProlongBlock) + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * kProlongBlock) {
    const int64_t c = i / nf, v = i - c * nf;
    const double* col = uc + c * nc;
    double x;
    if (v < nc) {
      x = col[v];
    } else {
      const int64_t j = v - nc;
      x = 0.5 * (col[parents[2 * j]] + col[parents[2 * j + 1]]);
    }
    uf[i] = x;
  }
}

}  // namespace

namespace k {
void prolong(const Mesh& fine, int cols, const double* u_coarse, double* u_fine, hipStream_t s) {
  SP_REQUIRE(fine.n_coarse > 0 && fine.parents_d.p, SP_EINVAL, "prolong: mesh was not refined");
  const int64_t total = int64_t(cols) * fine.n;
  if (total == 0) return;
  const int64_t blocks = std::min<int64_t>((total + kProlongBlock - 1) / kProlongBlock, 65536);
  hipLaunchKernelGGL(k_prolong, dim3(unsigned(blocks)), dim3(kProlongBlock), 0, s, fine.n_coarse,
                     fine.n, total, fine.parents_d.p, u_coarse, u_fine);
  SP_HIP(hipGetLastError());
}
}  // namespace k

}  // namespace sp
