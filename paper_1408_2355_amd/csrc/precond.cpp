// Coefficients of the CG's degree-1 polynomial preconditioner (host side).
//
// Each heat step of Algorithm 2.2 solves (M + tau A) u~ = M u.  The CG is
// preconditioned by z = p(D^-1 K) D^-1 r with K = M + tau A, D its diagonal
// and p(lambda) = c0 + c1 lambda the degree-1 polynomial whose residual
// 1 - lambda p(lambda) is the scaled Chebyshev polynomial
// T_2((a + b - 2 lambda) / (b - a)) / T_2((a + b) / (b - a)): the smallest
// maximum of |1 - lambda p(lambda)| over [a, b] (Chebyshev's minimax
// property).  With theta = (a + b) / 2, delta = (b - a) / 2,
//   c0 = 4 theta / (2 theta^2 - delta^2),  c1 = -2 / (2 theta^2 - delta^2).
// p(lambda) > 0 for lambda < a + b = 2 theta, so the preconditioner
// D^-1/2 p(S) D^-1/2 (S = D^-1/2 K D^-1/2) is symmetric positive definite
// whenever the spectrum of S lies below a + b; the CG's stopping test is on
// the unpreconditioned residual, so [a, b] only changes the iteration count.
//
// [a, b]: the extreme Ritz values of a Lanczos run on S from a fixed
// pseudo-random start.  Ritz values lie inside the spectrum, so b is raised
// to max(1.02 b, g - a / 2), g the Gershgorin bound of D^-1 K (a rigorous
// upper bound on the spectrum): then a + b > g >= lambda_max always.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "internal.h"

namespace sp {

namespace {

constexpr int kLanczosSteps = 40;

// Eigenvalue of the symmetric tridiagonal (al[0..m), be[1..m)) with index
// `which` in increasing order, by bisection on the Sturm count.
double tri_eig(const std::vector<double>& al, const std::vector<double>& be, int which) {
  const int m = int(al.size());
  double lo = al[0], hi = al[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(be[i]) : 0.0) + (i + 1 < m ? std::fabs(be[i + 1]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  auto below = [&](double x) {  // eigenvalues < x (signs of the LDL^T pivots)
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      d = al[i] - x - (i > 0 ? be[i] * be[i] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-14 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) > which)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

void Mesh::cheb_coefs(double tau, double* c0, double* c1) {
  std::lock_guard<std::mutex> g(pmu);
  for (const auto& e : pcache)
    if (e[0] == tau) {
      *c0 = e[1];
      *c1 = e[2];
      return;
    }
  const size_t wn = size_t(W) * size_t(n);
  std::vector<double> Mh(wn), Ah(wn);
  SP_HIP(hipMemcpy(Mh.data(), M64.p, wn * 8, hipMemcpyDeviceToHost));
  SP_HIP(hipMemcpy(Ah.data(), A64.p, wn * 8, hipMemcpyDeviceToHost));
  std::vector<double> K(wn), s(n);
  for (size_t i = 0; i < wn; ++i) K[i] = Mh[i] + tau * Ah[i];
  double gersh = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    SP_REQUIRE(K[i] > 0.0, SP_EMESH, "mesh: M + tau A has a non-positive diagonal entry");
    s[i] = 1.0 / std::sqrt(K[i]);
    double row = 0.0;
    for (int k = 0; k < W; ++k) row += std::fabs(K[size_t(k) * n + i]);
    gersh = std::max(gersh, row / K[i]);
  }
  auto apply = [&](const std::vector<double>& v, std::vector<double>& w) {  // w = S v
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int k = 0; k < W; ++k) {
        const int32_t c = h_cols[size_t(k) * n + i];
        acc += K[size_t(k) * n + i] * s[c] * v[c];
      }
      w[i] = s[i] * acc;
    }
  };
  // fixed pseudo-random start (a 64-bit LCG), normalised
  std::vector<double> v(n), vp(n, 0.0), w(n);
  uint64_t x = 0x2545F4914F6CDD1DULL;
  double nn = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    x = x * 6364136223846793005ULL + 1442695040888963407ULL;
    v[i] = double(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    nn += v[i] * v[i];
  }
  for (auto& e : v) e /= std::sqrt(nn);
  std::vector<double> al, be(1, 0.0);
  const int steps = int(std::min<int64_t>(kLanczosSteps, n));
  for (int j = 0; j < steps; ++j) {
    apply(v, w);
    double a = 0.0;
    for (int64_t i = 0; i < n; ++i) a += w[i] * v[i];
    al.push_back(a);
    double b2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      w[i] -= a * v[i] + be.back() * vp[i];
      b2 += w[i] * w[i];
    }
    const double b = std::sqrt(b2);
    if (j + 1 == steps || !(b > 1e-12 * std::fabs(a))) break;
    be.push_back(b);
    for (int64_t i = 0; i < n; ++i) {
      vp[i] = v[i];
      v[i] = w[i] / b;
    }
  }
  be.resize(al.size());
  double lo = tri_eig(al, be, 0);
  double hi = tri_eig(al, be, int(al.size()) - 1);
  lo = std::max(lo, 1e-6 * hi);
  hi = std::max(1.02 * hi, gersh - 0.5 * lo);
  const double th = 0.5 * (hi + lo), de = 0.5 * (hi - lo);
  const double den = 2.0 * th * th - de * de;
  *c0 = 4.0 * th / den;
  *c1 = -2.0 / den;
  if (std::getenv("SEGPART_DEBUG_PRECOND"))
    std::fprintf(stderr, "precond: tau %g Ritz [%g, %g] Gershgorin %g -> [%g, %g] c0 %g c1 %g\n",
                 tau, tri_eig(al, be, 0), tri_eig(al, be, int(al.size()) - 1), gersh, lo, hi,
                 *c0, *c1);
  pcache.push_back({tau, *c0, *c1});
}

}  // namespace sp
