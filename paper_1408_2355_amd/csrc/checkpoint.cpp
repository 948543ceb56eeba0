// Checkpoint and restore of a batch's full device state (see engine.h).
//
// A time step reads more than the state u: the mixed-precision step starts
// each heat solve from an extrapolation of the columns' previous heat
// increments (kept per column), from A v of the last normalisation pass, and
// it may hold the last normalisation factor unapplied (deferred scaling).
// Continuing a run exactly needs all of it, and the tilings whose fixed
// reduction orders the arithmetic followed.  The checkpoint is a byte image in
// the solver's internal layout (renumbered vertices, padded columns): it is
// restored only into a solver of the same mesh size, column layout,
// precision, extrapolation depth, tau and restarts (m, eps), which the header
// records and the restore checks.
#include <cstring>

#include "engine.h"

namespace sp {

namespace {

constexpr char kMagic[8] = {'S', 'P', 'C', 'K', 'P', 'T', '0', '2'};

struct Header {
  char magic[8];
  int64_t n, rp, R, nres, nres_p;
  int32_t precision, q, n_prev, flags;  // flags: 1 u_pending, 2 aw_fresh, 4 lam_fresh, 8 small
  int32_t last_sweeps, reserved;
  int64_t steps_done;
  double tau;
  Tile tm, t64, tp;
  int32_t seps_direct, seps_nper;
  int64_t hist_pairs;  // energy-history pairs over all restarts
  int64_t total;       // bytes of the whole image
};

// Cursor over the image (writing or reading).
struct Cursor {
  char* p;
  size_t left;
  void take(size_t k) {
    SP_REQUIRE(k <= left, SP_EINVAL, "checkpoint: buffer too small");
    p += k;
    left -= k;
  }
};

}  // namespace

int64_t Solver::checkpoint_size() {
  const size_t nv = size_t(mesh_->n) * rp_;
  int64_t pairs = 0;
  for (const auto& h : hist_) pairs += int64_t(h.size());
  int64_t b = sizeof(Header);
  b += int64_t(nres()) * (sizeof(int32_t) + sizeof(double));  // m, eps
  b += int64_t(nv) * 8;                                       // u
  b += int64_t(colf_.n) * 8 + int64_t(coli_.n) * 4;           // column scalars and tables
  b += int64_t(lam_.n) * 8 + int64_t(stat_.n) * 8;
  const int q = prm_.precision != SP_FP64 ? prm_.extrapolate : 0;
  b += int64_t(q) * int64_t(nv) * 4;  // increments, newest first
  if (q) b += int64_t(nv) * 8;        // A v of the last norm pass
  b += int64_t(nres()) * 8 + pairs * 16;  // history: count per restart, (step, E) pairs
  return b;
}

void Solver::checkpoint(void* buf, int64_t bytes) {
  SP_REQUIRE(buf != nullptr, SP_EINVAL, "checkpoint: NULL buffer");
  SP_REQUIRE(args_.mask == nullptr, SP_EINVAL, "checkpoint: state is restricted to regions");
  const int64_t need = checkpoint_size();
  SP_REQUIRE(bytes >= need, SP_EINVAL, "checkpoint: buffer too small");
  const size_t nv = size_t(mesh_->n) * rp_;
  const int q = prm_.precision != SP_FP64 ? prm_.extrapolate : 0;
  Header h{};
  std::memcpy(h.magic, kMagic, 8);
  h.n = mesh_->n;
  h.rp = rp_;
  h.R = R_;
  h.nres = nres();
  h.nres_p = nres_p_;
  h.precision = prm_.precision;
  h.q = q;
  h.n_prev = n_prev_;
  h.flags = (u_pending_ ? 1 : 0) | (aw_fresh_ ? 2 : 0) | (lam_fresh_ ? 4 : 0) | (small_ ? 8 : 0);
  h.last_sweeps = last_sweeps_;
  h.steps_done = steps_done_;
  h.tau = prm_.tau;
  h.tm = args_.tm;
  h.t64 = args_.t64;
  h.tp = args_.tp;
  h.seps_direct = sp_.direct;
  h.seps_nper = sp_.nper;
  int64_t pairs = 0;
  for (const auto& e : hist_) pairs += int64_t(e.size());
  h.hist_pairs = pairs;
  h.total = need;
  Cursor c{static_cast<char*>(buf), size_t(bytes)};
  auto put = [&](const void* src, size_t k) {
    char* at = c.p;
    c.take(k);
    std::memcpy(at, src, k);
  };
  auto put_dev = [&](const void* dsrc, size_t k) {
    char* at = c.p;
    c.take(k);
    SP_HIP(hipMemcpyAsync(at, dsrc, k, hipMemcpyDeviceToHost, s_));
  };
  put(&h, sizeof(h));
  put(spec_.m.data(), spec_.m.size() * sizeof(int));
  put(spec_.eps.data(), spec_.eps.size() * sizeof(double));
  put_dev(u_.p, nv * 8);
  put_dev(colf_.p, colf_.n * 8);
  put_dev(coli_.p, coli_.n * 4);
  put_dev(lam_.p, lam_.n * 8);
  put_dev(stat_.p, stat_.n * 8);
  for (int i = 0; i < q; ++i) put_dev(dh_[i], nv * 4);
  if (q) put_dev(xg_.p, nv * 8);
  for (const auto& e : hist_) {
    const int64_t k = int64_t(e.size());
    put(&k, 8);
  }
  for (const auto& e : hist_)
    for (const auto& pr : e) {
      put(&pr.first, 8);
      put(&pr.second, 8);
    }
  SP_HIP(hipStreamSynchronize(s_));  // the copies land in the caller's buffer
}

void Solver::restore(const void* buf, int64_t bytes) {
  SP_REQUIRE(buf != nullptr, SP_EINVAL, "restore: NULL buffer");
  SP_REQUIRE(args_.mask == nullptr, SP_EINVAL, "restore: state is restricted to regions");
  SP_REQUIRE(bytes >= int64_t(sizeof(Header)), SP_EINVAL, "restore: buffer too small");
  Header h;
  std::memcpy(&h, buf, sizeof(h));
  const int q = prm_.precision != SP_FP64 ? prm_.extrapolate : 0;
  SP_REQUIRE(std::memcmp(h.magic, kMagic, 8) == 0, SP_EINVAL, "restore: not a checkpoint image");
  SP_REQUIRE(h.total <= bytes, SP_EINVAL, "restore: image truncated");
  SP_REQUIRE(h.n == mesh_->n && h.rp == rp_ && h.R == R_ && h.nres == nres() &&
                 h.nres_p == nres_p_ && h.precision == prm_.precision && h.q == q &&
                 h.tau == prm_.tau,
             SP_EINVAL, "restore: the checkpoint belongs to a different batch or parameters");
  const size_t nv = size_t(mesh_->n) * rp_;
  Cursor c{const_cast<char*>(static_cast<const char*>(buf)) + sizeof(Header),
           size_t(h.total) - sizeof(Header)};
  auto get = [&](void* dst, size_t k) {
    const char* at = c.p;
    c.take(k);
    std::memcpy(dst, at, k);
  };
  std::vector<int> m(nres());
  std::vector<double> eps(nres());
  get(m.data(), m.size() * sizeof(int));
  get(eps.data(), eps.size() * sizeof(double));
  SP_REQUIRE(m == spec_.m && eps == spec_.eps, SP_EINVAL,
             "restore: the checkpoint's restarts (m, eps) differ from this batch's");
  // nothing of the current state survives: pending factors, graphs and the
  // live masks are replaced by the image's
  auto get_dev = [&](void* ddst, size_t k) {
    const char* at = c.p;
    c.take(k);
    SP_HIP(hipMemcpyAsync(ddst, at, k, hipMemcpyHostToDevice, s_));
  };
  get_dev(u_.p, nv * 8);
  get_dev(colf_.p, colf_.n * 8);
  get_dev(coli_.p, coli_.n * 4);
  get_dev(lam_.p, lam_.n * 8);
  get_dev(stat_.p, stat_.n * 8);
  for (int i = 0; i < q; ++i) get_dev(dh_[i], nv * 4);
  if (q) get_dev(xg_.p, nv * 8);
  std::vector<int64_t> cnt(nres());
  for (auto& k : cnt) get(&k, 8);
  for (int r = 0; r < nres(); ++r) {
    hist_[r].clear();
    for (int64_t i = 0; i < cnt[r]; ++i) {
      std::pair<int64_t, double> pr;
      get(&pr.first, 8);
      get(&pr.second, 8);
      hist_[r].push_back(pr);
    }
  }
  // the host mirrors of the column tables that the image carries
  std::vector<int> ci(coli_.n);
  SP_HIP(hipMemcpyAsync(ci.data(), coli_.p, coli_.n * 4, hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
  const int* live = ci.data() + (args_.ct.live - coli_.p);
  const int* hlen = ci.data() + (args_.hlen - coli_.p);
  for (int col = 0; col < rp_; ++col) {
    h_live_[col] = live[col];
    h_hlen_[col] = hlen[col];
  }
  const int* rlive = ci.data() + (args_.ct.res_live - coli_.p);
  for (int r = 0; r < nres_p_; ++r) h_res_live_[r] = rlive[r];
  all_live_ = true;
  live_cols_ = 0;
  for (int col = 0; col < rp_; ++col) {
    if (h_seg_len_[col] > 0 && !h_live_[col]) all_live_ = false;
    live_cols_ += (h_seg_len_[col] > 0 && h_live_[col]) ? 1 : 0;
  }
  n_prev_ = h.n_prev;
  u_pending_ = (h.flags & 1) != 0;
  aw_fresh_ = (h.flags & 2) != 0;
  lam_fresh_ = (h.flags & 4) != 0;
  last_sweeps_ = h.last_sweeps;
  steps_done_ = h.steps_done;
  heat_x_ = u_.p;
  // the fixed reduction orders of the run that wrote the image
  args_.tm = h.tm;
  args_.t64 = h.t64;
  args_.tp = h.tp;
  sp_.direct = h.seps_direct;
  sp_.nper = h.seps_nper;
}

}  // namespace sp
