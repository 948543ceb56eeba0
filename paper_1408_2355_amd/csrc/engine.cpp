// Orchestration of the time step of Algorithm 2.2 for a batch of restarts.
//
// Step 1 (heat): per column, Jacobi-preconditioned CG on (M + tau A) x = M u
// started from x0 = u (so r0 = -tau A u).  SP_FP64 runs the CG in float64;
// SP_MIXED runs float32 CG inner solves inside float64 iterative refinement.
// Each column keeps its own CG scalars and stops on its own test
// ||r||_2 <= cg_rtol ||M u||_2, so a column's arithmetic does not depend on
// which other columns share the launch.  The host launches iterations in
// chunks of check_every and polls one device counter between chunks; the
// kernels of an iteration after global convergence exit at once.
// Step 2 (node step) and step 3 (L2 normalisation) follow; energies at the
// cadence energy_every (Section 2.2 checks the energy every M_tau steps).
#include "engine.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>

namespace sp {

namespace {
enum { CF_BB, CF_RZ, CF_TOL2, CF_ALPHA, CF_BETA, CF_RRO, CF_NRM, CF_BBN, CF_ISC, CF_COEF, CF_N };
enum { CI_ACT, CI_ACTO, CI_ITERS, CI_SWEEPS, CI_SEGLO, CI_SEGLEN, CI_LIVE, CI_HLEN, CI_ORD, CI_N };
constexpr int kSepsNperMax = 512;  // S_eps element-kernel workgroups per XCD, at most
}  // namespace

void validate_params(const sp_params& p) {
  SP_REQUIRE(std::isfinite(p.tau) && p.tau > 0, SP_EINVAL, "params: tau must be > 0");
  SP_REQUIRE(p.precision == SP_FP64 || p.precision == SP_MIXED, SP_EINVAL,
             "params: precision must be SP_FP64 or SP_MIXED");
  SP_REQUIRE(p.n_steps >= 0, SP_EINVAL, "params: n_steps must be >= 0");
  SP_REQUIRE(p.energy_every >= 0, SP_EINVAL, "params: energy_every must be >= 0");
  SP_REQUIRE(p.n_steps > 0 || p.energy_every > 0, SP_EINVAL,
             "params: stop mode (n_steps == 0) needs energy_every > 0");
  SP_REQUIRE(p.n_steps > 0 || (std::isfinite(p.stop_tol) && p.stop_tol > 0), SP_EINVAL,
             "params: stop_tol must be > 0");
  SP_REQUIRE(p.n_steps > 0 || p.max_steps > 0, SP_EINVAL, "params: max_steps must be > 0");
  SP_REQUIRE(std::isfinite(p.cg_rtol) && p.cg_rtol > 0 && p.cg_rtol < 1, SP_EINVAL,
             "params: cg_rtol must be in (0, 1)");
  SP_REQUIRE(p.cg_max_iter >= 1, SP_EINVAL, "params: cg_max_iter must be >= 1");
  SP_REQUIRE(p.check_every >= 0, SP_EINVAL, "params: check_every must be >= 0");
  SP_REQUIRE(p.extrapolate >= 0 && p.extrapolate <= kMaxExtrap, SP_EINVAL,
             "params: extrapolate must be in 0..8");
  SP_REQUIRE(p.precond == SP_PRECOND_JACOBI || p.precond == SP_PRECOND_CHEB1, SP_EINVAL,
             "params: precond must be SP_PRECOND_JACOBI or SP_PRECOND_CHEB1");
  if (p.precision == SP_MIXED) {
    SP_REQUIRE(std::isfinite(p.inner_rtol) && p.inner_rtol > 0 && p.inner_rtol < 1, SP_EINVAL,
               "params: inner_rtol must be in (0, 1)");
    SP_REQUIRE(p.max_outer >= 1, SP_EINVAL, "params: max_outer must be >= 1");
  }
}

void validate_batch(int32_t nres, const int32_t* m, const double* eps) {
  SP_REQUIRE(nres >= 1, SP_EINVAL, "batch: n_restarts must be >= 1");
  SP_REQUIRE(m && eps, SP_EINVAL, "batch: NULL m or eps");
  int64_t R = 0;
  for (int32_t r = 0; r < nres; ++r) {
    SP_REQUIRE(m[r] >= 1, SP_EINVAL, "batch: m must be >= 1 (restart " + std::to_string(r) + ")");
    SP_REQUIRE(std::isfinite(eps[r]) && eps[r] > 0, SP_EINVAL,
               "batch: eps must be > 0 (restart " + std::to_string(r) + ")");
    R += m[r];
  }
  SP_REQUIRE(R <= (1 << 24), SP_EINVAL, "batch: too many components");
}

Solver::Solver(Mesh* mesh, const sp_params& prm, const BatchSpec& spec, const hipStream_t* stream,
               int min_columns, int min_restarts, Arena* arena)
    : mesh_(mesh), arena_(arena), prm_(prm), spec_(spec) {
  validate_params(prm_);
  SP_REQUIRE(mesh_ != nullptr, SP_EINVAL, "NULL mesh");
  const int nres = int(spec_.m.size());
  SP_REQUIRE(nres >= 1 || min_columns > 0, SP_EINVAL, "batch: no restarts");
  for (int x : spec_.m) R_ += x;
  rp_ = ((std::max(std::max(R_, min_columns), 1) + 3) / 4) * 4;
  nres_p_ = std::max(std::max(nres, min_restarts), 1);
  if (stream) {
    s_ = *stream;
  } else {
    SP_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    own_stream_ = true;
  }
  try {
    const int n = int(mesh_->n);
    const size_t nv = size_t(n) * rp_;
    // small batches run whole steps in one workgroup (float64 CG) unless
    // SEGPART_SMALL=0
    const char* sm_env = std::getenv("SEGPART_SMALL");
    small_ = nv <= size_t(kSmallMaxValues) && rp_ <= kSmallMaxCols &&
             nres_p_ <= kSmallMaxRestarts && !(sm_env && std::strcmp(sm_env, "0") == 0);
    const bool poly = prm_.precond == SP_PRECOND_CHEB1 && !small_;
    if (arena_) {
      // this tau's K, K32, Jacobi diagonals (and preconditioner), built
      // below on the stream
      const size_t wn = size_t(mesh_->W) * size_t(mesh_->n);
      own_km_.tau = prm_.tau;
      get(own_km_.K64, wn);
      get(own_km_.K32, wn);
      get(own_km_.dinv64, size_t(mesh_->n));
      get(own_km_.dinv32, size_t(mesh_->n));
      if (poly) {
        mesh_->cheb_coefs(prm_.tau, &own_km_.pc0, &own_km_.pc1);
        get(own_km_.P64, wn);
        get(own_km_.P32, wn);
      }
      km_ = &own_km_;
    } else {
      km_ = mesh_->tau_mats(prm_.tau, poly);
    }
    Tile t = make_tile(n, rp_, 64, 1, 128);
    sp_.nt = int(mesh_->nt);
    sp_.tchunk = 64;
    sp_.nchunk = int((mesh_->nt + sp_.tchunk - 1) / sp_.tchunk);
    // S_eps workgroups per XCD: as many as 512 (the element kernels are
    // latency-bound and want every SIMD full); the tuner may pick 64
    sp_.nper = std::max(1, std::min(kSepsNperMax, (sp_.nchunk + 7) / 8));
    sp_.nres_p = nres_p_;
    get(seps_tiles_, nres_p_);
    get(u_, nv);
    heat_x_ = u_.p;
    get(r64_, nv);
    const char* gr_env = std::getenv("SEGPART_GRAPH");
    graph_on_ = !(gr_env && std::strcmp(gr_env, "0") == 0) && !arena_;  // instantiation allocates
    if (prm_.precision == SP_FP64 || small_) {
      get(p64_, nv);
      get(q64_, nv);
      if (poly) get(z64_, nv);
    }
    if (small_) get(small_hist_, size_t(kSmallChunk) * nres_p_);
    if (prm_.precision != SP_FP64) {
      get(d32_, nv);
      get(r32_, nv);
      get(p16_, nv);
      get(q32_, nv);
      if (poly) get(z16_, nv);
      // direction ring of the inner CG: p16_ is slot 0
      pring_[0] = p16_.p;
      for (int i = 1; i < kPRing; ++i) {
        get(pbuf_[i], nv);
        pring_[i] = pbuf_[i].p;
      }
      get(ah_, size_t(kPRing) * rp_);
      for (int i = 0; i < prm_.extrapolate; ++i) {
        get(dbuf_[i], nv);
        dh_[i] = dbuf_[i].p;
      }
      if (prm_.extrapolate) {
        get(xg_, nv);
        get(d0buf_, nv);
      }
    }
    // partial sums: one row per workgroup, sized for the widest tiling the
    // autotuner may pick
    int max_blk = t.nblk;
    for (const Tile& c : tile_candidates()) max_blk = std::max(max_blk, c.nblk);
    // three partial-sum slots per column, five for the extrapolation's order
    // control (float32 CG with two or more kept increments)
    const int part_slots =
        prm_.precision != SP_FP64 && prm_.extrapolate >= 2 ? std::max(3, k::kOrderProbes) : 3;
    get(part_, size_t(part_slots) * size_t(max_blk) * rp_);
    if (poly) get(part2_, size_t(max_blk) * rp_);
    get(part_s_, size_t(8 * sp_.nper) * nres_p_);
    get(colf_, size_t(CF_N) * rp_ + nres_p_);
    get(coli_, size_t(CI_N) * rp_ + 3 * size_t(nres_p_));
    get(ring_, 2 * kRing);
    get(stat_, kStats);
    get(lam_, rp_);
    get(seps_, nres_p_);
    get(energy_, nres_p_);
    if (arena_)
      h_poll_ = poll_host_;
    else
      SP_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_poll_), 64, hipHostMallocDefault));

    if (arena_) {
      // the region keeps the last user's contents: start from zeros, as a
      // fresh allocation does
      k::fill_i32(reinterpret_cast<int32_t*>(arena_->base), 0, arena_->used / 4, s_);
      k::tau_mats(*mesh_, own_km_, s_);
      if (poly) k::precond_mats(*mesh_, own_km_, s_);
    }
    k::fill_f64(u_.p, 0.0, nv, s_);
    k::fill_f64(r64_.p, 0.0, nv, s_);
    if (z64_.p) k::fill_f64(z64_.p, 0.0, nv, s_);
    if (z16_.p) k::fill_i32(reinterpret_cast<int32_t*>(z16_.p), 0, nv / 2, s_);
    for (int i = 0; i < kMaxExtrap; ++i)
      if (dh_[i]) k::fill_f32(dh_[i], 0.0f, nv, s_);
    for (int i = 0; i < kPRing; ++i)
      if (pring_[i]) k::fill_i32(reinterpret_cast<int32_t*>(pring_[i]), 0, nv / 2, s_);
    if (ah_.p) k::fill_f64(ah_.p, 0.0, ah_.n, s_);
    k::fill_f64(colf_.p, 0.0, colf_.n, s_);
    k::fill_i32(coli_.p, 0, coli_.n, s_);
    // every column starts at the full extrapolation order
    k::fill_i32(coli_.p + size_t(CI_ORD) * rp_, prm_.extrapolate, size_t(rp_), s_);
    k::fill_i32(ring_.p, 0, ring_.n, s_);
    k::fill_f64(reinterpret_cast<double*>(stat_.p), 0.0, stat_.n, s_);
    k::fill_f64(lam_.p, 0.0, lam_.n, s_);
    k::fill_f64(seps_.p, 0.0, seps_.n, s_);
    k::fill_f64(energy_.p, 0.0, energy_.n, s_);

    StepArgs& a = args_;
    a.t = t;   // streaming kernels: widest tiling (most workgroups in flight)
    a.ts = make_tile(n, rp_, 64, 1, 256);
    a.tm = t;   // gathering kernels: replaced by the autotuner's picks
    a.t64 = t;
    a.tp = t;
    // the extrapolation's order control samples about 8192 rows
    a.probe_stride = std::max(1, n / 8192);
    a.tprobe = make_tile((n + a.probe_stride - 1) / a.probe_stride, rp_, 64, 1, 64);
    a.W = mesh_->W;
    a.cols = mesh_->cols.p;
    a.M64 = mesh_->M64.p;
    a.A64 = mesh_->A64.p;
    a.K64 = km_->K64.p;
    a.dinv64 = km_->dinv64.p;
    a.K32 = km_->K32.p;
    a.dinv32 = km_->dinv32.p;
    a.tau = prm_.tau;
    a.rtol2 = prm_.cg_rtol * prm_.cg_rtol;
    a.inner_rtol2 = prm_.inner_rtol * prm_.inner_rtol;
    // an inner solve stops at 0.9 x the outer target: the float32 recursive
    // residual of the small corrections tracks the float64 one closely, so
    // the refinement check still passes after one sweep
    if (const char* e = std::getenv("SEGPART_INNER_FLOOR")) {
      const double f = std::atof(e);
      if (f > 0 && f < 1) a.inner_floor2 = f * f;
    }
    double* cf = colf_.p;
    int* ci = coli_.p;
    a.cg.bb = cf + CF_BB * rp_;
    a.cg.rz = cf + CF_RZ * rp_;
    a.cg.tol2 = cf + CF_TOL2 * rp_;
    a.cg.alpha = cf + CF_ALPHA * rp_;
    a.cg.beta = cf + CF_BETA * rp_;
    a.cg.rr_o = cf + CF_RRO * rp_;
    a.cg.nrm = cf + CF_NRM * rp_;
    a.cg.bb_next = cf + CF_BBN * rp_;
    a.cg.isc = cf + CF_ISC * rp_;
    a.ct.coef = cf + CF_COEF * rp_;
    a.ct.res_ieps2 = cf + CF_N * rp_;
    a.cg.act = ci + CI_ACT * rp_;
    a.cg.act_o = ci + CI_ACTO * rp_;
    a.cg.iters = ci + CI_ITERS * rp_;
    a.cg.sweeps = ci + CI_SWEEPS * rp_;
    a.ct.seg_lo = ci + CI_SEGLO * rp_;
    a.ct.seg_len = ci + CI_SEGLEN * rp_;
    a.ct.live = ci + CI_LIVE * rp_;
    a.hlen = ci + CI_HLEN * rp_;
    a.ord = ci + CI_ORD * rp_;
    a.ct.res_lo = ci + CI_N * rp_;
    a.ct.res_len = ci + CI_N * rp_ + nres_p_;
    a.ct.res_live = ci + CI_N * rp_ + 2 * nres_p_;
    a.ct.nres = nres;  // 0 for an empty server batch
    a.ct.nres_p = nres_p_;
    a.part = part_.p;
    if (poly) {
      a.poly = 1;
      a.part2 = part2_.p;
      a.P64 = km_->P64.p;
      a.P32 = km_->P32.p;
    }
    a.ring = ring_.p;
    a.oring = ring_.p + kRing;
    a.stat = stat_.p;

    // column tables: restart r owns columns [lo_r, lo_r + m_r)
    h_seg_lo_.assign(rp_, 0);
    h_hlen_.assign(rp_, 0);
    h_seg_len_.assign(rp_, 0);
    h_live_.assign(rp_, 0);
    h_coef_.assign(rp_, 0.0);
    h_res_lo_.assign(nres_p_, 0);
    h_res_len_.assign(nres_p_, 0);
    h_res_live_.assign(nres_p_, 0);
    h_res_ieps2_.assign(nres_p_, 0.0);
    int lo = 0;
    for (int r = 0; r < nres; ++r) {
      const int m = spec_.m[r];
      const double e = spec_.eps[r];
      for (int j = 0; j < m; ++j) {
        h_seg_lo_[lo + j] = lo;
        h_seg_len_[lo + j] = m;
        h_live_[lo + j] = 1;
        h_coef_[lo + j] = 2.0 * prm_.tau / (e * e);
      }
      h_res_lo_[r] = lo;
      h_res_len_[r] = m;
      h_res_live_[r] = 1;
      h_res_ieps2_[r] = 1.0 / (e * e);
      lo += m;
    }
    push_tables();
    hist_.assign(nres, {});
    autotune();
    // SEGPART_SEPS_KERNEL=staged|direct forces the S_eps element kernel
    // (otherwise the autotuner's pick; the staged one when it did not run)
    if (const char* e = std::getenv("SEGPART_SEPS_KERNEL")) {
      if (std::strcmp(e, "direct") == 0) sp_.direct = 1;
      if (std::strcmp(e, "staged") == 0) sp_.direct = 0;
      if (std::strcmp(e, "lanes") == 0) sp_.direct = 2;
    }
  } catch (...) {
    if (h_poll_ && !arena_) (void)hipHostFree(h_poll_);
    h_poll_ = nullptr;
    if (own_stream_) {
      (void)hipStreamSynchronize(s_);
      (void)hipStreamDestroy(s_);
    }
    throw;
  }
}

Solver::~Solver() {
  if (!detached_ || own_stream_) (void)hipStreamSynchronize(s_);
  for (auto& g : cg_graph_)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& e : ev_)
    for (auto x : e) (void)hipEventDestroy(x);
  if (h_poll_ && !arena_) (void)hipHostFree(h_poll_);
  if (own_stream_) (void)hipStreamDestroy(s_);
}

std::vector<Tile> Solver::tile_candidates() const {
  std::vector<Tile> out;
  const int n = int(mesh_->n);
  for (int tg : {8, 16, 32, 64})
    for (int passes : {1, 2, 4, 8})
      for (int nper : {64, 80, 96, 112, 128, 256}) {
        Tile c = make_tile(n, rp_, tg, passes, nper);
        bool dup = false;
        for (const Tile& o : out)
          dup |= o.tg == c.tg && o.ch == c.ch && o.nper == c.nper;
        if (!dup) out.push_back(c);
      }
  return out;
}

// Time `launch` under every candidate tiling placed in args_.*field and
// return the fastest (cached under key; see autotune.h).
TuneChoice Solver::tune_tiling(const std::string& key, Tile StepArgs::*field,
                               const std::function<void()>& launch) {
  TuneChoice best;
  if (tune_lookup(key, &best)) return best;
  hipEvent_t e0, e1;
  SP_HIP(hipEventCreate(&e0));
  SP_HIP(hipEventCreate(&e1));
  best.us = 1e30;
  const Tile keep = args_.*field;
  for (const Tile& c : tile_candidates()) {
    args_.*field = c;
    launch();
    SP_HIP(hipEventRecord(e0, s_));
    for (int i = 0; i < 3; ++i) launch();
    SP_HIP(hipEventRecord(e1, s_));
    SP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    SP_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double us = 1e3 * ms / 3.0;
    if (std::getenv("SEGPART_TUNE_VERBOSE"))
      std::fprintf(stderr, "[segpart tune] %s lanes=%d chunk=%d groups/xcd=%d: %.1f us\n",
                   key.c_str(), c.tg, c.ch, c.nper, us);
    if (us < best.us) {
      best.us = us;
      best.tg_cap = c.tg;
      best.passes = c.ch / c.tr;
      best.nper_cap = c.nper;
    }
  }
  args_.*field = keep;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  SP_HIP(hipStreamSynchronize(s_));
  tune_store(key, best);
  return best;
}

// Pick the tilings of the row-parallel gathering kernels by timing, once per
// (mesh size, ELL width, columns, precision, device): the CG matrix product
// sets the tiling of the product and the refinement update; in mixed
// precision the float64 gathers (solve set-up, norms) get their own, timed
// on the norm pass.
void Solver::autotune() {
  const size_t work = size_t(mesh_->n) * size_t(rp_);
  if (arena_ || !tune_enabled(work >= (size_t(1) << 22))) return;  // timing events, cache
  int dev = 0;
  SP_HIP(hipGetDevice(&dev));
  const bool f64 = prm_.precision == SP_FP64;
  const std::string key = "n" + std::to_string(mesh_->n) + "_W" + std::to_string(mesh_->W) +
                          "_rp" + std::to_string(rp_) + (f64 ? "_f64" : "_f32") + "_dev" +
                          std::to_string(dev);
  // matrix product: every column active, a nonzero iteration counter, p = 1
  k::fill_i32(args_.cg.act, 1, rp_, s_);
  k::fill_i32(ring_.p, 1, 1, s_);
  const size_t nv = size_t(mesh_->n) * rp_;
  if (f64)
    k::fill_f64(p64_.p, 1.0, nv, s_);
  else
    // bf16 ones, two per 32-bit word
    k::fill_i32(reinterpret_cast<int32_t*>(p16_.p), 0x3f803f80, nv / 2, s_);
  const TuneChoice best = tune_tiling(key, &StepArgs::tm, [&] {
    if (f64)
      k::matvec<double, double>(args_, km_->K64.p, p64_.p, q64_.p, s_);
    else
      k::matvec<float, bf16_t>(args_, km_->K32.p, p16_.p, q32_.p, s_);
  });
  k::fill_i32(args_.cg.act, 0, rp_, s_);
  k::fill_i32(ring_.p, 0, ring_.n, s_);
  args_.tm = make_tile(int(mesh_->n), rp_, best.tg_cap, best.passes, best.nper_cap);
  tuned_ = best;
  if (f64) {
    args_.t64 = args_.tm;
  } else {
    const TuneChoice b64 = tune_tiling(key + "_gather64", &StepArgs::t64,
                                       [&] { k::norm_dot(args_, u_.p, nullptr, s_); });
    args_.t64 = make_tile(int(mesh_->n), rp_, b64.tg_cap, b64.passes, b64.nper_cap);
  }
  if (args_.poly) {
    // the preconditioner pass gathers r (float32 or float64): its own tiling
    k::fill_i32(args_.cg.act, 1, rp_, s_);
    k::fill_i32(ring_.p, 1, 1, s_);
    if (f64)
      k::fill_f64(r64_.p, 1.0, nv, s_);
    else
      k::fill_f32(r32_.p, 1.0f, nv, s_);
    const TuneChoice bp = tune_tiling(key + "_precond", &StepArgs::tp, [&] {
      if (f64)
        k::precond_init<double, double>(args_, r64_.p, p64_.p, km_->P64.p, s_);
      else
        k::precond_init<float, bf16_t>(args_, r32_.p, p16_.p, km_->P32.p, s_);
    });
    k::fill_i32(args_.cg.act, 0, rp_, s_);
    k::fill_i32(ring_.p, 0, ring_.n, s_);
    args_.tp = make_tile(int(mesh_->n), rp_, bp.tg_cap, bp.passes, bp.nper_cap);
  }

  // S_eps element kernel: LDS-staged, direct corner reads or lane-split,
  // and 64, as many as are resident at once, or the full count of workgroups
  // per XCD, whichever is fastest for this batch's restart tiles (part_s_
  // holds the largest count's partials).  With every workgroup resident the
  // XCD walks each restart tile's triangles together, so the corner rows
  // that neighbouring triangles share meet in L2.
  // The pick is cached with the restart layout (as the tilings are), so every
  // state of the same batch runs the same S_eps kernel and partial-sum rows,
  // and so gets the same energies bit for bit.
  uint64_t lay = 1469598103934665603ull;  // FNV-1a over the restarts' columns
  for (int r = 0; r < nres_p_; ++r)
    for (int v : {h_res_lo_[r], h_res_len_[r]})
      for (int b = 0; b < 4; ++b) {
        lay ^= uint64_t((uint32_t(v) >> (8 * b)) & 0xffu);
        lay *= 1099511628211ull;
      }
  const std::string skey = key + "_nt" + std::to_string(mesh_->nt) + "_seps" + std::to_string(lay);
  const int seps_nper_max = std::max(1, std::min(kSepsNperMax, (sp_.nchunk + 7) / 8));
  TuneChoice cached;
  if (sp_.ntile > 0 && tune_lookup(skey, &cached) && (cached.tg_cap != 2 || sp_.lanes_ok) &&
      cached.tg_cap >= 0 && cached.tg_cap <= 2 && cached.nper_cap >= 1 &&
      cached.nper_cap <= seps_nper_max) {
    sp_.direct = cached.tg_cap;
    sp_.nper = cached.nper_cap;
  } else if (sp_.ntile > 0) {
    hipEvent_t e0, e1;
    SP_HIP(hipEventCreate(&e0));
    SP_HIP(hipEventCreate(&e1));
    const int nmode = sp_.lanes_ok ? 3 : 2;
    const int nper_max = std::max(1, std::min(kSepsNperMax, (sp_.nchunk + 7) / 8));
    const int resident = std::min(nper_max, k::seps_resident_groups());
    double t_best = 0.0;
    int best = 0, best_nper = nper_max;
    std::vector<int> cands = {nper_max};
    for (int c : {resident, 64})
      if (c < nper_max && std::find(cands.begin(), cands.end(), c) == cands.end()) cands.push_back(c);
    for (int nper : cands) {
      sp_.nper = nper;
      for (int mode = 0; mode < nmode; ++mode) {
        sp_.direct = mode;
        k::energy_seps(args_, sp_, mesh_->tri.p, mesh_->tarea.p, u_.p, part_s_.p, s_);
        SP_HIP(hipEventRecord(e0, s_));
        for (int i = 0; i < 2; ++i)
          k::energy_seps(args_, sp_, mesh_->tri.p, mesh_->tarea.p, u_.p, part_s_.p, s_);
        SP_HIP(hipEventRecord(e1, s_));
        SP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (std::getenv("SEGPART_TUNE_VERBOSE"))
          std::fprintf(stderr, "[segpart tune] S_eps %s, %d groups/xcd: %.1f us\n",
                       mode == 2 ? "lanes" : mode ? "direct" : "staged", nper, 500.0 * ms);
        if ((nper == nper_max && mode == 0) || ms < t_best) {
          t_best = ms;
          best = mode;
          best_nper = nper;
        }
      }
    }
    sp_.direct = best;
    sp_.nper = best_nper;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TuneChoice pick;  // (kernel mode, workgroups per XCD) in the tiling fields
    pick.tg_cap = best;
    pick.passes = 1;
    pick.nper_cap = best_nper;
    pick.us = 500.0 * t_best;
    tune_store(skey, pick);
  }
}

void Solver::push_tables() {
  flush_scale();  // the pending factors belong to the current live masks
  lam_fresh_ = false;
  all_live_ = true;
  for (int c = 0; c < rp_; ++c)
    if (h_seg_len_[c] > 0 && !h_live_[c]) all_live_ = false;
  // the node step's simple kernel: every column in a restart that starts and
  // ends on a multiple of 4 and does not cross a 256-column tile edge
  live_cols_ = 0;
  for (int c = 0; c < rp_; ++c) live_cols_ += (h_seg_len_[c] > 0 && h_live_[c]) ? 1 : 0;
  int fast = args_.ts.tg == 64;
  for (int c = 0; c < rp_ && fast; ++c) {
    const int lo = h_seg_lo_[c], len = h_seg_len_[c];
    fast = len > 0 && ((lo | len) & 3) == 0 && lo / 256 == (lo + len - 1) / 256;
  }
  args_.nodal_fast = fast;
  const int nres = args_.ct.nres;
  args_.ct.nres = nres;
  SP_HIP(hipMemcpyAsync(const_cast<int*>(args_.ct.seg_lo), h_seg_lo_.data(), rp_ * sizeof(int),
                        hipMemcpyHostToDevice, s_));
  SP_HIP(hipMemcpyAsync(const_cast<int*>(args_.ct.seg_len), h_seg_len_.data(), rp_ * sizeof(int),
                        hipMemcpyHostToDevice, s_));
  SP_HIP(hipMemcpyAsync(const_cast<int*>(args_.ct.live), h_live_.data(), rp_ * sizeof(int),
                        hipMemcpyHostToDevice, s_));
  SP_HIP(hipMemcpyAsync(const_cast<double*>(args_.ct.coef), h_coef_.data(), rp_ * sizeof(double),
                        hipMemcpyHostToDevice, s_));
  SP_HIP(hipMemcpyAsync(const_cast<int*>(args_.ct.res_lo), h_res_lo_.data(), nres_p_ * sizeof(int),
                        hipMemcpyHostToDevice, s_));
  SP_HIP(hipMemcpyAsync(const_cast<int*>(args_.ct.res_len), h_res_len_.data(), nres_p_ * sizeof(int),
                        hipMemcpyHostToDevice, s_));
  SP_HIP(hipMemcpyAsync(const_cast<int*>(args_.ct.res_live), h_res_live_.data(),
                        nres_p_ * sizeof(int), hipMemcpyHostToDevice, s_));
  SP_HIP(hipMemcpyAsync(const_cast<double*>(args_.ct.res_ieps2), h_res_ieps2_.data(),
                        nres_p_ * sizeof(double), hipMemcpyHostToDevice, s_));
  std::vector<int4> tiles = k::seps_tiles(h_res_lo_, h_res_len_, nres);
  sp_.ntile = int(tiles.size());
  // the lane-split S_eps kernel needs restarts on 4-column boundaries and
  // tiles of at most 256 columns
  sp_.lanes_ok = 1;
  sp_.wide = 0;
  for (const int4& tl : tiles) {
    if (tl.w - tl.z > 256) sp_.lanes_ok = 0, sp_.wide = 1;
    for (int r = tl.x; r < tl.y; ++r)
      if (h_res_len_[r] > 0 && (h_res_lo_[r] % 4 != 0 || h_res_len_[r] % 4 != 0)) sp_.lanes_ok = 0;
  }
  sp_.tiles = seps_tiles_.p;
  if (!tiles.empty())
    SP_HIP(hipMemcpyAsync(seps_tiles_.p, tiles.data(), tiles.size() * sizeof(int4),
                          hipMemcpyHostToDevice, s_));
  // the host vectors may change right after: wait for the copies
  SP_HIP(hipStreamSynchronize(s_));
}

void Solver::set_columns(const std::vector<int>& seg_lo, const std::vector<int>& seg_len,
                         const std::vector<double>& coef, const std::vector<int>& live,
                         const std::vector<int>& res_lo, const std::vector<int>& res_len,
                         const std::vector<double>& res_ieps2) {
  SP_REQUIRE(int(seg_lo.size()) == rp_ && int(res_lo.size()) <= nres_p_, SP_EINVAL,
             "set_columns: table sizes");
  h_seg_lo_ = seg_lo;
  h_seg_len_ = seg_len;
  h_coef_ = coef;
  h_live_ = live;
  std::fill(h_res_lo_.begin(), h_res_lo_.end(), 0);
  std::fill(h_res_len_.begin(), h_res_len_.end(), 0);
  std::fill(h_res_ieps2_.begin(), h_res_ieps2_.end(), 0.0);
  std::fill(h_res_live_.begin(), h_res_live_.end(), 0);
  for (size_t r = 0; r < res_lo.size(); ++r) {
    h_res_lo_[r] = res_lo[r];
    h_res_len_[r] = res_len[r];
    h_res_ieps2_[r] = res_ieps2[r];
    h_res_live_[r] = res_len[r] > 0;
  }
  args_.ct.nres = int(res_lo.size());
  push_tables();
  aw_fresh_ = false;
}

void Solver::set_restart_live(int r, bool live) {
  SP_REQUIRE(r >= 0 && r < args_.ct.nres, SP_EINVAL, "restart index");
  const int lo = h_res_lo_[r], m = h_res_len_[r];
  for (int j = 0; j < m; ++j) h_live_[lo + j] = live ? 1 : 0;
  h_res_live_[r] = live ? 1 : 0;
  push_tables();
  aw_fresh_ = false;
}

int Solver::poll(const int* dev_counter) {
  SP_HIP(hipMemcpyAsync(h_poll_, dev_counter, sizeof(int), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
  return h_poll_[0];
}

void Solver::sync() { SP_HIP(hipStreamSynchronize(s_)); }

void Solver::acct(double per_elem, double extra) {
  fixed_bytes_ += per_elem * double(mesh_->n) * double(live_cols_) + extra;
}

double Solver::mat_bytes(double value_bytes, int n_mats) const {
  return double(mesh_->n) * double(mesh_->W) * (4.0 + value_bytes * n_mats);
}

void Solver::upload_host(const double* u0, bool normalise) {
  flush_scale();
  aw_fresh_ = false;
  SP_REQUIRE(u0 != nullptr, SP_EINVAL, "NULL u0");
  lam_fresh_ = false;
  const size_t cnt = size_t(R_) * mesh_->n;
  for (size_t i = 0; i < cnt; ++i)
    SP_REQUIRE(std::isfinite(u0[i]), SP_EINVAL, "u0 holds a non-finite value");
  forget_history(0, rp_);
  DevBuf<double> tmp(cnt);
  SP_HIP(hipMemcpyAsync(tmp.p, u0, cnt * sizeof(double), hipMemcpyHostToDevice, s_));
  k::pack(args_.t, 0, R_, tmp.p, mesh_->perm_d.p, u_.p, s_);
  if (normalise) {
    normalise_columns();
  }
  SP_HIP(hipStreamSynchronize(s_));
}

void Solver::upload_device(const double* d_u0, bool normalise, bool check_norms) {
  flush_scale();
  aw_fresh_ = false;
  SP_REQUIRE(d_u0 != nullptr, SP_EINVAL, "NULL u0");
  lam_fresh_ = false;
  forget_history(0, rp_);
  k::pack(args_.t, 0, R_, d_u0, mesh_->perm_d.p, u_.p, s_);
  if (normalise) {
    if (check_norms) {
      normalise_columns();
    } else {
      k::norm_dot(args_, u_.p, nullptr, s_);
      k::red_norm(args_, lam_.p, s_);
      k::scale(args_, u_.p, u_.p, s_);
      lam_fresh_ = all_live_;
    }
  }
}

void Solver::normalise_columns() {
  flush_scale();
  k::norm_dot(args_, u_.p, nullptr, s_);
  k::red_norm(args_, lam_.p, s_);
  std::vector<double> nrm(rp_);
  SP_HIP(hipMemcpyAsync(nrm.data(), args_.cg.nrm, rp_ * sizeof(double), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
  for (int c = 0; c < rp_; ++c)
    if (h_live_[c])
      SP_REQUIRE(std::isfinite(nrm[c]) && nrm[c] > 0, SP_EINVAL,
                 "a component of u0 has zero (or non-finite) L2 norm (column " +
                     std::to_string(c) + ")");
  k::scale(args_, u_.p, u_.p, s_);
  lam_fresh_ = all_live_;
}

void Solver::pack_range(int c_lo, int Rq, const double* d_src) {
  flush_scale();
  aw_fresh_ = false;
  SP_REQUIRE(c_lo >= 0 && Rq >= 0 && c_lo + Rq <= rp_, SP_EINVAL, "column range");
  // the new columns have no previous increment; the other columns keep theirs
  // (each column extrapolates from its own history)
  forget_history(c_lo, Rq);
  lam_fresh_ = false;
  k::pack(args_.t, c_lo, Rq, d_src, mesh_->perm_d.p, u_.p, s_);
}

void Solver::forget_history(int c_lo, int cnt) {
  if (c_lo == 0 && cnt >= rp_) n_prev_ = 0;
  if (cnt <= 0) return;
  std::fill(h_hlen_.begin() + c_lo, h_hlen_.begin() + c_lo + cnt, 0);
  k::fill_i32(args_.hlen + c_lo, 0, size_t(cnt), s_);
  k::fill_i32(args_.ord + c_lo, prm_.extrapolate, size_t(cnt), s_);
}

void Solver::unpack_range(int c_lo, int Rq, double* d_dst) {
  flush_scale();
  SP_REQUIRE(c_lo >= 0 && Rq >= 0 && c_lo + Rq <= rp_, SP_EINVAL, "column range");
  k::unpack(args_.t, c_lo, Rq, u_.p, mesh_->perm_d.p, d_dst, s_);
}

void Solver::normalise_range(int c_lo, int Rq) {
  aw_fresh_ = false;
  std::vector<int> saved = h_live_;
  for (int c = 0; c < rp_; ++c) h_live_[c] = (c >= c_lo && c < c_lo + Rq) ? saved[c] : 0;
  push_tables();
  try {
    normalise_columns();
  } catch (...) {
    h_live_ = saved;
    push_tables();
    throw;
  }
  h_live_ = saved;
  push_tables();
}

void Solver::download_host(double* u) {
  flush_scale();
  const size_t cnt = size_t(R_) * mesh_->n;
  DevBuf<double> tmp(cnt);
  k::unpack(args_.t, 0, R_, u_.p, mesh_->perm_d.p, tmp.p, s_);
  SP_HIP(hipMemcpyAsync(u, tmp.p, cnt * sizeof(double), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
}

void Solver::download_device(double* d_u) {
  flush_scale();
  k::unpack(args_.t, 0, R_, u_.p, mesh_->perm_d.p, d_u, s_);
}

void Solver::heat_fp64() {
  flush_scale();
  k::fill_i32(ring_.p, 0, ring_.n, s_);
  k::init_fp64(args_, u_.p, r64_.p, args_.poly ? nullptr : p64_.p, s_);
  acct(args_.poly ? 16.0 : 24.0, mat_bytes(8.0, 2));
  k::red_init_fp64(args_, s_);
  if (args_.poly) {
    k::precond_init<double, double>(args_, r64_.p, p64_.p, km_->P64.p, s_);
    acct(16.0, mat_bytes(8.0, 1));
  }
  int last = 0;
  for (int it = 0; it < prm_.cg_max_iter; ++it) {
    k::cg_iter<double>(args_, it, u_.p, r64_.p, p64_.p, q64_.p, z64_.p, km_->K64.p,
                       km_->dinv64.p, km_->P64.p, s_, prof_events());
    last = it + 1;
    if (prm_.check_every > 0 && last % prm_.check_every == 0 && last < prm_.cg_max_iter)
      if (poll(ring_.p + last % kRing) == 0) break;
  }
  k::flag_nonconv(args_, ring_.p + last % kRing, s_);
  heat_x_ = u_.p;
}

void Solver::heat_mixed() {
  const bool extrap = prm_.extrapolate != 0;
  double* x = u_.p;
  k::fill_i32(ring_.p, 0, ring_.n, s_);
  const int q = prm_.extrapolate;
  float* acc = extrap ? dh_[q - 1] : nullptr;  // receives g, then this step's increment
  // the norm pass that scaled u left A u (times ||v||_M) in xg_
  const bool fast = aw_fresh_ && extrap && n_prev_ >= 1;
  aw_fresh_ = false;
  if (!fast) flush_scale();  // the other starts read u_ as it is
  if (extrap && n_prev_ >= 1) {
    // start from x0 = u + g, g the polynomial extrapolation of the last heat
    // increments d_k, d_{k-1}, ... (as many as kept and available):
    // g = sum_j (-1)^j C(use, j+1) d_{k-j}, e.g. 3 d_k - 3 d_{k-1} + d_{k-2};
    // g overwrites the oldest kept increment (acc) and x0 goes to xg_
    const int use = std::min(n_prev_, q);
    // q = 1 keeps the newest increment in acc already: nothing to form
    // unless some live column has no history yet
    bool skip = use == 1 && acc == dh_[0];
    for (int c = 0; c < rp_ && skip; ++c) skip = !h_live_[c] || h_hlen_[c] >= 1;
    if (!skip) {
      ExtrapArgs e;
      e.n = use;
      for (int j = 0; j < use; ++j) e.x[j] = dh_[j];
      SP_REQUIRE(q < 2 || size_t(k::kOrderProbes) * size_t(args_.tprobe.nchunk) * rp_ <= part_.n,
                 SP_EINVAL, "extrapolation: partial-sum buffer too small for the order control");
      k::extrap(args_, e, acc, q, s_);
      acct(4.0 * use + 4.0);
    }
    if (fast) {
      // A u and ||M u||^2 from the last step's norm pass: no float64 gather
      k::refine_start(args_, xg_.p, acc, r64_.p, r32_.p, args_.poly ? nullptr : p16_.p, s_);
      acct(args_.poly ? 24.0 : 26.0, mat_bytes(8.0, 1));
      precond_start();
    } else {
      k::init_outer(args_, u_.p, acc, xg_.p, r64_.p, s_);
      acct(32.0, mat_bytes(8.0, 3));
      k::red_outer_init(args_, s_);
    }
    x = xg_.p;
  } else {
    k::init_outer(args_, u_.p, nullptr, nullptr, r64_.p, s_);
    acct(16.0, mat_bytes(8.0, 2));
    k::red_outer_init(args_, s_);
    if (extrap) {
      k::fill_f32(acc, 0.0f, dbuf_[0].n, s_);
      acct(4.0);
    }
  }
  int olast = 0;
  bool prepared = false;  // the last update wrote this sweep's inner start
  // sweep 0 of a fast start expected to need another sweep keeps its
  // correction in d0buf_ and leaves the iterate to the next sweep (one pass
  // over u, x and dacc fewer); deferred: the iterate is not formed yet
  bool deferred = false;
  for (int o = 0; o < prm_.max_outer; ++o) {
    if (!(fast && o == 0) && !prepared) {
      k::inner_init(args_, o, r64_.p, d32_.p, r32_.p, args_.poly ? nullptr : p16_.p, s_);
      acct(args_.poly ? 12.0 : 14.0);
      k::red_inner_init(args_, o, s_);
      precond_start();
    }
    // inner CG in direction-ring form: d is formed from the stored
    // directions when the ring fills and after the last iteration
    int flushed = 0, last = 0;
    const bool blocks = graph_on_ && !prof_ && s_ != nullptr && prm_.check_every == kPRing;
    for (int it = 0; it < prm_.cg_max_iter;) {
      if (blocks && it % kPRing == 0 && it + kPRing <= prm_.cg_max_iter) {
        cg_block(flushed);
        flushed = 1;
        it += kPRing;
      } else {
        k::cg_iter_ring(args_, it, r32_.p, pring_, q32_.p, z16_.p, ah_.p, d32_.p, &flushed, s_,
                        prof_events());
        ++it;
      }
      last = it;
      if (prm_.check_every > 0 && last % prm_.check_every == 0 && last < prm_.cg_max_iter)
        if (poll(ring_.p + last % kRing) == 0) break;
    }
    if (last % kPRing) {
      k::materialize(args_, pring_, ah_.p, 0, last % kPRing, flushed, d32_.p, s_);
      acct(2.0 * (last % kPRing) + (flushed ? 8.0 : 4.0));
    }
    acct(2.0 * (last - last % kPRing) + 12.0 * (last / kPRing));  // ring folds inside the solve
    // with a poll after this sweep the new residual is stored only if
    // another sweep follows (most steps need one); when the last step needed
    // more than one sweep, the update writes the next sweep's start as well
    const bool polled = prm_.check_every > 0 && o + 1 < prm_.max_outer;
    const bool prep = polled && o + 1 < last_sweeps_;
    const bool defer = fast && o == 0 && prep && d0buf_.p;
    const bool formx = deferred;  // this sweep forms the iterate sweep 0 deferred
    const bool ubase = (fast && o == 0 && !defer) || formx;
    args_.usc = ubase && u_pending_ ? args_.cg.isc : nullptr;
    if (defer) {
      k::outer_update(args_, o, nullptr, nullptr, r64_.p, d32_.p, nullptr, true, r32_.p,
                      args_.poly ? nullptr : p16_.p, d0buf_.p, 1, s_);
      acct(28.0 + (args_.poly ? 0.0 : 2.0), mat_bytes(8.0, 1));
    } else {
      k::outer_update(args_, o, x, ubase ? u_.p : nullptr, r64_.p, d32_.p, acc, !polled,
                      prep ? r32_.p : nullptr, prep && !args_.poly ? p16_.p : nullptr,
                      formx ? d0buf_.p : nullptr, formx ? 2 : 0, s_);
      acct(28.0 + (polled && !prep ? 0.0 : 8.0) + (acc ? 8.0 : 0.0) +
               (prep ? (args_.poly ? 4.0 : 6.0) : 0.0) + (formx ? 4.0 : 0.0),
           mat_bytes(8.0, 1));
    }
    deferred = defer;
    args_.usc = nullptr;
    if (prep) {
      k::red_outer_prep(args_, o, s_);
      precond_start();
    } else {
      k::red_outer(args_, o, s_);
    }
    olast = o + 1;
    prepared = prep;
    if (polled) {
      if (poll(args_.oring + olast % kRing) == 0) break;
      if (!prep) {
        k::outer_residual(args_, olast, r64_.p, d32_.p, s_);
        acct(20.0, mat_bytes(8.0, 1));
      }
    }
  }
  if (deferred) {
    // the solve ended after the deferred sweep 0: form the iterate (no
    // column is refining, so no residual work)
    args_.usc = u_pending_ ? args_.cg.isc : nullptr;
    k::outer_update(args_, olast, x, u_.p, r64_.p, d32_.p, acc, false, nullptr, nullptr,
                    d0buf_.p, 2, s_);
    acct(28.0);
    args_.usc = nullptr;
  }
  last_sweeps_ = olast;
  k::flag_nonconv(args_, args_.oring + olast % kRing, s_);
  if (extrap) {
    for (int i = q - 1; i > 0; --i) dh_[i] = dh_[i - 1];
    dh_[0] = acc;
    n_prev_ = std::min(n_prev_ + 1, q);
    k::hist_advance(args_, q, s_);
    for (int c = 0; c < rp_; ++c) h_hlen_[c] = h_live_[c] ? std::min(h_hlen_[c] + 1, q) : 0;
  }
  heat_x_ = x;
}

// First direction of a float32 inner solve under the polynomial
// preconditioner: p = z = P r on the columns starting it, with their r.z.
void Solver::precond_start() {
  if (!args_.poly) return;
  k::precond_init<float, bf16_t>(args_, r32_.p, p16_.p, km_->P32.p, s_);
  acct(6.0, mat_bytes(4.0, 1));
}

void Solver::cg_block(int flushed) {
  const int v = flushed ? 1 : 0;
  if (cg_graph_[v] && std::memcmp(&cg_graph_args_[v], &args_, sizeof(StepArgs)) != 0) {
    SP_HIP(hipGraphExecDestroy(cg_graph_[v]));
    cg_graph_[v] = nullptr;
  }
  if (!cg_graph_[v]) {
    // iterations 0..kPRing-1 use the same ring slots as any block that
    // starts at a multiple of kPRing (kRing divides kPRing)
    static_assert(kPRing % kRing == 0, "ring periods");
    hipGraph_t g = nullptr;
    SP_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
    try {
      int f = flushed;
      for (int i = 0; i < kPRing; ++i)
        k::cg_iter_ring(args_, i, r32_.p, pring_, q32_.p, z16_.p, ah_.p, d32_.p, &f, s_, nullptr);
    } catch (...) {
      (void)hipStreamEndCapture(s_, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    SP_HIP(hipStreamEndCapture(s_, &g));
    hipError_t e = hipGraphInstantiate(&cg_graph_[v], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      cg_graph_[v] = nullptr;
      throw Error(SP_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    std::memcpy(&cg_graph_args_[v], &args_, sizeof(StepArgs));
  }
  SP_HIP(hipGraphLaunch(cg_graph_[v], s_));
}

void Solver::heat() {
  lam_fresh_ = false;
  if (prm_.precision == SP_FP64)
    heat_fp64();
  else
    heat_mixed();
}

void Solver::stage_heat() {
  flush_scale();
  aw_fresh_ = false;
  heat();
  if (heat_x_ != u_.p)
    SP_HIP(hipMemcpyAsync(u_.p, heat_x_, u_.n * sizeof(double), hipMemcpyDeviceToDevice, s_));
  heat_x_ = u_.p;
}

// node step of the heat solution (the iterate the last solve left, u or xg_)
void Solver::node_to_r() {
  if (heat_x_ == xg_.p && xg_.p) {
    // the solve left x in xg_ (mixed precision, extrapolated start): the
    // node step writes v into u_, whose pending state the solve has used
    u_pending_ = false;
    k::nodal(args_, heat_x_, u_.p, true, s_);
    acct(16.0);
    node_out_ = u_.p;
  } else {
    flush_scale();
    k::nodal(args_, heat_x_, r64_.p, false, s_);
    acct(16.0);
    node_out_ = r64_.p;
  }
  heat_x_ = u_.p;
}

void Solver::norm_dot_scale(const double* v, bool defer) {
  // in a step the norm pass also leaves A v in xg_ (free after the node
  // step) for the next step's refinement start
  double* w = (xg_.p && (v == r64_.p || defer)) ? xg_.p : nullptr;
  k::norm_dot(args_, v, w, s_);
  acct(w ? 16.0 : 8.0, mat_bytes(8.0, 2));
  k::red_norm(args_, lam_.p, s_);
  if (defer) {
    u_pending_ = true;  // v is in u_; the state is v * isc
  } else {
    k::scale(args_, v, u_.p, s_);
    acct(16.0);
  }
  lam_fresh_ = all_live_;
  aw_fresh_ = w != nullptr;
}

void Solver::flush_scale() {
  if (!u_pending_) return;
  u_pending_ = false;
  k::scale(args_, u_.p, u_.p, s_);
  acct(16.0);
}

void Solver::stage_node() {
  flush_scale();
  aw_fresh_ = false;
  lam_fresh_ = false;
  node_to_r();
  k::fill_f64(args_.cg.nrm, 1.0, rp_, s_);
  k::scale(args_, r64_.p, u_.p, s_);
}

void Solver::stage_norm() {
  flush_scale();
  aw_fresh_ = false;
  norm_dot_scale(u_.p, false);
}

void Solver::energy() {
  if (args_.ct.nres == 0) return;
  // right after a normalisation of every column the Rayleigh quotients are
  // already in lam (see red_norm); otherwise evaluate them now
  const bool need_rq = !lam_fresh_;
  if (need_rq) {
    k::energy_rq(args_, u_.p, s_);  // quotients: the pending factor cancels
    acct(8.0, mat_bytes(8.0, 2));
  }
  if (sp_.wide) flush_scale();
  args_.usc = u_pending_ ? args_.cg.isc : nullptr;
  k::energy_seps(args_, sp_, mesh_->tri.p, mesh_->tarea.p, u_.p, part_s_.p, s_);
  acct(8.0, double(mesh_->nt) * 20.0);
  args_.usc = nullptr;
  k::red_energy(args_, sp_, part_s_.p, need_rq, lam_.p, seps_.p, energy_.p, s_);
}

void Solver::multipliers_to_host(double* lam_eps) {
  SP_REQUIRE(lam_eps != nullptr, SP_EINVAL, "NULL output");
  flush_scale();
  energy();  // Rayleigh quotients of the current state in lam_
  DevBuf<double> part(size_t(8 * sp_.nper) * rp_), out(rp_);
  k::multipliers(args_, sp_, mesh_->tri.p, mesh_->tarea.p, u_.p, part.p, lam_.p, out.p, s_);
  SP_HIP(hipMemcpyAsync(lam_eps, out.p, R_ * sizeof(double), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
}

void Solver::energy_to_host(double* lam, double* seps, double* E) {
  energy();
  if (lam) SP_HIP(hipMemcpyAsync(lam, lam_.p, R_ * sizeof(double), hipMemcpyDeviceToHost, s_));
  const int nres = int(spec_.m.size());
  if (seps) SP_HIP(hipMemcpyAsync(seps, seps_.p, nres * sizeof(double), hipMemcpyDeviceToHost, s_));
  if (E) SP_HIP(hipMemcpyAsync(E, energy_.p, nres * sizeof(double), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
}

// Steps of a small batch: chunks of up to kSmallChunk steps, one launch each
// (the float64 form whatever the precision setting: at this size it costs
// nothing more); energies at the cadence come back from the device history.
void Solver::step_small(int64_t k) {
  flush_scale();
  const int nres = int(spec_.m.size());
  while (k > 0) {
    const int chunk = int(std::min<int64_t>(k, kSmallChunk));
    SmallArgs sa;
    sa.nsteps = chunk;
    sa.every = int(prm_.energy_every);
    sa.step0 = steps_done_;
    sa.max_iter = prm_.cg_max_iter;
    sa.u = u_.p;
    sa.r = r64_.p;
    sa.p = p64_.p;
    sa.q = q64_.p;
    sa.tri = mesh_->tri.p;
    sa.tarea = mesh_->tarea.p;
    sa.nt = int(mesh_->nt);
    sa.lam = lam_.p;
    sa.seps = seps_.p;
    sa.energy = energy_.p;
    sa.hist = small_hist_.p;
    k::small_steps(args_, sa, s_);
    if (record_history && prm_.energy_every > 0 && nres > 0) {
      std::vector<int> due;
      for (int i = 0; i < chunk; ++i)
        if ((steps_done_ + i + 1) % prm_.energy_every == 0) due.push_back(i);
      if (!due.empty()) {
        std::vector<double> h(size_t(chunk) * nres_p_);
        SP_HIP(hipMemcpyAsync(h.data(), small_hist_.p, h.size() * sizeof(double),
                              hipMemcpyDeviceToHost, s_));
        SP_HIP(hipStreamSynchronize(s_));
        for (int i : due)
          for (int r = 0; r < nres; ++r)
            if (h_res_live_[r]) hist_[r].push_back({steps_done_ + i + 1, h[size_t(i) * nres_p_ + r]});
      }
    }
    steps_done_ += chunk;
    k -= chunk;
  }
  lam_fresh_ = all_live_;
  forget_history(0, rp_);
  aw_fresh_ = false;
  heat_x_ = u_.p;
}

void Solver::step(int64_t k) {
  SP_REQUIRE(k >= 0, SP_EINVAL, "step count must be >= 0");
  if (small_) {
    step_small(k);
    return;
  }
  const int nres = int(spec_.m.size());
  std::vector<double> E(nres);
  for (int64_t i = 0; i < k; ++i) {
    heat();
    node_to_r();
    norm_dot_scale(node_out_, node_out_ == u_.p);
    ++steps_done_;
    if (prm_.energy_every > 0 && steps_done_ % prm_.energy_every == 0) {
      if (record_history) {
        energy_to_host(nullptr, nullptr, E.data());
        for (int r = 0; r < nres; ++r)
          if (h_res_live_[r]) hist_[r].push_back({steps_done_, E[r]});
      } else {
        energy();
      }
    }
  }
}

void Solver::run_to_stop() {
  const int nres = int(spec_.m.size());
  std::vector<double> E(nres), Eprev(nres);
  energy_to_host(nullptr, nullptr, Eprev.data());
  for (int r = 0; r < nres; ++r) hist_[r].push_back({steps_done_, Eprev[r]});
  restart_steps.assign(nres, 0);
  int running = nres;
  const int64_t every = prm_.energy_every;
  while (running > 0 && steps_done_ < prm_.max_steps) {
    const int64_t k = std::min<int64_t>(every - steps_done_ % every, prm_.max_steps - steps_done_);
    step(k);
    if (steps_done_ % every != 0) break;  // hit max_steps between checks
    for (int r = 0; r < nres; ++r) {
      if (!h_res_live_[r]) continue;
      E[r] = hist_[r].back().second;
      restart_steps[r] = steps_done_;
      if (std::fabs(E[r] - Eprev[r]) < prm_.stop_tol) {
        set_restart_live(r, false);
        --running;
      }
      Eprev[r] = E[r];
    }
  }
  for (int r = 0; r < nres; ++r)
    if (h_res_live_[r]) restart_steps[r] = steps_done_;
  // make every restart visible again for the final energies and labels
  for (int r = 0; r < nres; ++r) h_res_live_[r] = 1;
  for (int c = 0; c < R_; ++c) h_live_[c] = 1;
  push_tables();
}

void Solver::labels_device(int32_t* d_lab, int32_t* d_lab_am) {
  flush_scale();
  if (args_.ct.nres == 0) return;
  k::labels(args_, u_.p, mesh_->perm_d.p, d_lab, d_lab_am, s_);
}

void Solver::labels_host(int32_t* lab, int32_t* lab_am) {
  flush_scale();
  const size_t cnt = size_t(spec_.m.size()) * mesh_->n;
  DevBuf<int32_t> a(lab ? cnt : 0), b(lab_am ? cnt : 0);
  k::labels(args_, u_.p, mesh_->perm_d.p, a.p, b.p, s_);
  if (lab) SP_HIP(hipMemcpyAsync(lab, a.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s_));
  if (lab_am) SP_HIP(hipMemcpyAsync(lab_am, b.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
}

sp_stats Solver::stats() {
  long long st[kStats] = {};
  std::vector<int> it(rp_);
  SP_HIP(hipMemcpyAsync(st, stat_.p, sizeof(st), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipMemcpyAsync(it.data(), args_.cg.iters, rp_ * sizeof(int), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
  sp_stats out{};
  out.steps_done = steps_done_;
  out.cg_iters = st[0];
  out.outer_sweeps = st[1];
  out.col_iters_max = it.empty() ? 0 : *std::max_element(it.begin(), it.end());
  out.converged = st[2] == 0;
  // CG iterations: the columns still iterating (device count) x the
  // iteration's bytes per element (kernel_time's classes), and the matrices
  // once per iteration with work
  const bool f64 = prm_.precision == SP_FP64 || small_;
  const double n = double(mesh_->n), vb = f64 ? 8.0 : 4.0;
  const bool poly = args_.poly != 0;
  double per_elem = 0.0;
  for (int k = 0; k < kKernelClasses; ++k) per_elem += class_bytes(k, f64);
  out.hbm_bytes = fixed_bytes_ + double(st[3]) * n * per_elem +
                  double(st[0]) * mat_bytes(vb, 1) * (poly ? 2.0 : 1.0);
  return out;
}

bool Solver::converged() { return stats().converged != 0; }

int64_t Solver::column_iters(int c_lo, int cnt) {
  SP_REQUIRE(c_lo >= 0 && cnt >= 0 && c_lo + cnt <= rp_, SP_EINVAL, "column range");
  std::vector<int> it(size_t(cnt) + 1);
  if (cnt > 0) {
    SP_HIP(hipMemcpyAsync(it.data(), args_.cg.iters + c_lo, size_t(cnt) * sizeof(int),
                          hipMemcpyDeviceToHost, s_));
    SP_HIP(hipStreamSynchronize(s_));
  }
  int64_t tot = 0;
  for (int i = 0; i < cnt; ++i) tot += it[i];
  return tot;
}

const hipEvent_t* Solver::prof_events() {
  if (!prof_) return nullptr;
  if (ev_used_ == ev_.size()) {
    if (ev_.size() >= 4096) prof_flush();
    if (ev_used_ == ev_.size()) {
      std::array<hipEvent_t, 8> e{};
      for (auto& x : e) SP_HIP(hipEventCreate(&x));
      ev_.push_back(e);
    }
  }
  return ev_[ev_used_++].data();
}

void Solver::prof_flush() {
  if (ev_used_ == 0) return;
  SP_HIP(hipStreamSynchronize(s_));
  for (size_t i = 0; i < ev_used_; ++i) {
    for (int k = 0; k < (args_.poly ? 4 : 3); ++k) {
      float ms = 0.f;
      SP_HIP(hipEventElapsedTime(&ms, ev_[i][2 * k], ev_[i][2 * k + 1]));
      prof_ms_[k] += ms;
      ++prof_launches_[k];
    }
  }
  ev_used_ = 0;
}

void Solver::read_stat(long long* st) {
  SP_HIP(hipMemcpyAsync(st, stat_.p, kStats * sizeof(long long), hipMemcpyDeviceToHost, s_));
  SP_HIP(hipStreamSynchronize(s_));
}

void Solver::profile(bool on) {
  prof_flush();
  prof_ = on;
  for (int k = 0; k < kKernelClasses; ++k) {
    prof_launches_[k] = 0;
    prof_ms_[k] = 0.0;
  }
  read_stat(prof_stat0_);
}

// Bytes per element that one CG iteration's kernel class moves per column
// still iterating (vectors only; the matrices and diagonals are added per
// launch).  float64 CG: 0 q = K p reads p, writes q; 1 x += a p, r -= a q
// reads x, r, p, q, writes x, r; 2 p = z + b p reads r (or z), p, writes p;
// 3 z = P r reads r, writes z.  float32 inner CG: r and q float32, the ring
// directions p and the preconditioner output z bf16; 1 reads r, q and
// writes r (no iterate).
double Solver::class_bytes(int which, bool f64) const {
  if (f64 || small_) {
    const double b[kKernelClasses] = {16.0, 48.0, 24.0, args_.poly ? 16.0 : 0.0};
    return b[which];
  }
  const double b[kKernelClasses] = {6.0, 12.0, args_.poly ? 6.0 : 8.0, args_.poly ? 6.0 : 0.0};
  return b[which];
}

void Solver::kernel_time(int which, int64_t* launches, double* ms, double* bytes_per_launch) {
  SP_REQUIRE(which >= 0 && which < kKernelClasses, SP_EINVAL, "kernel class must be 0, 1, 2 or 3");
  prof_flush();
  if (launches) *launches = prof_launches_[which];
  if (ms) *ms = prof_ms_[which];
  if (bytes_per_launch) {
    // Minimum HBM traffic, summed over the profiled launches and divided by
    // their count: the vectors of every column still iterating
    // (class_bytes), plus per launch with work the matrix K (class 0) or P
    // (class 3) as indices and values, or the Jacobi diagonal (classes 1 and
    // 2 without the polynomial preconditioner).  Launches after convergence
    // exit at once and move no data.
    long long st[kStats];
    read_stat(st);
    const double work_iters = double(st[0] - prof_stat0_[0]);
    const double col_iters = double(st[3] - prof_stat0_[3]);
    const double s = prm_.precision == SP_FP64 ? 8.0 : 4.0;
    const double n = double(mesh_->n);
    const double mat = n * double(mesh_->W) * (4.0 + s);
    double b = n * col_iters * class_bytes(which, prm_.precision == SP_FP64);
    b += work_iters * (which == 0 || which == 3 ? mat : args_.poly ? 0.0 : n * s);
    *bytes_per_launch = prof_launches_[which] ? b / double(prof_launches_[which]) : 0.0;
  }
}

namespace {
std::mutex g_dead_mu;
std::vector<Solver*> g_dead;
}  // namespace

void defer_delete(Solver* s) {
  std::lock_guard<std::mutex> g(g_dead_mu);
  g_dead.push_back(s);
}

void reap_deferred() {
  std::vector<Solver*> v;
  {
    std::lock_guard<std::mutex> g(g_dead_mu);
    v.swap(g_dead);
  }
  for (Solver* s : v) delete s;
}

}  // namespace sp
