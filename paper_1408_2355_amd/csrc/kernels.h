// Launchers of the time-step kernels (kernels.hip).  All arrays are device
// pointers.  Vector layout: [n][rp] row-major (the rp values of one vertex
// are contiguous; column c is one component of one restart).
#pragma once

#include "internal.h"

namespace sp {

constexpr int kRing = 4;  // slots of the per-iteration active-column counters

// bfloat16 storage element: the upper half of a float32 (rounded to nearest
// even on store).  The float32 inner CG keeps its directions in it.
struct bf16_t {
  uint16_t bits;
};

// Per-column tables of a batch (device).
struct ColTab {
  const int* seg_lo = nullptr;   // first column of the column's restart
  const int* seg_len = nullptr;  // m of the column's restart
  const double* coef = nullptr;  // 2 tau / eps^2 of the column's restart
  const int* live = nullptr;     // 1 = column belongs to a running restart
  const int* res_lo = nullptr;   // per restart: first column (for the energy)
  const int* res_len = nullptr;  // per restart: m
  const double* res_ieps2 = nullptr;  // per restart: 1 / eps^2
  const int* res_live = nullptr;      // per restart: running
  int nres = 0;
  int nres_p = 0;  // padded restart count used by the triangle tiling
};

// Per-column CG scalars (device).
struct CgCols {
  double* bb;     // ||b||^2 = ||M u||^2
  double* rz;     // r . z
  double* tol2;   // squared absolute stopping threshold of the current solve
  double* alpha;
  double* beta;
  double* rr_o;   // outer residual norm^2 (mixed)
  double* nrm;    // M-norms (normalisation)
  double* bb_next;  // ||M u||^2 of the state the last norm pass scaled
  double* isc;      // 1 / nrm (1 on columns that were not live)
  int* act;       // column active in the current (inner) CG
  int* act_o;     // column active in the outer refinement (mixed)
  int* iters;     // CG iterations taken (cumulative)
  int* sweeps;    // outer sweeps taken (cumulative)
};

struct StepArgs {
  Tile t;   // tiling of the streaming row kernels (no neighbour gathers)
  Tile ts;  // tiling of the streaming kernels without column sums (node step,
            // ring fold, extrapolation, scaling): more workgroups in flight
  Tile tm;  // tiling of the CG matrix product and the refinement update (gathers
            // float32 in mixed precision); same n, rp
  Tile t64;  // tiling of the kernels that gather float64 values (solve set-up,
             // norms, Rayleigh quotients); same n, rp
  Tile tprobe;           // tiling over the sampled rows of the extrapolation's
  int probe_stride = 1;  // order control (every probe_stride-th row)
  Tile tp;   // tiling of the polynomial preconditioner's pass (its own gather,
              // timed separately: its operand is the float32 r)
  int W;
  int nodal_fast = 0;  // set by the host when every column group lies in one 4-aligned
                       // restart inside its 256-column tile (ts one row per
                       // wavefront): the node step then runs without its general path
  const int* cols;
  const double* M64;
  const double* A64;
  const double* K64;
  const double* dinv64;
  const float* K32;
  const float* dinv32;
  double tau;
  double rtol2;        // cg_rtol^2
  double inner_rtol2;  // inner_rtol^2
  double inner_floor2 = 0.81;  // an inner solve stops at sqrt(this) x the outer target
  // Deferred normalisation: non-null while the state vector holds v and the
  // state is v * usc[c] per column (usc = cg.isc); the refinement update's
  // ubase and the S_eps kernels apply it as they read.
  const double* usc = nullptr;
  // Region mask [n][rp] (0/1 per vertex and column), float64 solves only: the
  // heat solve is restricted to the vertices of each column's region (the
  // Dirichlet eigenproblems of a partition); null = no restriction.
  const uint8_t* mask = nullptr;
  ColTab ct;
  CgCols cg;
  int* hlen = nullptr;  // per column: heat increments kept for the extrapolated
                        // start (0 .. extrapolate)
  int* ord = nullptr;   // per column: order of its next extrapolation (0 ..
                        // extrapolate), chosen from its increments' differences
  // Polynomial preconditioner of the CG (poly != 0): z = P r with
  // P = D^-1 (c0 I + c1 K D^-1), the Chebyshev polynomial of degree 1 for the
  // spectrum of D^-1 K applied to the Jacobi step, stored on K's pattern
  // (P64 / P32); part2 [nblk][rp] holds its pass's partial sums r.z (tiling
  // tp).  poly == 0: Jacobi, z = D^-1 r formed inside the update kernels.
  int poly = 0;
  const double* P64 = nullptr;
  const float* P32 = nullptr;
  double* part2 = nullptr;
  double* part;        // [3][nchunk][rp] partial sums
  int* ring;           // [kRing] inner active counts
  int* oring;          // [kRing] outer active counts
  long long* stat;     // [0] CG iterations with work, [1] outer sweeps, [2] cap hit,
                       // [3] active columns summed over CG iterations
};

// Direction ring of the float32 inner CG (see kernels.hip).
constexpr int kPRing = 8;
struct RingArgs {
  const bf16_t* p[kPRing] = {};
  int row[kPRing] = {};  // coefficient row (ring slot) of each direction
  int n = 0;
  int accumulate = 0;    // 0: d = sum, 1: d += sum
};

// Extrapolated start: the kept heat increments, newest first (up to
// kMaxExtrap); each column uses as many as its history length allows.
constexpr int kMaxExtrap = 8;
struct ExtrapArgs {
  const float* x[kMaxExtrap] = {};
  int n = 0;
};

// Batches with n * rp <= kSmallMaxValues, rp <= kSmallMaxCols and at most
// kSmallMaxRestarts restarts can run whole time steps in one resident
// workgroup (small_steps).
constexpr int kSmallMaxValues = 16384;
constexpr int kSmallMaxCols = 256;
constexpr int kSmallMaxRestarts = 64;
struct SmallArgs {
  int nsteps = 0;
  int every = 0;        // energy cadence (0: none)
  long long step0 = 0;  // steps taken before this launch
  int max_iter = 0;     // CG iteration cap per solve
  double* u = nullptr;  // state (also the CG iterate)
  double* r = nullptr;  // residual, then the node-step output
  double* p = nullptr;
  double* q = nullptr;
  const int* tri = nullptr;
  const double* tarea = nullptr;
  int nt = 0;
  double* lam = nullptr;     // per column
  double* seps = nullptr;    // per restart
  double* energy = nullptr;  // per restart
  double* hist = nullptr;    // [nsteps][nres_p] energies at the cadence (nullable)
};

// Triangle-chunk x restart-tile plan of the S_eps element kernel.
struct SepsPlan {
  const int4* tiles = nullptr;  // (r0, r1, c0, c1): restarts [r0, r1) use columns [c0, c1)
  int ntile = 0;
  int nchunk = 0;  // triangle chunks
  int tchunk = 0;  // triangles per chunk
  int nper = 0;    // workgroups per XCD (8 * nper partial rows per restart)
  int nt = 0;      // triangles
  int nres_p = 0;  // row stride of the partial sums
  int direct = 0;  // 0 = staged in LDS, 1 = corners read from global memory by one
                   // lane per restart, 2 = lane-split restarts (needs lanes_ok)
  int wide = 0;      // some tile spans more than 256 columns (the direct kernel
                     // then cannot stage its column factors)
  int lanes_ok = 0;  // every restart of every tile starts and ends on a multiple of 4
};
namespace k {
std::vector<int4> seps_tiles(const std::vector<int>& res_lo, const std::vector<int>& res_len,
                             int nres);
void flag_nonconv(const StepArgs& a, const int* counter, hipStream_t s);
// float64 CG (plain form): x is the state u itself.  p nullable (the
// preconditioner pass writes the first direction: precond_init).
void init_fp64(const StepArgs& a, const double* u, double* r, double* p, hipStream_t s);
// Polynomial preconditioner at the start of a solve (a.poly): p = z = P r on
// the columns starting this solve (activity count ring[0]), and their r.z
// into cg.rz.  z is the pass's output buffer (here: the first direction;
// Z = bf16_t for the float32 CG's ring, double for the float64 CG).
template <typename T, typename Z>
void precond_init(const StepArgs& a, const T* r, Z* p, const T* P, hipStream_t s);
void red_init_fp64(const StepArgs& a, hipStream_t s);
// one CG iteration on type T vectors (the float64 plain CG); ev,
// when given, holds 8 events recorded around the matrix product, the x/r
// update, the p update and (a.poly) the preconditioner pass (before/after
// each; without a.poly the last pair stays unrecorded).  z, P: the preconditioner's
// output and matrix (used when a.poly).
template <typename T>
void cg_iter(const StepArgs& a, int it, T* x, T* r, T* p, T* q, T* z, const T* K, const T* dinv,
             const T* P, hipStream_t s, const hipEvent_t* ev);
// one iteration of the float32 inner CG in direction-ring form: directions
// in pring[kPRing] (bf16; iteration it uses slot it % kPRing and writes the
// next), alpha rows in ah[kPRing][rp]; when the ring fills, d (+)= sum
// alpha p and *flushed is set (later folds accumulate).  z (bf16): the
// polynomial preconditioner's output.
void cg_iter_ring(const StepArgs& a, int it, float* r, bf16_t* const* pring, float* q, bf16_t* z,
                  double* ah, float* d, int* flushed, hipStream_t s, const hipEvent_t* ev);
// d (+)= sum over count ring slots from first (cyclic) of alpha_slot p_slot
void materialize(const StepArgs& a, bf16_t* const* pring, const double* ah, int first, int count,
                 int accumulate, float* d, hipStream_t s);
// the CG matrix product alone (q = K p over the active columns; needs
// ring[0] != 0), used to time tilings; p stored as S (float32 CG: bf16)
template <typename T, typename S>
void matvec(const StepArgs& a, const T* K, const S* p, T* q, hipStream_t s);
// mixed precision refinement
// r64 = M u - K x0 with x0 = u + g (g nullable: x0 = u, nothing written to
// x0); x0 must not alias u
void init_outer(const StepArgs& a, const double* u, const float* g, double* x0, double* r64,
                hipStream_t s);
void red_outer_init(const StepArgs& a, hipStream_t s);
// (p nullable: the polynomial preconditioner's pass writes the first direction)
void inner_init(const StepArgs& a, int o, const double* r64, float* d, float* r, bf16_t* p,
                hipStream_t s);
// refinement start and first inner start from the norm pass's A v (w) and
// ||M u||^2; replaces init_outer, red_outer_init, inner_init and
// red_inner_init of sweep 0 (the iterate u + g is formed by the first
// outer_update in ubase mode)
void refine_start(const StepArgs& a, const double* w, const float* g, double* r64, float* r,
                  bf16_t* p, hipStream_t s);  // p nullable as in inner_init
void red_inner_init(const StepArgs& a, int o, hipStream_t s);
// x += d (ubase given: x = ubase + dacc + d), r64 -= K d on the columns
// still refining; dacc (nullable) += d; store_r false: r64 not stored (then
// outer_residual before another sweep).  rn, pn (nullable, both or neither):
// also the next sweep's inner start r = float(r64), p = D r (r64 stored);
// reduce with red_outer_prep instead of red_outer
// d0mode 1 (deferred iterate; x, ubase, dacc unused): d0 = d where the column
// is refining, 0 on the other columns of live groups; d0mode 2 (ubase given):
// x = ubase + dacc + d0 (+ d), dacc += d0 (+ d) on every live group.
void outer_update(const StepArgs& a, int o, double* x, const double* ubase, double* r64,
                  const float* d, float* dacc, bool store_r, float* rn, bf16_t* pn, float* d0,
                  int d0mode, hipStream_t s);
// outer test of sweep o and, for the columns still refining, the scalars of
// the inner start that outer_update(rn, pn) wrote
void red_outer_prep(const StepArgs& a, int o, hipStream_t s);
// r64 -= K d on the columns still refining after sweep o - 1
void outer_residual(const StepArgs& a, int o, double* r64, const float* d, hipStream_t s);
// y = sum_{j < h_c} (-1)^j C(h_c, j+1) e.x[j] per live column c, h_c =
// min(hlen[c], e.n); 0 on the others; y may be one of the sources
// h_c = min(hlen[c], ord[c], e.n).  qmax >= 2: first the order control, on
// a sample of rows: ord of every live column with two or more kept increments
// is set to the order j of least backward difference D_j of its increments
// (qmax when the differences still fall at the deepest one kept).  It writes
// kOrderProbes slots of partial sums (tiling tprobe): a.part must hold
// kOrderProbes x tprobe.nchunk x rp doubles.
constexpr int kOrderProbes = 5;
void extrap(const StepArgs& a, const ExtrapArgs& e, float* y, int qmax, hipStream_t s);
// hlen[c] = live ? min(hlen[c] + 1, q) : 0 (after a heat solve)
void hist_advance(const StepArgs& a, int q, hipStream_t s);
void red_outer(const StepArgs& a, int o, hipStream_t s);
// node step and normalisation
// keep: columns that are not live keep out's value (out is the state)
void nodal(const StepArgs& a, const double* u, double* out, bool keep, hipStream_t s);
// v.Mv, v.Av, ||Mv||^2 partials; w (nullable) receives A v
void norm_dot(const StepArgs& a, const double* v, double* w, hipStream_t s);
// M-norms of the live columns of the vector norm_dot saw; lam (nullable)
// receives their Rayleigh quotients
void red_norm(const StepArgs& a, double* lam, hipStream_t s);
// u *= mask (region restriction of the state)
void apply_mask(const StepArgs& a, double* u, hipStream_t s);
// adjacency of regions across mesh edges: adj[off[r] + i * m_r + j] = 1 when
// a vertex of region i of restart r neighbours one of region j (labels
// [nres][n] in the renumbered order; values outside 0..m_r-1 are ignored)
void region_graph(const StepArgs& a, const int32_t* labels, const int* off, const int* mres,
                  int nres, uint8_t* adj, hipStream_t s);
// Lagrange multipliers lambda^eps [rp] of the state u (unit norm, lam its
// Rayleigh quotients); part [8 sp.nper][rp] scratch
void multipliers(const StepArgs& a, const SepsPlan& sp, const int32_t* tri, const double* tarea,
                 const double* u, double* part, const double* lam, double* out, hipStream_t s);
// u = v / nrm on the live columns (u may be v)
void scale(const StepArgs& a, const double* v, double* u, hipStream_t s);
// energies
void energy_rq(const StepArgs& a, const double* u, hipStream_t s);
void energy_seps(const StepArgs& a, const SepsPlan& sp, const int32_t* tri, const double* tarea,
                 const double* u, double* part_s, hipStream_t s);
// workgroups of the lane-split S_eps kernel resident on one XCD at once
int seps_resident_groups();
void red_energy(const StepArgs& a, const SepsPlan& sp, const double* part_s, bool with_lambda,
                double* lam,
                double* seps, double* energy, hipStream_t s);
// nsteps whole time steps (float64 CG) of a small batch in one workgroup
void small_steps(const StepArgs& a, const SmallArgs& sa, hipStream_t s);
// labels and layout changes
void labels(const StepArgs& a, const double* u, const int32_t* perm, int32_t* lab,
            int32_t* lab_am, hipStream_t s);
void pack(const Tile& t, int c_lo, int Rq, const double* u0, const int32_t* perm, double* u,
          hipStream_t s);
void unpack(const Tile& t, int c_lo, int Rq, const double* u, const int32_t* perm, double* out,
            hipStream_t s);
}  // namespace k

}  // namespace sp
