/*
 * segpart.h -- C ABI of libsegpart, a single-GPU (AMD MI355X, gfx950) time
 * stepper for the eigenfunction-segregation method of Elliott & Ranner,
 * "A computational approach to an optimal partition problem on surfaces"
 * (arXiv 1408.2355).
 *
 * The method (Section 2 of the paper) looks for m nonnegative functions u_i
 * on a triangulated closed surface Gamma_h, each of unit L2 norm, that
 * minimise sum_i int |grad u_i|^2 plus the segregation penalty
 * (1/eps^2) int sum_i sum_{j!=i} u_i^2 u_j^2.  It runs the operator-splitting
 * gradient flow of Algorithm 2.2: per time step tau,
 *   1. heat step   (M + tau A) u~_i = M u_i            (implicit Euler, P1 FEM)
 *   2. node step   u^_i = u~_i exp(-(2 tau/eps^2)(S - u~_i^2)),  S = sum_j u~_j^2
 *   3. normalise   u_i = u^_i / ||u^_i||_{L2(Gamma_h)}
 * and reads off the eigenvalue estimates lambda_i = u_i^T A u_i / u_i^T M u_i
 * (Section 3.2), S_eps (equation Seps-u), E = sum lambda_i + S_eps, and the
 * partition {v_i > 0}, v_i = u_i - sum_{j!=i} u_j (equation vi).
 *
 * Conventions shared by every entry point:
 *  - Every int-returning call returns SP_OK (0) or a negative status below;
 *    no C++ exception crosses the ABI.  sp_last_error() gives the message of
 *    the last failure on the calling thread.
 *  - Pointers named d_* are device pointers (HIP global memory on the current
 *    device); all other array pointers are host pointers.  The caller owns
 *    every buffer it passes; the library copies inputs during the call and
 *    never keeps a caller pointer after returning (except the async call,
 *    whose buffers must stay valid until its stream passes the call).
 *  - Vertex numbering is always the caller's: the library may renumber
 *    vertices internally for locality and undoes it on output.
 *  - A batch holds n_restarts independent restarts.  Restart r has m[r] >= 1
 *    components and its own eps[r] > 0; all restarts of a batch share the
 *    mesh and tau.  State arrays u0 / u are float64 with shape
 *    [sum_r m[r]][n_vert]: restart r's components are the m[r] consecutive
 *    rows starting at sum_{s<r} m[s], one component per row.
 *  - Per-component outputs (lambda) have length sum_r m[r] in the same
 *    order; per-restart outputs (s_eps, energy) have length n_restarts;
 *    labels are int32 [n_restarts][n_vert].
 */
#ifndef SEGPART_H
#define SEGPART_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SP_VERSION_MAJOR 1
#define SP_VERSION_MINOR 3  /* 1.1: continuation, partition post-processing, multipliers;
                               1.2: checkpoint/restore, sp_stats.hbm_bytes, per-column
                               extrapolation history, sp_solve_async_noalloc;
                               1.3: sp_params.precond (polynomial preconditioner) */

enum sp_status {
  SP_OK = 0,
  SP_EINVAL = -1,    /* invalid argument (sizes, m < 1, eps <= 0, tau <= 0, NaN input,
                        a component of u0 with zero L2 norm, bad stage id ...)   */
  SP_EMESH = -2,     /* not a closed triangulated surface: index out of range, zero-area
                        triangle, an edge not shared by exactly two triangles      */
  SP_ENOMEM = -3,    /* host or device allocation failed, or the server's HBM budget
                        cannot hold the request                                    */
  SP_EDEVICE = -4,   /* HIP runtime error (no device, launch failure ...)          */
  SP_ENOCONV = -5,   /* a linear solve reached its iteration cap before its
                        tolerance; all outputs were still written                   */
  SP_EAGAIN = -6,    /* server: the request has not finished yet                   */
  SP_ENOTFOUND = -7  /* server: unknown or already fetched ticket                  */
};

/* Message of the last failure on this thread ("" if none).  Never NULL. */
const char* sp_last_error(void);
/* Library version; either pointer may be NULL. */
int sp_version(int* major, int* minor);

/* ------------------------------------------------------------------ mesh --
 * The triangulated surface Gamma_h of Section 2.1: vertices on the smooth
 * surface, flat triangles, P1 space S_h.  Creating a mesh validates it,
 * assembles the consistent mass matrix M (int phi_z phi_w) and the stiffness
 * matrix A (int grad phi_z . grad phi_w) on the GPU and keeps them there.
 */
typedef struct sp_mesh sp_mesh;

/* xyz: host float64 [n_vert][3]; tri: host int32 [n_tri][3] vertex indices.
 * Errors: SP_EINVAL (n_vert < 3, n_tri < 1, NULL), SP_EMESH (see above),
 * SP_ENOMEM, SP_EDEVICE.  On success *out owns device memory until
 * sp_mesh_destroy. */
int sp_mesh_create(int64_t n_vert, const double* xyz, int64_t n_tri, const int32_t* tri,
                   sp_mesh** out);
/* Sizes of a mesh: vertices, triangles, stored nonzeros of M (and of A, same
 * pattern), and |Gamma_h| = sum of triangle areas.  NULL outputs are skipped. */
int sp_mesh_info(const sp_mesh* mesh, int64_t* n_vert, int64_t* n_tri, int64_t* nnz,
                 double* area);
enum { SP_MAT_M = 0, SP_MAT_A = 1 };
/* Copy M (which = SP_MAT_M) or A (SP_MAT_A) out as CSR in the caller's vertex
 * numbering, columns sorted within each row.  row_ptr [n_vert + 1] int64,
 * col [nnz] int32, val [nnz] float64 (host). */
int sp_mesh_export(const sp_mesh* mesh, int32_t which, int64_t* row_ptr, int32_t* col,
                   double* val);
/* Frees the mesh.  Every state, solve and server request using it must be
 * finished first.  NULL is ignored. */
void sp_mesh_destroy(sp_mesh* mesh);

/* ------------------------------------------------------------- parameters --
 * precision SP_FP64: every vector and reduction in float64, plain Jacobi-
 * preconditioned CG on (M + tau A) per column.
 * precision SP_MIXED: float64 outer iterative refinement (residual
 * r = b - (M + tau A) x in float64, x += d) around float32 Jacobi-CG inner
 * solves for d; the M-norm, the node step and the energies stay float64.
 */
enum { SP_FP64 = 0, SP_MIXED = 1 };

typedef struct {
  double tau;           /* time step, > 0 (Algorithm 2.2)                           */
  int64_t n_steps;      /* > 0: run exactly this many steps.  0: run until E changes
                           by less than stop_tol between two energy checks, per
                           restart (Section 2.2), at most max_steps                 */
  double stop_tol;      /* stopping threshold on |E_k - E_{k-energy_every}| (paper: 1e-6) */
  int64_t max_steps;    /* cap for n_steps == 0                                      */
  int64_t energy_every; /* energy cadence in steps (paper: M_tau with M_tau tau = 0.1);
                           0 = energy only at the end (not allowed with n_steps == 0) */
  int32_t precision;    /* SP_FP64 or SP_MIXED.  Small batches (vertices x columns
                           padded to 4 <= 16384, <= 256 columns, <= 64 restarts) run
                           whole steps in one resident workgroup with float64 CG
                           whatever this says (at that size it costs nothing more);
                           the environment variable SEGPART_SMALL=0 turns that off */
  double cg_rtol;       /* per column stop when ||b - (M+tau A) x||_2 <= cg_rtol ||M u||_2 */
  int32_t cg_max_iter;  /* cap on CG iterations per solve (per inner solve in SP_MIXED) */
  double inner_rtol;    /* SP_MIXED: relative residual reduction of each float32 solve */
  int32_t max_outer;    /* SP_MIXED: cap on refinement sweeps per time step          */
  int32_t check_every;  /* CG iterations between host-side convergence polls; 0 = no
                           polling (cg_max_iter device iterations are enqueued and the
                           kernels exit at once after convergence)                  */
  int32_t extrapolate;  /* SP_MIXED only: number q (0..8) of previous heat increments
                           d = u~ - u used to start each heat solve from u + g
                           instead of from u; g extrapolates the increments with a
                           polynomial through the last q of them,
                           g = sum_{j<q} (-1)^j C(q, j+1) d_{k-j} (q = 1: d_k;
                           q = 3: 3 d_k - 3 d_{k-1} + d_{k-2}), with fewer terms
                           while fewer steps have been taken.  The solution is the
                           same to cg_rtol, only the start moves.  Costs q float32
                           vectors and one float64 vector per batch.  0 = start
                           from u.  Ignored in SP_FP64 (always starts from u).
                           Each column keeps its own history: a request admitted
                           to a running server batch starts from its own state
                           and the resident columns keep theirs.  q >= 2 is the
                           largest order: before each extrapolation every column
                           picks its order j in 0..q as the one whose backward
                           difference of its kept increments, D_j = sum_{i<=j}
                           (-1)^i C(j, i) d_{k-i}, is smallest on a sample of
                           about 8192 vertices (q when the differences still fall
                           at the deepest one kept): low orders while the flow
                           still smooths a rough start, q once it is smooth  */
  int32_t precond;      /* CG preconditioner (both precisions).  SP_PRECOND_JACOBI:
                           z = D^-1 r, D the diagonal of M + tau A.
                           SP_PRECOND_CHEB1: z = (c0 I + c1 D^-1 K) D^-1 r, the
                           degree-1 Chebyshev polynomial for the spectrum [a, b]
                           of D^-1 K (K = M + tau A; a, b estimated once per mesh
                           and tau by a host Lanczos run, b widened by 2%), i.e.
                           1 - lambda p(lambda) = T_2((a+b-2 lambda)/(b-a)) /
                           T_2((a+b)/(b-a)).  Symmetric positive definite for
                           any spectrum below a + b.  One more gather pass per
                           iteration, about half the iterations.  Ignored by the
                           small-batch path (float64, one workgroup, Jacobi).
                           The solution is the same to cg_rtol, which measures
                           the unpreconditioned residual either way            */
} sp_params;
enum { SP_PRECOND_JACOBI = 0, SP_PRECOND_CHEB1 = 1 };
/* There is no fixed-iteration-count mode: the CG stops on its tolerance.  The
 * CPU reference this library is checked against solves each heat step exactly
 * (sparse LU), so a fixed iteration count would compare a different
 * computation; the parity tests run the float64 solves to a tight cg_rtol
 * (1e-12 to 1e-14) instead. */

/* Fill *p with defaults for time step tau: n_steps 100, stop_tol 1e-6,
 * max_steps 10^6, energy_every = round(0.1 / tau), SP_MIXED, cg_rtol 1e-10,
 * cg_max_iter 500, inner_rtol 1e-5, max_outer 8, check_every 8, extrapolate 5,
 * precond SP_PRECOND_CHEB1. */
void sp_params_default(sp_params* p, double tau);

typedef struct {
  int64_t steps_done;      /* time steps taken (max over restarts)                   */
  int64_t cg_iters;        /* CG iterations, summed over steps (and sweeps), counting
                              the slowest column of each solve                        */
  int64_t outer_sweeps;    /* SP_MIXED refinement sweeps summed over steps            */
  int64_t col_iters_max;   /* largest per-column CG iteration total                  */
  double seconds;          /* wall time of the call                                   */
  int32_t converged;       /* 1 if every solve met its tolerance                      */
  int32_t reserved;
  double hbm_bytes;        /* algorithmic (minimum) HBM bytes of the kernels run so far,
                              by the per-element model of each kernel: the CG
                              iterations over the columns still iterating (counted on
                              the device), every other pass over all live columns (an
                              upper bound where a kernel skips converged columns), and
                              the matrix once per gathering launch; not a measurement */
} sp_stats;

/* ------------------------------------------------------------- batch solve --
 * Run a batch of restarts for prm->n_steps steps (or to the stop rule) and
 * return the final state and its energies and labels.
 * m [n_restarts], eps [n_restarts], u0 [sum m][n_vert] (host, not normalised:
 * each component is first scaled to unit L2 norm, as the random start of
 * Section 2.2 does).  Outputs, each nullable: u_out like u0; labels and
 * labels_argmax [n_restarts][n_vert] (v-partition with -1 = void, and argmax
 * of u); lambda [sum m]; s_eps, energy [n_restarts]; stats.
 * Returns SP_ENOCONV (after writing outputs) if some CG solve hit its cap. */
int sp_solve(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts, const int32_t* m,
             const double* eps, const double* u0, double* u_out, int32_t* labels,
             int32_t* labels_argmax, double* lambda, double* s_eps, double* energy,
             sp_stats* stats);

/* Device-pointer form: inputs and outputs in device memory, all work enqueued
 * on hip_stream (a hipStream_t passed as void*; NULL = default stream).  m and
 * eps stay host arrays.  With prm->check_every == 0 and n_steps > 0 the call
 * returns without waiting for the GPU; otherwise it synchronises the stream
 * when it polls convergence.  Work buffers are allocated and freed by the
 * call (freed after the stream is synchronised).  Nullable outputs as in
 * sp_solve.  Stop mode (n_steps == 0) is not available here (SP_EINVAL). */
int sp_solve_async(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts,
                   const int32_t* m, const double* eps, const double* d_u0, double* d_u_out,
                   int32_t* d_labels, int32_t* d_labels_argmax, double* d_lambda,
                   double* d_s_eps, double* d_energy, void* hip_stream);

/* Allocation-free form of sp_solve_async, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid allocation.  Same arguments, layouts and results as
 * sp_solve_async (the same kernels; the default tilings, with no tiling
 * search).  Every work buffer of the batch, the matrix K = M + tau A of this
 * tau included, is carved from one static device scratch array of
 * SP_NOALLOC_SCRATCH_BYTES (128 MiB) that each device the library runs on
 * holds until the process ends; the call allocates no device or pinned host
 * memory and creates no stream, event or graph.  The mesh's own matrices are
 * inputs (sp_mesh_create allocated them).  Limit: a batch whose buffers do not
 * fit in the scratch is rejected with SP_ENOMEM before any work is enqueued
 * (roughly n_vert x padded columns x 88 bytes in SP_MIXED with extrapolate 5,
 * x 32 bytes in SP_FP64, plus 12 x 8 x n_vert for the matrices; e.g. 16
 * columns of the 40962-vertex sphere fit in SP_MIXED).  The scratch keeps the
 * last call's contents and is cleared at the start of each call; every call
 * on one device uses the same scratch, so calls that overlap in time on one
 * device race: enqueue them on one stream (or wait for the previous call's
 * stream to pass its work) before the next call.  Host polling as in
 * sp_solve_async (prm->check_every > 0 synchronises the stream). */
#define SP_NOALLOC_SCRATCH_BYTES (128LL << 20)
int sp_solve_async_noalloc(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts,
                           const int32_t* m, const double* eps, const double* d_u0,
                           double* d_u_out, int32_t* d_labels, int32_t* d_labels_argmax,
                           double* d_lambda, double* d_s_eps, double* d_energy,
                           void* hip_stream);

/* ------------------------------------------------------------ step state --
 * A batch kept on the device between calls: stepping, single stages of
 * Algorithm 2.2, energies, checkpoint and restore.  A state is used by one
 * thread at a time. */
typedef struct sp_state sp_state;

/* u0 as in sp_solve (normalised on upload).  hip_stream as in
 * sp_solve_async (NULL: the library creates its own stream). */
int sp_state_create(const sp_mesh* mesh, const sp_params* prm, int32_t n_restarts,
                    const int32_t* m, const double* eps, const double* u0, void* hip_stream,
                    sp_state** out);
/* Advance every restart by k >= 1 full time steps (steps 1-3 of Algorithm
 * 2.2), with energies at the cadence of prm->energy_every.  Synchronous.
 * Returns SP_ENOCONV if a solve hit its cap (the steps were still taken). */
int sp_state_step(sp_state* st, int64_t k);

/* One stage of Algorithm 2.2 applied in place to the current state:
 * SP_STAGE_HEAT  u <- (M + tau A)^{-1} M u         (step 1)
 * SP_STAGE_NODE  u <- u exp(-(2 tau/eps^2)(S - u^2)) (step 2)
 * SP_STAGE_NORM  u <- u / ||u||_{L2(Gamma_h)}       (step 3)
 * The step counter is not advanced. */
enum { SP_STAGE_HEAT = 1, SP_STAGE_NODE = 2, SP_STAGE_NORM = 3 };
int sp_state_stage(sp_state* st, int32_t stage);

/* Evaluate lambda [sum m], s_eps and energy [n_restarts] of the current state
 * now (float64 on the GPU).  Nullable outputs. */
int sp_state_energy(sp_state* st, double* lambda, double* s_eps, double* energy);
/* Lagrange multipliers of the gradient flow at the current state (Section
 * 2.2, after Caffarelli and Lin): lambda_eps [sum m] (host),
 * lambda_i^eps = int |grad u_i|^2 + (2/eps^2) int (sum_{j != i} u_j^2) u_i^2,
 * the coupling integrated exactly per triangle.  Their sum is
 * sum_i lambda_i + 2 S_eps. */
int sp_state_multipliers(sp_state* st, double* lambda_eps);
/* Copy the current state out ([sum m][n_vert], host) and the step counter. */
int sp_state_read(sp_state* st, double* u, int64_t* step);
/* Overwrite the state (parity set-up, a new start) and step counter;
 * normalise != 0 scales each component to unit L2 norm first.  The heat
 * increments kept for the extrapolated start are forgotten (the next step
 * starts from u), so in SP_MIXED a run continued from sp_state_read /
 * sp_state_write agrees with the uninterrupted one only to the solver
 * tolerance; sp_state_checkpoint / sp_state_restore continue it exactly. */
int sp_state_write(sp_state* st, const double* u, int64_t step, int32_t normalise);
/* Checkpoint and resume.  *bytes receives the size of a checkpoint image of
 * the state: the state itself, the per-column solver scalars and history
 * lengths, the kept heat increments and the last normalisation's A v (SP_MIXED
 * with extrapolate > 0), the tilings the kernels used, the step counter and
 * the energy history.  The image is opaque, in the library's internal layout
 * (renumbered vertices, padded columns) and version. */
int sp_state_checkpoint_size(sp_state* st, int64_t* bytes);
/* Write the image into buf (host, caller-owned, bytes >= the size above;
 * SP_EINVAL otherwise).  Synchronous. */
int sp_state_checkpoint(sp_state* st, void* buf, int64_t bytes);
/* Replace the state by an image written by sp_state_checkpoint for the same
 * batch: same mesh size, column layout, precision, extrapolate, tau and
 * restarts (m, eps) -- SP_EINVAL otherwise, with the state unchanged.  After
 * the restore the run continues exactly (bit for bit) as the one that wrote
 * the image would have.  Not for states restricted to regions
 * (sp_region_eigen's internal use). */
int sp_state_restore(sp_state* st, const void* buf, int64_t bytes);
/* Labels of the current state, [n_restarts][n_vert] each (nullable). */
int sp_state_labels(sp_state* st, int32_t* labels, int32_t* labels_argmax);
/* Energy history of restart r: up to cap (step, E) pairs, oldest first;
 * *count receives the number available. */
int sp_state_history(sp_state* st, int32_t r, int64_t cap, int64_t* steps, double* energies,
                     int64_t* count);
int sp_state_stats(sp_state* st, sp_stats* stats);
/* Kernel timing with HIP events recorded on the state's stream around the
 * three large kernels of every CG iteration.  enable != 0 starts recording
 * (and clears the totals); enable == 0 stops. */
int sp_state_profile(sp_state* st, int32_t enable);
enum { SP_KERNEL_MATVEC = 0, SP_KERNEL_UPDATE = 1, SP_KERNEL_DIRECTION = 2,
       SP_KERNEL_PRECOND = 3 };
/* For kernel class `which` -- SP_KERNEL_MATVEC (q = (M + tau A) p and the
 * per-column p.q), SP_KERNEL_UPDATE (x += alpha p, r -= alpha q, z = D r and
 * the per-column r.z, r.r; without z under SP_PRECOND_CHEB1),
 * SP_KERNEL_DIRECTION (p = z + beta p) or SP_KERNEL_PRECOND (z = P r and
 * the per-column r.z, SP_PRECOND_CHEB1 only) -- the launch count and summed
 * duration (ms) since profiling was enabled, and the algorithmic (minimum)
 * HBM bytes of one launch over the live columns: float32 vectors in
 * SP_MIXED, float64 in SP_FP64. */
int sp_state_kernel_time(sp_state* st, int32_t which, int64_t* launches, double* total_ms,
                         double* bytes_per_launch);
/* Tiling the state's matrix-product kernels use (the autotuned one): lanes
 * per vertex row (each lane owns 4 columns), rows per chunk, workgroups per
 * XCD row range, and the autotuner's measured time (us) of one matrix product
 * with it (0 when the default tiling was used: small problems or
 * SEGPART_AUTOTUNE=0).  The streaming vector kernels always use the widest
 * tiling.  Nullable outputs. */
int sp_state_tiling(sp_state* st, int32_t* lanes_per_row, int32_t* rows_per_chunk,
                    int32_t* groups_per_xcd, double* matvec_us);
void sp_state_destroy(sp_state* st);

/* --------------------------------------------------------------- serving --
 * A request loop on one GPU.  Requests (a mesh, parameters, restarts and
 * u0) are queued; a scheduler thread admits them into column slots of
 * per-(mesh, tau, precision) batches while the HBM budget allows, advances
 * every resident batch one time step per round, and retires requests as they
 * finish, so requests that arrive while others run join the running batch
 * (continuous batching).  Thread-safe. */
typedef struct sp_server sp_server;

/* hbm_budget_bytes: cap on device memory for request state (matrices of
 * resident meshes are counted too).  max_batch_columns: column capacity of
 * one batch (0 = default 4096). */
int sp_server_create(int64_t hbm_budget_bytes, int32_t max_batch_columns, sp_server** out);
/* Queue a request (inputs copied; prm->n_steps must be > 0).  Returns at once
 * with a ticket.  SP_ENOMEM if the request alone exceeds the budget. */
int sp_server_submit(sp_server* srv, const sp_mesh* mesh, const sp_params* prm,
                     int32_t n_restarts, const int32_t* m, const double* eps, const double* u0,
                     int64_t* ticket);
/* *done = 1 once the request finished (results ready to fetch). */
int sp_server_poll(sp_server* srv, int64_t ticket, int32_t* done);
/* Block until the request finished or timeout_s elapsed (SP_EAGAIN). */
int sp_server_wait(sp_server* srv, int64_t ticket, double timeout_s);
/* Copy out and release a finished request's results (nullable outputs, layouts
 * as in sp_solve) and its latency (finish - submit, seconds).  SP_EAGAIN if
 * not finished, SP_ENOTFOUND for an unknown ticket. */
int sp_server_fetch(sp_server* srv, int64_t ticket, double* u_out, int32_t* labels,
                    double* lambda, double* s_eps, double* energy, double* latency_s);
/* Cost of a finished request (before sp_server_fetch): CG iterations summed
 * over its components (inner iterations in SP_MIXED) and the time steps it
 * took.  SP_EAGAIN if not finished, SP_ENOTFOUND for an unknown or fetched
 * ticket.  Nullable outputs. */
int sp_server_request_stats(sp_server* srv, int64_t ticket, int64_t* col_iters, int64_t* steps);
/* Latency percentiles over finished requests, achieved component-DOF updates
 * per second since the first submit, and the number of finished requests. */
int sp_server_stats(sp_server* srv, double* p50_s, double* p99_s, double* cdof_per_s,
                    int64_t* completed);
/* Stops the scheduler (abandoning unfinished requests) and frees everything. */
void sp_server_destroy(sp_server* srv);

/* ------------------------------------------------------------ continuation --
 * The convergence study in eps of Section 3.1 (table tab:u-eps): a minimiser
 * is computed on a coarse mesh at a large eps; then, level after level, the
 * mesh is refined, tau and eps shrink, and the previous minimiser is the new
 * initial condition, each level running until the stopping rule of Section
 * 2.2 holds. */

/* Moves the n points xyz [n][3] (host, in place) onto the surface. */
typedef void (*sp_project_fn)(double* xyz, int64_t n, void* ctx);

/* Refinement of Section 3.1: every triangle split into four at its edge
 * midpoints (two of the paper's bisections, which halve h).  The fine mesh
 * keeps the coarse vertices 0..n-1 (caller numbering) and appends one vertex
 * per edge: vertex n + j is the midpoint of the j-th edge (a, b), a < b, in
 * lexicographic order of (a, b), moved onto the surface by project (NULL:
 * left at the midpoint; project is called once, on all new vertices, before
 * this returns).  Coarse triangle t = (a, b, c) with midpoints ab, bc, ca
 * becomes fine triangles 4t..4t+3 = (a, ab, ca), (b, bc, ab), (c, ca, bc),
 * (ab, bc, ca).  *fine is a new mesh (sp_mesh_destroy) that remembers its
 * parents.  Errors as sp_mesh_create (the projected points are validated). */
int sp_mesh_refine(const sp_mesh* coarse, sp_project_fn project, void* ctx, sp_mesh** fine);
/* Parents of a refined mesh's new vertices: parents [n_fine - n_coarse][2]
 * (host), the edge (a, b) of each new vertex; *n_coarse (nullable) receives
 * the coarse vertex count.  SP_EINVAL if the mesh was not made by
 * sp_mesh_refine. */
int sp_mesh_parents(const sp_mesh* fine, int32_t* parents, int64_t* n_coarse);
/* The coarse state carried to a refined mesh as the P1 function it is: a
 * coarse vertex keeps its value, new vertex n + j takes the mean of its two
 * parents' values (the coarse function at the edge midpoint).  u_coarse
 * [n_cols][n_coarse] -> u_fine [n_cols][n_fine], host arrays; the work runs on
 * the GPU. */
int sp_prolong(const sp_mesh* fine, int32_t n_cols, const double* u_coarse, double* u_fine);

typedef struct {
  double eps;       /* this level's eps                                         */
  double tau;       /* this level's time step; the energy is checked every
                       M_tau = round(0.1 / tau) steps (Section 2.2)             */
  int32_t refine;   /* 1: refine the mesh (sp_mesh_refine) before this level and
                       carry the state over (sp_prolong); must be 0 on level 0 */
  int32_t reserved;
} sp_level;

typedef struct {
  int64_t n_vert;   /* vertices of the level's mesh                             */
  int64_t steps;    /* time steps the restart took on the level                 */
  double energy;    /* E = sum lambda + S_eps at the level's final state        */
  double s_eps;     /* S_eps of equation (Seps-u) there                         */
  double seconds;   /* wall time of the level (refinement included)             */
  int32_t converged;  /* 1 if every linear solve of the level met its tolerance */
  int32_t reserved;
} sp_level_result;

/* Level loop for n_restarts independent restarts of m components each, run
 * as one batch (the paper starts from random states; several starts and the
 * best final energy guard against local minima).  prm supplies the
 * precision, the CG settings, stop_tol and max_steps; its tau and
 * energy_every are replaced per level (tau = levels[l].tau, energy_every =
 * M_tau), eps = levels[l].eps for every restart; each restart stops on its
 * own when the stopping rule holds for it (the batch level ends when all have
 * stopped); with prm->n_steps > 0 every level runs exactly that many steps.
 * u0 [n_restarts * m][n_vert of mesh0] (host, restart-major, normalised on
 * upload like sp_solve's).  Outputs (host): results [n_levels][n_restarts]
 * (steps, energy and s_eps per restart; n_vert, seconds and converged per
 * level, repeated); lambda [n_levels][n_restarts * m] (nullable);
 * *final_mesh (nullable) receives the last level's mesh as a new handle when
 * any level refined, else NULL; u_final [n_restarts * m][n_vert of the last
 * level] (nullable; the caller sizes it, e.g. n_vert grows to
 * n + (3/2) n_tri per refinement of a closed surface).  project as in
 * sp_mesh_refine.  on_level (nullable) is called on the calling thread after
 * each level with the level index and its n_restarts results (progress of a
 * long study).  Returns SP_ENOCONV (after writing outputs) if some linear
 * solve hit its cap. */
typedef void (*sp_level_fn)(int32_t level, const sp_level_result* results, void* ctx);
int sp_continue(const sp_mesh* mesh0, const sp_params* prm, int32_t n_restarts, int32_t m,
                const double* u0, int32_t n_levels, const sp_level* levels,
                sp_project_fn project, void* ctx, sp_level_result* results, double* lambda,
                sp_mesh** final_mesh, double* u_final, sp_level_fn on_level,
                void* level_ctx);

/* ------------------------------------------------------------ partitions --
 * Post-processing of a computed partition given as vertex labels (e.g. the
 * argmax labels of sp_solve): region i of restart r is the set of vertices
 * labelled i; other values (-1, the void of equation (vi)) belong to no
 * region.  labels [n_restarts][n_vert] int32, caller numbering. */

/* First Dirichlet eigenvalue of every region: the smallest eigenvalue of
 * A x = lambda M x over the P1 functions that vanish at every vertex outside
 * the region (the partition problem's energy, Problem 1.1, is their sum; on
 * the sphere the lunes of the Y-partition give 15/4 each).  Computed by
 * inverse iteration u <- (M + shift A)^{-1} M u restricted to the region
 * (float64 Jacobi-CG to relative residual 1e-12 each), normalised, until the
 * Rayleigh quotient of every region changes by at most tol (relative)
 * between iterations; each iteration contracts the error by about
 * (1 + shift lambda_1) / (1 + shift lambda_2).  m [n_restarts]; u0 [sum m]
 * [n_vert] start vectors (nullable: 1 on the region; the partition's own
 * components are good starts), restricted to the regions before use.
 * Outputs (host): lambda [sum m] (NaN for an empty region); u_out [sum m]
 * [n_vert] (nullable) the eigenvectors, unit L2 norm, zero outside;
 * iterations (nullable).  shift > 0, tol > 0, max_iter >= 1.
 * interior = 0: the functions vanish at the vertices outside the region, so
 * they reach half an element beyond it and, on labels that cover the surface,
 * the value lies below the region's own (O(h)); interior = 1: the region's
 * boundary vertices (those with a mesh neighbour labelled otherwise) are
 * left out too and the value lies above.  The two bracket the eigenvalue of
 * the region the labels describe.  Returns SP_ENOCONV (after writing the
 * outputs) if max_iter iterations did not meet tol. */
int sp_region_eigen(const sp_mesh* mesh, int32_t n_restarts, const int32_t* m,
                    const int32_t* labels, int32_t interior, const double* u0, double shift,
                    double tol, int32_t max_iter, double* lambda, double* u_out,
                    int32_t* iterations);

/* Which regions touch: adjacency [sum_r m_r^2] (host) holds, per restart in
 * order, an m_r x m_r block with 1 where a vertex of region i and a vertex of
 * region j (i != j) share a mesh edge; sides [sum m] (nullable) counts each
 * region's neighbours (its sides, one arc per neighbour).  With triple
 * junctions only, the counts n_k of k-sided regions satisfy the identity
 * derived from Euler's formula (equation gauss-bonnet),
 * 4 n_2 + 3 n_3 + 2 n_4 + n_5 = 6 chi + sum_{k>=7} (k - 6) n_k.  m_r <= 4096 and
 * sum_r m_r^2 < 2^31 (SP_EINVAL otherwise). */
int sp_region_graph(const sp_mesh* mesh, int32_t n_restarts, const int32_t* m,
                    const int32_t* labels, uint8_t* adjacency, int32_t* sides);

#ifdef __cplusplus
}
#endif
#endif /* SEGPART_H */
