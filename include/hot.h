/*
 * hot.h -- C ABI of the MI355X implicit MPM step of "Hierarchical Optimization
 * Time Integration for CFL-rate MPM Stepping" (HOT, arXiv 1911.07913).
 *
 * One call of hot_step advances a particle scene by one implicit-Euler MPM
 * step (Sec. 3.1): APIC particle-to-grid transfer, minimisation of the
 * incremental potential of Eq. 1 over grid velocity increments by HOT
 * (Alg. HOT: L-BFGS whose initial inverse Hessian is one multigrid V-cycle of
 * Alg. V-cycle over the node-embedding Galerkin hierarchy of Sec. 4), then
 * grid-to-particle transfer, deformation update and advection.
 *
 * Conventions for every function below:
 *   - all functions are extern "C", never throw, and return hot_status
 *     (0 = OK, > 0 = warning with the step completed, < 0 = error);
 *   - host arrays are owned by the caller; they are copied in at
 *     hot_init_scene and copied out by hot_read_particles;
 *   - a scene owns its device memory, obtained through the hot_allocator
 *     given at creation (NULL: hipMalloc/hipFree) and released by
 *     hot_destroy_scene;
 *   - all device work of a scene is issued on the HIP stream given at
 *     creation (NULL: a non-blocking stream created and owned by the scene);
 *   - SI units; particle arrays are row-major, n rows, in the caller's order;
 *   - a scene is not thread-safe; distinct scenes may be used from distinct
 *     host threads;
 *   - on error, hot_last_error() returns a message (thread-local, valid until
 *     the next call on the same thread).
 */
#ifndef HOT_H_
#define HOT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HOT_OK = 0,
  HOT_W_NOT_CONVERGED = 1,  /* step done; CN tolerance not met (iteration cap or
                               line search exhausted) */
  HOT_E_INVALID = -1,       /* bad argument; nothing changed */
  HOT_E_NOMEM = -2,         /* device allocation failed; nothing changed */
  HOT_E_DEVICE = -3,        /* HIP runtime error */
  HOT_E_NONFINITE = -4,     /* non-finite energy/gradient: particle state rolled back */
  HOT_E_BUSY = -5
} hot_status;

/* Elastic energy density (Sec. 7.1 uses fixed-corotated for every scene). */
typedef enum { HOT_FCR = 0, HOT_NEOHOOKEAN = 1 } hot_model;

/* Precision policy: HOT_FP64 runs every kernel in FP64.  HOT_MIXED runs the
 * V-cycle (smoothing, SpMV, coarse solve) in FP32 over BF16-stored Hessian
 * blocks with FP32 accumulation; energy, line search, gradient, CN test and
 * the L-BFGS history stay FP64. */
typedef enum { HOT_FP64 = 0, HOT_MIXED = 1 } hot_precision;

/* Smoother of the V-cycle's non-coarsest levels (Alg. V-cycle).
 * HOT_SMOOTH_L1_JACOBI (0, the default): l1 block-Jacobi,
 *   u += D~^{-1} (b - H u), D~ the 3x3 diagonal block plus the l1 sums of the
 *   rest of the row on its diagonal; one fully parallel pass per sweep.
 * HOT_SMOOTH_SGS (1): the paper's coloured symmetric block Gauss-Seidel
 *   (Sec. 5.3, Sec. 8): nodes coloured by grid coordinate mod 3 per axis (27
 *   colours), a forward pass over colours 0..26 then a backward pass 26..0,
 *   each node taking u_i = H_ii^{-1} (b_i - sum_{j != i} H_ij u_j); costlier
 *   per cycle, far fewer L-BFGS iterations on stiff scenes.
 * smoother_sweeps counts sweeps (Jacobi) or forward-backward pairs (SGS). */
typedef enum { HOT_SMOOTH_L1_JACOBI = 0, HOT_SMOOTH_SGS = 1 } hot_smoother;

/* Solver of the step's minimisation.
 * HOT_SOLVER_HOT (0, the default): Alg. HOT, L-BFGS whose initial inverse
 *   Hessian is one V-cycle of the start-of-step Galerkin hierarchy.
 * HOT_SOLVER_PN_PCG (1): the paper's baseline of Alg. 1, projected Newton
 *   whose linear systems H(dv) p = -g are solved by CG preconditioned with
 *   the scalar diagonal, to the adaptive relative tolerance
 *   k = min(1/2, sqrt(max(sqrt(r0^T M r0), tau))) of Sec. 5.3 (tau = tol;
 *   at most 10,000 CG iterations); mg_levels is ignored.
 * HOT_SOLVER_PN_MGPCG (2): the same with one V-cycle (smoother and levels as
 *   set) as the preconditioner, the hierarchy rebuilt from each Newton
 *   iteration's Hessian (Sec. 5.1).
 * For the Newton solvers, hot_step_stats.iters counts Newton iterations and
 * cg_iters_total the CG iterations of their linear solves. */
typedef enum { HOT_SOLVER_HOT = 0, HOT_SOLVER_PN_PCG = 1, HOT_SOLVER_PN_MGPCG = 2 } hot_solver;

typedef struct {
  int32_t model;        /* hot_model */
  double E;             /* Young's modulus, Pa, > 0 */
  double nu;            /* Poisson ratio, in (-1, 0.5) */
  double density;       /* kg/m^3, > 0 (particle mass = density * vol0) */
  double yield_stress;  /* von Mises yield stress, Pa; 0 = purely elastic.
                           Applied once per step after the solve (lagged
                           plasticity, Sec. 2 and Sec. 8). */
  double snow_clamp[2]; /* snow-type plastic flow (Sec. 7, table of material
                           parameters, after Stomakhin et al. 2013): after
                           each step the singular values of F are clamped
                           into [snow_clamp[0], snow_clamp[1]] (the paper
                           uses [0.99, 1.001]); {0, 0} = none.  Requires
                           0 < lo <= 1 <= hi and yield_stress = 0. */
} hot_material;

/* Dirichlet boundary conditions, resolved by projection at every level
 * (Sec. 4.1).  All are sticky: every velocity component is prescribed on the
 * grid nodes they select.  Later entries override earlier ones. */
typedef enum {
  HOT_BC_BOX_WALLS = 0, /* p[0] = thickness t in cells: nodes with index <= t or
                           >= grid_cells - t on any axis are held at rest */
  HOT_BC_GRIP = 1,      /* p[0..2] box min, p[3..5] box max (world, inclusive),
                           p[6..8] point on the axis, p[9..11] axis direction,
                           p[12] angular speed w (rad/s): nodes in the box move
                           with w * (a x (x - c)) */
  HOT_BC_SPHERE = 2     /* p[0..2] centre at t = 0, p[3] radius, p[4..6]
                           velocity: nodes inside the sphere at the end of the
                           step move with the sphere */
} hot_bc_kind;

typedef struct {
  int32_t kind;         /* hot_bc_kind */
  double p[16];
} hot_bc;

/* Device allocator hook (e.g. a framework's caching allocator).  alloc returns
 * device memory of at least `bytes` bytes, aligned to 256 bytes (as hipMalloc's
 * is), or NULL; free releases it.  A misaligned block is freed again and the
 * call that needed it fails with HOT_E_INVALID. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} hot_allocator;

/* Problem statement (Sec. 3.1, Sec. 7.1 simulation settings). */
typedef struct {
  double dx;               /* grid spacing, m, > 0 */
  int32_t grid_cells[3];   /* cells per axis; nodes sit at origin + i*dx,
                              i = 0..grid_cells */
  double origin[3];
  double gravity[3];       /* m/s^2, applied to the grid velocity before the solve */
  double cfl;              /* time-step rule dt = min(max_dt, cfl*dx/v_max), 0.6 */
  double max_dt;           /* 1/FPS, e.g. 1/24 */
  double tol;              /* CN tolerance eps of Sec. 5.2: stop when
                              ||g_hat|| <= eps * sqrt(#active fine nodes) */
  int32_t lbfgs_history;   /* window w of Alg. HOT (paper default 8) */
  int32_t mg_levels;       /* levels M of the hierarchy (>= 1) */
  int32_t max_iters;       /* L-BFGS iteration cap (e.g. 500) */
  int32_t smoother_sweeps; /* smoothing sweeps per level and direction (1) */
  int32_t precision;       /* hot_precision */
  int32_t smoother;        /* hot_smoother */
  int32_t graph;           /* 1: each step's V-cycles run as one captured HIP
                              graph (captured at the step's first cycle, then
                              launched once per cycle; same kernels and
                              results as 0, fewer launches from the host).
                              Ignored while kernel tracing is on. */
  int32_t solver;          /* hot_solver */
} hot_params;

typedef struct {
  double dt;               /* time step used */
  double t;                /* scene time after the step */
  double E0, E;            /* incremental potential at dv = 0 and at the end */
  double cn0, cn;          /* CN-scaled gradient norm at start and end */
  double cn_tol;           /* eps * sqrt(n) */
  int32_t iters;           /* L-BFGS iterations (line searches performed) */
  int32_t backtracks;      /* total step-length halvings */
  int32_t cg_iters_total;  /* coarsest-level PCG iterations over all V-cycles */
  int32_t converged;       /* 1 if the CN test passed */
  int32_t fallbacks;       /* non-descent directions replaced */
  int32_t skipped_pairs;   /* secant pairs rejected by the curvature test */
  int32_t n_nodes;         /* active fine nodes */
  int32_t n_levels;
  float ms_prepare;        /* binning + grid + P2G */
  float ms_hierarchy;      /* Hessian assembly + Galerkin coarsening */
  float ms_solve;          /* quasi-Newton loop */
  float ms_g2p;            /* G2P + deformation update + advection */
} hot_step_stats;

typedef struct hot_scene hot_scene;

/* Upper bound of the device bytes hot_init_scene would allocate for this
 * particle set (positions x[n][3], host).  Used for admission by HBM
 * footprint. */
hot_status hot_scene_footprint(const hot_params* params, int64_t n, const double* x,
                               size_t* bytes_out);

/* Create a scene from host particle arrays (copied).  x, v: [n][3]; F, C:
 * [n][9] row-major (F NULL = identity, C NULL = zero; C is the APIC affine
 * velocity matrix); vol0: [n] initial volumes; mat_id: [n] indices into mats.
 * Particles must lie in [origin + 2dx, origin + (grid_cells - 3)dx] and all
 * values must be finite; otherwise HOT_E_INVALID. */
hot_status hot_init_scene(const hot_params* params, int64_t n, const double* x, const double* v,
                          const double* F, const double* C, const double* vol0,
                          const int32_t* mat_id, const hot_material* mats, int32_t n_mats,
                          const hot_bc* bcs, int32_t n_bcs, const hot_allocator* alloc,
                          void* hip_stream, hot_scene** out);

/* Advance one implicit step.  dt <= 0 selects the CFL rule above.  Either
 * completes the step (HOT_OK or HOT_W_NOT_CONVERGED) or leaves the particle
 * state unchanged (errors).  stats may be NULL. */
hot_status hot_step(hot_scene* scene, double dt, hot_step_stats* stats);

/* Copy particle state back to host arrays in the caller's original order.
 * n must equal the scene's particle count; F and C may be NULL. */
hot_status hot_read_particles(const hot_scene* scene, int64_t n, double* x, double* v,
                              double* F, double* C);

/* Particle count and current scene time. */
hot_status hot_scene_info(const hot_scene* scene, int64_t* n, double* t);

void hot_destroy_scene(hot_scene* scene);
const char* hot_last_error(void);

/* Device bytes the scene holds now and the working-size estimate made at
 * init (the hot_scene_footprint figure). */
hot_status hot_scene_memory(const hot_scene* scene, size_t* live_bytes, size_t* estimate_bytes);

/* ---- stepping without device allocation ----------------------------------
 * For callers that cannot allocate device memory where they step: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and status codes as hot_step (bit-identical
 * output), but the call makes no hipMalloc or hipFree and calls no
 * allocating library routine:
 *   - the scene's own buffers (particles, grids, hierarchy, solver vectors)
 *     must already be large enough, as sized by hot_init_scene and earlier
 *     hot_step calls (which keep 25% headroom).  A step that would need one
 *     to grow (a scene's first step, or more active nodes than any earlier
 *     step had) returns HOT_E_NOMEM before writing past it; the particle
 *     state and scene time are unchanged, and a hot_step call sizes the
 *     buffers;
 *   - the per-call scratch (reduction partial sums, the scalar block, an
 *     error flag, the coarsest-level PCG vectors, grid barrier and
 *     iteration counts) comes from one fixed 1 MiB device array per GPU,
 *     held from the first call on that GPU until the process ends.  A step
 *     whose coarsest level needs more (above about 6,700 rows), or whose
 *     max_iters needs more PCG counters than fit, is refused with
 *     HOT_E_INVALID and a message naming the size;
 *   - every call on one GPU shares that array, which keeps the last call's
 *     contents; each call writes every scratch value before reading it.
 *     Calls that overlap in time on one GPU (several host threads, or
 *     several streams) race on the array and must be serialised by the
 *     caller;
 *   - kernel tracing (hot_profile_enable) must be off: HOT_E_INVALID;
 *   - with hot_params.graph set, the V-cycles run eagerly in this call
 *     (same kernels and results; instantiating a graph may allocate). */
hot_status hot_step_noalloc(hot_scene* scene, double dt, hot_step_stats* stats);

/* ---- serving: continuous batching of independent scenes ------------------
 * Steps of many independent scenes (the paper's per-frame solve applied to
 * a stream of requests) share one GPU.  A batch owns an HBM budget and
 * max_slots slots (1 to 64; HOT_E_INVALID otherwise), each served by one
 * host thread.  Any number of scenes may step at once, in batches or on the
 * caller's own threads and streams: a coarsest-level solve that uses grid
 * barriers takes at most 1/16 of the device's resident work-groups, and the
 * library lets at most 16 of them run at once per device (a step's solve
 * holds one of 16 tickets and waits for one when all are taken).  hot_batch_add admits a
 * scene with a number of steps to run when a slot is free and the larger of
 * the scene's live bytes and its footprint estimate fits in the budget that
 * resident scenes leave; otherwise it returns HOT_E_NOMEM and the caller
 * defers the request.  An admitted scene starts at once and runs its steps
 * back to back (dt from the CFL rule) on its own stream from its slot's
 * thread, so the device interleaves the kernels of all resident scenes.  A
 * scene's arithmetic does not depend on what else is resident.
 * A scene's slot is free again as soon as its last step ends; its budget
 * stays reserved until hot_batch_poll hands it out (all steps done, or
 * stopped by an error; waiting up to wait_ms for one), since its device
 * memory lives until the caller, who still owns each hot_scene, destroys it.  While a scene is
 * resident the caller must not use it.  Times are seconds on a steady clock
 * started by hot_batch_create.  hot_batch_destroy lets each resident scene
 * finish its current step, then stops the slot threads. */
#define HOT_BATCH_MAX_STEPS 64
typedef struct {
  int64_t tag;
  int32_t status;     /* worst step status (HOT_OK, a warning, or the error that stopped it) */
  int32_t steps;      /* steps completed */
  int32_t iters;      /* quasi-Newton iterations summed over the steps */
  int32_t reserved;
  double t_admit;     /* admission time */
  double t_step_end[HOT_BATCH_MAX_STEPS]; /* completion time of each of the first 64 steps */
  char message[160];  /* error text when status < 0 */
  hot_scene* scene;   /* the request's scene (hot_batch_add: the caller's; hot_batch_submit:
                         the one the batch created, now owned by the caller, who reads and
                         destroys it; NULL if its creation failed) */
  double t_created;   /* when the scene was ready to step (hot_batch_submit: after its
                         creation on the slot thread; hot_batch_add: t_admit) */
} hot_batch_result;

/* The arguments of hot_init_scene, for a request whose scene the batch
 * creates (hot_batch_submit). */
typedef struct {
  const hot_params* params;
  int64_t n;
  const double* x;
  const double* v;
  const double* F;    /* nullable */
  const double* C;    /* nullable */
  const double* vol0;
  const int32_t* mat_id;
  const hot_material* mats;
  int32_t n_mats;
  const hot_bc* bcs;
  int32_t n_bcs;
} hot_scene_desc;
typedef struct hot_batch hot_batch;
hot_status hot_batch_create(size_t hbm_budget_bytes, int32_t max_slots, hot_batch** out);
hot_status hot_batch_capacity(hot_batch* batch, size_t* free_bytes, int32_t* free_slots);
hot_status hot_batch_add(hot_batch* batch, hot_scene* scene, int32_t n_steps, int64_t tag);
/* Admit a request as a scene description: the same admission rule, with the
 * reservation taken from hot_scene_footprint, but the slot's thread creates
 * the scene itself (hot_init_scene, validation included) with device memory
 * from the batch's pool and a stream of its own, then runs its steps.  The
 * admission path does no device work.  The arrays desc points to must stay
 * valid until the request's result is collected (*desc and *desc->params are
 * copied).  The result carries the scene; the caller reads it and destroys it
 * (its buffers return to the pool) before destroying the batch.  A scene that
 * fails validation comes back with the error in status and message. */
hot_status hot_batch_submit(hot_batch* batch, const hot_scene_desc* desc, int32_t n_steps,
                            int64_t tag);
hot_status hot_batch_poll(hot_batch* batch, hot_batch_result* results, int32_t cap,
                          int32_t* n_done, int32_t* n_resident, int32_t wait_ms);
double hot_batch_clock(const hot_batch* batch);
void hot_batch_destroy(hot_batch* batch);

/* ---- tracing: HIP-event timing of individual kernels ---------------------
 * When enabled, the library records a pair of HIP events on the scene's
 * stream around every launch of the kernels below and accumulates, per
 * kernel, the summed launch durations, the launch count and the algorithmic
 * bytes those launches had to move (structural matrix blocks plus the node
 * vectors each launch reads and writes once; padding and re-reads are not
 * counted).  Enabling resets the counters. */
enum {
  HOT_PROF_SMOOTH0 = 0,    /* level-0 smoothing sweep (fused SpMV + update) */
  HOT_PROF_RESIDUAL0 = 1,  /* level-0 residual b - H u */
  HOT_PROF_ASSEMBLE = 2,   /* level-0 Hessian assembly */
  HOT_PROF_RAP0 = 3,       /* Galerkin product level 0 -> 1 */
  HOT_PROF_EVAL = 4,       /* per-particle energy / stress evaluation */
  HOT_PROF_GRAD = 5,       /* gradient gather */
  HOT_PROF_PHESS = 6,      /* per-particle projected stress derivative */
  HOT_PROF_SGS0 = 7,       /* level-0 symmetric Gauss-Seidel smoothing (53 colour passes) */
  HOT_PROF_VCYCLE = 8,     /* one whole V-cycle: every level's smoothing, residual and
                              transfers, the coarsest solve, the precision conversions */
  HOT_PROF_COUNT = 9
};
hot_status hot_profile_enable(hot_scene* scene, int32_t enable);
hot_status hot_profile_read(const hot_scene* scene, int32_t kernel, double* total_ms,
                            int64_t* launches, double* total_bytes);

/* ---- test hooks (parity checks against an independent implementation) --- */
enum {
  HOT_DBG_PERM = 1,        /* int32 [n]: original index of each particle in binned order */
  HOT_DBG_LEVEL_NODES = 10,/* int32 [n_m]: linear node index (x fastest) at level m */
  HOT_DBG_LEVEL_PATTERN = 11, /* uint32 [n_m][4]: bit s set if block slot s is
                                structurally present (s = dx+2 + 5(dy+2) + 25(dz+2)) */
  HOT_DBG_LEVEL_MATRIX = 12,  /* double [n_m][125][3][3] block rows (FP64 copy) */
  HOT_DBG_LEVEL_FREE = 13,    /* uint8 [n_m][3]: 1 = free DOF, 0 = constrained */
  HOT_DBG_LEVEL_MATRIX_BF16 = 14, /* uint16 [n_m][125][3][3] BF16 bit patterns of the
                                 blocks the mixed V-cycle reads (HOT_MIXED only) */
  HOT_DBG_LEVEL_COLOR_ROWS = 15, /* int32 [n_m]: rows of level m ordered by
                                    Gauss-Seidel colour, ascending within a
                                    colour (HOT_SMOOTH_SGS, m < levels - 1) */
  HOT_DBG_NODE_MASS = 20,     /* double [n_0] */
  HOT_DBG_NODE_VSTAR = 21,    /* double [n_0][3]: v after gravity and BCs */
  HOT_DBG_NODE_XI = 22,       /* double [n_0]: CN stiffness field */
  HOT_DBG_NODE_FIXED = 23,    /* int32 [n_0] */
  HOT_DBG_DV = 30,            /* double [n_0][3]: last solve's dv */
  HOT_DBG_LOG_INT = 40,       /* int32 [iters][4]: halvings (-1 failed), pair skipped,
                                 fallback, coarse-PCG iterations of the iteration's V-cycle */
  HOT_DBG_LOG_CN = 41,        /* double [iters + 1] */
  HOT_DBG_COUNTS = 50         /* int32 [16]: n, n_levels, nodes per level... */
};
/* Copy an internal array (see HOT_DBG_*) of level `level` to host memory.
 * *needed receives the byte size; dst may be NULL to query it. */
hot_status hot_debug_read(const hot_scene* scene, int32_t what, int32_t level, void* dst,
                          size_t bytes, size_t* needed);
/* Run the step up to and including the Galerkin hierarchy (no solve, no G2P,
 * particle state unchanged) with time step dt (<= 0: CFL rule). */
hot_status hot_debug_prepare(hot_scene* scene, double dt);
/* Process-wide settings for tests, applied to launches issued after the call.
 * HOT_SET_MULTIROW_MIN: level size (rows) from which the smoothing and
 *   residual sweeps of the V-cycle run as work-groups over runs of 16
 *   consecutive rows with the iterate window staged in LDS, instead of one
 *   row per wave (default 16384 rows; a negative value restores the default).
 *   Both forms compute every row with the same per-lane arithmetic, so a test
 *   can run either one on any level.
 * *previous (nullable) receives the old value; an unknown key is
 * HOT_E_INVALID. */
enum { HOT_SET_MULTIROW_MIN = 1 };
hot_status hot_debug_set(int32_t key, int64_t value, int64_t* previous);
/* After hot_debug_prepare: apply an operator to a host vector of n_0*3
 * doubles.  op 0: one V-cycle; op 1: gradient at dv = in; op 2: energy at
 * dv = in (out[0]); op 3: level-0 matrix product. */
hot_status hot_debug_apply(hot_scene* scene, int32_t op, const double* in, double* out);

#ifdef __cplusplus
}
#endif
#endif /* HOT_H_ */
