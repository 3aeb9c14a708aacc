/*
 * solid_lbm.h -- C ABI of the MI355X solid lattice-Boltzmann library.
 *
 * The library solves the steady linear-elastic state of a D2Q8 moment-space
 * lattice-Boltzmann scheme (paper Sec. "LBM scheme for solids": eq. moments to
 * eq. local_stream, appendix matrix M and relaxation-time table) to a
 * pseudo-time fixed point (eq. primal_fixed_point), evaluates the discrete
 * objective (eq. node_J, eq. discrete_J), runs the discrete adjoint fixed-point
 * iteration (eq. adjoint_streaming, eq. adjoint_collision, eq.
 * adjoint_iteration, eq. adjoint_init; Algorithm "ALBM") and assembles the
 * gradient of the objective w.r.t. the control (eq. optimality).
 *
 * Conventions
 *  - Every number is IEEE double.  Fields are SoA, component-major, x fastest:
 *      a[c * nx * ny + iy * nx + ix].
 *    Per-link fields use c * 8 + q as the component (q in the direction order
 *    Q of eq. direction_order: (1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1)).
 *  - Units: diffusive scaling dt = dx^2, kappa = 1, so lattice moduli equal
 *    the physical ones; the forcing is g = dx^2 F (eq. forcing); stresses and
 *    tractions in lattice units are dx times the physical ones.
 *  - Pointers marked "host" must be host memory.  Pointers passed with
 *    ptr_kind = SLBM_PTR_DEVICE must be device memory of the context's GPU
 *    (e.g. a torch CUDA tensor's data_ptr()); SLBM_PTR_HOST means host memory.
 *  - Ownership: the library copies every input it needs during the call and
 *    never keeps a caller pointer; outputs are written into caller memory.
 *  - Errors: negative return codes leave the context unchanged and set the
 *    message returned by solid_lbm_last_error().  A positive code (only
 *    SLBM_NOT_CONVERGED) means the outputs were written but the solve stopped
 *    at max_steps before the residual reached tol.
 *  - Threading: one context per host thread at a time; all work of a context
 *    is queued on its stream (problem.stream, NULL = the default stream) and
 *    every call returns after that stream has drained.
 */
#ifndef SOLID_LBM_H
#define SOLID_LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SLBM_OK = 0,
    SLBM_NOT_CONVERGED = 1,
    SLBM_EINVAL = -1,     /* bad sizes, moduli, flags, or a plate touching the box edge */
    SLBM_ENOMEM = -2,     /* device allocation failed */
    SLBM_EHIP = -3,       /* a HIP runtime call failed (message holds the HIP error) */
    SLBM_ESTATE = -4,     /* call order: adjoint before a converged primal, etc. */
    SLBM_ENONFINITE = -5  /* non-finite control or input field */
};

/* Domain kinds: periodic torus (Sec. "Problem formulation": Omega = T^2) or a
 * plate given as a node mask inside a box, with Dirichlet / Neumann links. */
enum { SLBM_PERIODIC = 0, SLBM_MASKED = 1 };

/* Control kinds (Table "overview_cases" and the controls of the benchmarks):
 *  FORCE_MODES   F = sum_i a_i B_i(x)           control: n_modes doubles
 *  FORCE_NODAL   F(x_n) = P(alpha)(x_n)         control: 2 * nx * ny doubles
 *                (P = eq. zero_mean_projection when zero_mean_projection != 0)
 *  E_NODAL       E(x_n) = alpha(x_n)            control: nx * ny doubles
 *  E_SCALAR_SQ   E = alpha^2 (eq. E_substitution) control: 1 double          */
enum { SLBM_CTRL_FORCE_MODES = 0, SLBM_CTRL_FORCE_NODAL = 1, SLBM_CTRL_E_NODAL = 2,
       SLBM_CTRL_E_SCALAR_SQ = 3 };

enum { SLBM_PTR_HOST = 0, SLBM_PTR_DEVICE = 1 };
enum { SLBM_CONV_KLAG = 0, SLBM_CONV_CV = 1 };

/* Link kinds of link_bc. */
enum { SLBM_LINK_INTERIOR = 0, SLBM_LINK_DIRICHLET = 1, SLBM_LINK_NEUMANN = 2 };

/* Fields readable with solid_lbm_get_field (sizes in doubles). */
enum {
    SLBM_FIELD_DISP = 0,      /* 2N: converged two-step-averaged displacement d   */
    SLBM_FIELD_STRESS = 1,    /* 3N: (sxx, syy, sxy) lattice units of the averaged state */
    SLBM_FIELD_ADJ_DISP = 2,  /* 2N: adjoint displacement of the averaged adjoint  */
    SLBM_FIELD_POPS = 3,      /* 8N: current primal post-streaming populations f^S */
    SLBM_FIELD_ADJ_POPS = 4,  /* 8N: current adjoint post-collision populations phi^C
                                 (SLBM_ESTATE before any adjoint solve or steps) */
    SLBM_FIELD_RESIDUAL = 5,  /* 2N: r = d - d* on the observation set (0 elsewhere) */
    SLBM_FIELD_CUR_DISP = 6,  /* 2N: bared displacement of the current state f^S   */
    SLBM_FIELD_AVG_POPS = 7   /* 8N: two-step-averaged populations of the last completed
                                 primal solve (the converged state; a checkpoint for
                                 solid_lbm_restore_solve) */
};

typedef struct slbm_ctx slbm_ctx; /* opaque; owns all device buffers */

/*
 * Problem description.  All pointers are host memory, read during
 * solid_lbm_init only.  N = nx * ny.
 */
typedef struct {
    int32_t nx, ny;            /* nodes per direction (>= 3 each) */
    double dx;                 /* lattice spacing (> 0; with check_interval 0, 0.005 / dx^2 < 1e18); dt = dx^2 */
    double E, nu;              /* uniform Young's modulus (> 0) and Poisson ratio
                                  (-1 < nu < 1); E ignored for E controls */
    int32_t domain;            /* SLBM_PERIODIC or SLBM_MASKED */
    const uint8_t *node_mask;  /* MASKED: N bytes, 1 = node of the domain.  No
                                  domain node may lie on the box edge. */
    const uint8_t *link_bc;    /* MASKED: 8N bytes [q * N + n]: kind of the link
                                  carrying f_q into node n from n - c_q; must be
                                  non-zero exactly when n - c_q is outside */
    const double *link_wall;   /* MASKED: 16N [(c * 8 + q) * N + n]: wall value per
                                  cut link: d_D (Dirichlet) or T (Neumann), lattice units */
    const double *link_normal; /* MASKED: 16N: outward unit normal per Neumann link */
    const double *fixed_force; /* 2N body force F for the E controls (NULL = 0) */
    const double *target;      /* 2N target displacement d* (required) */
    const uint8_t *obs_mask;   /* N bytes observation set (NULL = all domain nodes) */
    int32_t control_kind;      /* SLBM_CTRL_* */
    int32_t n_modes;           /* FORCE_MODES: number of modes k (1..64) */
    const double *force_modes; /* FORCE_MODES: k * 2N mode fields B_i */
    int32_t zero_mean_projection; /* FORCE_NODAL on PERIODIC: project control and
                                     gradient (eq. zero_mean_projection); 1 = on */
    int32_t normalize_objective;  /* 1: divide J by Cbar of eq. node_J; 0: plain 1/2 L2 */
    double tol;                /* residual tolerance (e.g. 1e-10); <= 0: run max_steps; NaN rejected */
    int64_t max_steps;         /* step limit per solve (>= 1) */
    int32_t check_interval;    /* K of the residual ||d(t) - d(t-K)|| / ||d(t)||;
                                  0 -> 2 * ceil(0.005 / dx^2) (even K) */
    void *stream;              /* hipStream_t for all work (NULL = default stream) */
    int32_t convergence;       /* SLBM_CONV_KLAG (0, default): the K-lag residual
                                  above < tol.  SLBM_CONV_CV (1): the paper's test
                                  (eq. convergence, eq. convergence_crit): c(t) =
                                  mean over domain nodes of |d(t)|^2 at every check
                                  (every K steps), converged when std(c) / mean(c)
                                  over the last cv_window checks (population std) is
                                  below tol (c = 0 throughout counts as converged).
                                  The adjoint uses its displacement likewise.  Single
                                  problems only: batches and tangent_solve return
                                  SLBM_EINVAL for SLBM_CONV_CV. */
    int32_t cv_window;         /* SLBM_CONV_CV: window in checks, 2..32 (0 -> 10) */
} slbm_problem;

typedef struct {
    int64_t steps;     /* step index t at which the residual test passed (or stopped) */
    int64_t sweeps;    /* lattice sweeps executed, including the averaging step */
    double residual;   /* last residual (SLBM_CONV_CV: last std(c) / mean(c)) */
    double wall_s;     /* wall time of the solve (host clock, stream drained) */
    double device_ms;  /* device time of the sweep loop: HIP events recorded on the
                          context's stream before the first and after the last sweep */
    int32_t converged; /* 1 if residual < tol */
    /* With solid_lbm_set_launch_timing on (else 0): the fused launches of the
     * sweep loop (several time steps per launch: wave strips or LDS tiles)
     * up to its final step, the sweeps they made, and their device time, from
     * HIP events on the context's stream around each run of back-to-back
     * fused launches.  The loop reads each residual check one check late;
     * the launches it issued after the converging check return at once and
     * are not counted. */
    int64_t fused_launches;
    int64_t fused_sweeps;
    double fused_ms;
} slbm_solve_info;

/*
 * Creates a context for one problem on the current HIP device: validates and
 * copies every input, allocates all device buffers (populations in two
 * SoA buffers of 8 planes, forcing, target, observation mask, plate records).
 * Returns SLBM_OK and *out, or a negative code (then *out = NULL).
 */
int solid_lbm_init(const slbm_problem *problem, slbm_ctx **out);

/*
 * Primal solve to steady state (eq. primal_fixed_point) for the given control:
 * control -> forcing or moduli, pseudo-time march from f^S(0) (cold: all
 * zero, eq. discrete_G closed by f^S(0) of d_0 = 0; warm: the equilibrium
 * populations of init_disp (2N)), residual test every K steps, then the
 * two-step average d = (d(t) + d(t+1)) / 2.  Leaves the averaged state, d,
 * r = d - d* and J in the context.  With tol <= 0 it runs exactly max_steps
 * steps and forms the same average (info->steps = max_steps).  control /
 * init_disp are read according to ptr_kind; init_disp may be NULL.  info may
 * be NULL.
 */
int primal_solve(slbm_ctx *ctx, const double *control, const double *init_disp,
                 int32_t ptr_kind, slbm_solve_info *info);

/*
 * Adjoint solve (Algorithm "ALBM"): from phi^C(0) = 0 iterate
 * phi^S = S^T phi^C, phi^C = (dC/df)^T phi^S - (dJ/df)^T at the converged
 * primal state, residual test on the adjoint displacement every K steps, then
 * the two-step average.  Requires a completed primal_solve (else
 * SLBM_ESTATE).  info may be NULL.
 */
int adjoint_solve(slbm_ctx *ctx, slbm_solve_info *info);

/*
 * Objective and gradient for one control: primal_solve (cold start) + J +
 * adjoint_solve + eq. optimality.  *J (host) receives the objective; grad
 * (length n_modes, 2N, N or 1 by control kind; NULL = J only, no adjoint)
 * is written according to ptr_kind.  primal_info / adjoint_info may be NULL.
 */
int objective_and_grad(slbm_ctx *ctx, const double *control, double *J, double *grad,
                       int32_t ptr_kind, slbm_solve_info *primal_info,
                       slbm_solve_info *adjoint_info);

/*
 * Vector-Jacobian product of the solution map at the last completed primal
 * solve: grad = (d dbar / d control)^T d_cot for a displacement cotangent d_cot
 * (2N; entries outside the domain are ignored; on periodic domains its mean
 * is removed, which does not change the product because dbar has zero mean).
 * This is Algorithm "ALBM" with the objective's source (dJ/df)^T replaced by
 * the cotangent and eq. optimality applied to it.  d_cot and grad (length as
 * for objective_and_grad) are read/written according to ptr_kind.  The
 * cotangent is staged in the context's own adjoint-source buffer: the primal
 * state, r = d - d* and J stay as they were, so a later adjoint_solve still
 * differentiates the objective.
 */
int adjoint_solve_vjp(slbm_ctx *ctx, const double *d_cot, double *grad, int32_t ptr_kind,
                      slbm_solve_info *info);

/* As objective_and_grad, with the primal solve started from init_disp (2N,
 * NULL = cold start) instead of d_0 = 0: a warm start changes the number of
 * steps, not the fixed point. */
int objective_and_grad_from(slbm_ctx *ctx, const double *control, const double *init_disp, double *J,
                            double *grad, int32_t ptr_kind, slbm_solve_info *primal_info,
                            slbm_solve_info *adjoint_info);

/* Forward-mode (tangent) solve, the f-AD of Sec. "Forward automatic
 * differentiation" on the GPU: J at `control` and its directional derivative
 * dJ = (dJ/dcontrol) . direction, from one iteration that carries every
 * population together with its derivative along the direction (dual numbers
 * through the same node map, closures and gamma included) to the K-lag test
 * on both the value and the derivative displacement, then the two-step
 * average.  direction has the length of the control; force directions are
 * projected to zero mean as the control is.  One solve per direction (the
 * cost that makes the adjoint preferable for many controls); a cross-check
 * of the adjoint gradient and the gradient for scalar controls.  control and
 * direction per ptr_kind; J, dJ host.  The primal state of ctx is
 * invalidated (primal_solve afresh before adjoint_solve).  SLBM_NOT_CONVERGED
 * (> 0) if max_steps ended the iteration first. */
int tangent_solve(slbm_ctx *ctx, const double *control, const double *direction, double *J, double *dJ,
                  int32_t ptr_kind, slbm_solve_info *info);

/* ---- helpers ---- */

/* Reinstates a converged primal state from a checkpoint: sets the control
 * (as primal_solve) and takes avg_pops (8N, the SLBM_FIELD_AVG_POPS of a
 * solve with that control) as the two-step-averaged fixed point; recomputes
 * d, r and J from it.  Afterwards adjoint_solve / adjoint_solve_vjp run as
 * after primal_solve. */
int solid_lbm_restore_solve(slbm_ctx *ctx, const double *control, const double *avg_pops,
                            int32_t ptr_kind);

/* Objective J of the last completed primal solve (host). */
int solid_lbm_objective(slbm_ctx *ctx, double *J);

/* Sets the forcing/moduli from a control (as primal_solve) and resets the
 * primal state to f^S(0) (cold, or warm from init_disp); no stepping. */
int solid_lbm_set_control(slbm_ctx *ctx, const double *control, const double *init_disp,
                          int32_t ptr_kind);

/* Advances the current primal state by n >= 0 steps (fixed-step mode). */
int solid_lbm_run_steps(slbm_ctx *ctx, int64_t n);

/* Resets the adjoint to phi^C = 0 and advances it by n >= 0 steps using the
 * residual of the last primal_solve (fixed-step mode). */
int solid_lbm_run_adjoint_steps(slbm_ctx *ctx, int64_t n);

/* Copies a field (SLBM_FIELD_*) into out (host or device per ptr_kind; out
 * holds the size listed with the field).  SLBM_ESTATE if the context does not
 * hold the state the field comes from: a completed primal_solve (DISP, STRESS,
 * RESIDUAL, AVG_POPS), a primal state (POPS, CUR_DISP), a completed
 * adjoint_solve (ADJ_DISP) or any adjoint state (ADJ_POPS); SLBM_EINVAL for an
 * unknown field or a NULL out. */
int solid_lbm_get_field(slbm_ctx *ctx, int32_t which, double *out, int32_t ptr_kind);

/* Timing helper: runs n primal (adjoint = 0) or adjoint (adjoint = 1) sweeps
 * on the current state and returns the device time of those sweeps in
 * *ms (HIP events recorded on the context's stream around them).  The state
 * advances; the outputs of the last completed solve stay as they were. */
int solid_lbm_time_sweeps(slbm_ctx *ctx, int32_t adjoint, int64_t n, double *ms);

/* Launch shape of the sweeps.  steps_per_launch: -1 automatic (default), 0 or
 * 1 = one time step per launch, else that many time steps fused in one
 * launch: 2, 4, 6 or 8 for periodic, uniform-material problems (wave-strip
 * kernel), 2 .. 8 for plates, E-field controls and problems given a tile by
 * solid_lbm_set_tiles (LDS-tiled kernel).  Automatic: the LDS-tiled kernel
 * for plates, E fields and periodic grids up to 131072 nodes (8 steps up to
 * 131072 nodes; above, the most of 6, 5, 4, 3 steps whose (32 - 2 steps)^2
 * tiles number no more than the device's compute units, else 6), the
 * wave-strip kernel with 8 steps for larger
 * periodic grids, with as many rows per wave as keep the wave count at or
 * below the device's SIMD count.  rows_per_wave: rows each wave of a wave-strip launch
 * covers (0 = automatic).  Every setting gives the same result bit for bit:
 * a fused launch performs exactly the arithmetic of its single sweeps.
 * SLBM_EINVAL if the value is out of range, or if a tile set by
 * solid_lbm_set_tiles would not fit with a halo of steps_per_launch. */
int solid_lbm_set_tuning(slbm_ctx *ctx, int32_t steps_per_launch, int32_t rows_per_wave);

/* Interior tile (tile_w x tile_h nodes) of each workgroup of the LDS-tiled
 * fused sweeps (selects that kernel also for periodic uniform problems); the
 * tile plus a halo of
 * steps_per_launch nodes on every side must hold at most 1024 nodes (one
 * node per thread of a 1024-thread workgroup; 8 FP64 planes in 64 KiB of
 * LDS, two copies for plates).  0, 0 = automatic (a 32 x 32 region; with
 * 8 steps per launch, grids that 16 x 16 tiles would leave short of one
 * workgroup per compute unit take 8 x 8 or 12 x 12 tiles).  Shapes whose
 * tiles all fit the device's compute units run with a launch plan (each
 * thread's node, code and staged boundary record, 16 KiB per tile) built at
 * the first solve of the shape.  Does not change results.  SLBM_EINVAL for
 * one zero and one nonzero value, negative values, or a region over 1024
 * nodes. */
int solid_lbm_set_tiles(slbm_ctx *ctx, int32_t tile_w, int32_t tile_h);

/* Progress report of long solves: fn(user, phase, step, residual) is called
 * on the calling thread from inside primal_solve / adjoint_solve /
 * objective_and_grad (and the other solving calls) when a residual check has
 * been read back and at least every_s seconds have passed since the last
 * report; phase 0 = primal, 1 = adjoint, 2 = tangent; step and residual are those of the
 * latest completed check.  fn = NULL turns reports off.  The callback must not
 * call into the library with the same ctx. */
typedef void (*slbm_progress_fn)(void *user, int32_t phase, int64_t step, double residual);
int solid_lbm_set_progress(slbm_ctx *ctx, slbm_progress_fn fn, void *user, double every_s);

/* Measurement switch: on != 0 makes the solve loops time their fused
 * launches (fields fused_launches, fused_sweeps, fused_ms of slbm_solve_info)
 * with one pair of HIP events per run of launches between residual checks;
 * off (default) leaves those fields 0.  Does not change results. */
int solid_lbm_set_launch_timing(slbm_ctx *ctx, int32_t on);

/* Message of the last error on ctx (or of the last failed init if ctx is NULL). */
const char *solid_lbm_last_error(const slbm_ctx *ctx);

/* Frees every device buffer of ctx (NULL is a no-op). */
void solid_lbm_destroy(slbm_ctx *ctx);

/* ---- batches: many independent problems solved together ----
 *
 * A batch holds up to 128 problems of any sizes and kinds (periodic or plate,
 * any control) that share tol, max_steps and stream.  All of them
 * advance in the same launches: one launch per time step (or per T fused
 * steps for the periodic ones) covers every instance still running, each with
 * its own residual test every K_i steps and its own stop.  Results equal those
 * of the same problems solved one by one (the per-instance arithmetic is the
 * same). */
typedef struct slbm_batch slbm_batch;

/* Creates a batch from count problems (validated and copied as by
 * solid_lbm_init).  Returns SLBM_OK and *out or a negative code.  Beyond the
 * per-instance buffers, the first batched solve of a tile shape gives each
 * tiled instance (plates, E fields) a launch plan of 16 KiB per tile (plus
 * 388 B of record list), kept until the shape changes or the batch is
 * destroyed; the no-allocation call uses none. */
int solid_lbm_batch_init(const slbm_problem *problems, int32_t count, slbm_batch **out);

/* Objective and gradient of every instance: controls[i] (length per the
 * instance's control kind), J[i] (host), grads[i] (NULL array = J only);
 * controls and grads per ptr_kind; primal_info / adjoint_info: NULL or arrays
 * of count entries (device_ms and wall_s are those of the whole batch). */
int batch_objective_and_grad(slbm_batch *batch, const double *const *controls, double *J,
                             double *const *grads, int32_t ptr_kind, slbm_solve_info *primal_info,
                             slbm_solve_info *adjoint_info);

/* As batch_objective_and_grad, with each instance's primal started from
 * init_disps[i] (2N, read per ptr_kind; a NULL array or NULL entry = cold
 * start d_0 = 0) instead of d_0 = 0 -- the warm start of
 * objective_and_grad_from, per instance: fewer steps, the same fixed point. */
int batch_objective_and_grad_from(slbm_batch *batch, const double *const *controls,
                                  const double *const *init_disps, double *J, double *const *grads,
                                  int32_t ptr_kind, slbm_solve_info *primal_info,
                                  slbm_solve_info *adjoint_info);

/* No-allocation variant of batch_objective_and_grad, for callers that cannot
 * allocate device memory during the call (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and return codes.  batch_objective_and_grad builds the work-lists of its
 * fused launches (one (instance, strip or tile) entry per work item) in
 * device memory that the batch allocates and grows on demand; this variant
 * writes them into a static device array of 65536 entries (512 KiB) that
 * the library holds on each GPU it runs on until the process ends, and calls
 * no allocating routine.  SLBM_EINVAL, before any work, if the batch's
 * current launch shape needs more entries (the message says how many).  The
 * array is rewritten by every call: calls that overlap on one GPU (other
 * threads, other streams) race on it and must be serialised by the caller. */
int batch_objective_and_grad_noalloc(slbm_batch *batch, const double *const *controls, double *J,
                                     double *const *grads, int32_t ptr_kind, slbm_solve_info *primal_info,
                                     slbm_solve_info *adjoint_info);

/* Adjoints and gradients of every instance at the state of the last
 * batch_objective_and_grad call (made with grads = NULL, so that a caller can
 * report between the two halves): grads[i] (length per the instance's
 * control kind, per ptr_kind; none may be NULL); adjoint_info: NULL or count
 * entries.  SLBM_ESTATE if an instance has no completed primal solve;
 * SLBM_NOT_CONVERGED (> 0) if an adjoint did not reach tol. */
int batch_gradient(slbm_batch *batch, double *const *grads, int32_t ptr_kind, slbm_solve_info *adjoint_info);

/* Fused launch shape of the batch's periodic instances (as solid_lbm_set_tuning). */
int solid_lbm_batch_set_tuning(slbm_batch *batch, int32_t steps_per_launch, int32_t rows_per_wave);

/* Steps per launch of the batch's tiled instances (plates and E-field
 * controls), which run in LDS tiles of (32 - 2 steps)^2 nodes: -1 automatic
 * (6), 1 single steps, 2 .. 8 fused; other values SLBM_EINVAL.  Independent
 * of the wave strips' shape; persistent launches run every instance in tiles
 * of this many steps.  Results do not change (a fused launch of k steps
 * equals k single steps bit for bit). */
int solid_lbm_batch_set_tile_steps(slbm_batch *batch, int32_t steps_per_launch);

/* Times n batched primal (adjoint = 0) or adjoint sweeps of every instance on
 * whatever the buffers hold (zeros after init); the instance states are
 * invalidated (the next solve starts from its control as always). */
int solid_lbm_batch_time_sweeps(slbm_batch *batch, int32_t adjoint, int64_t n, double *ms);

/* Persistent launches (on != 0): the batch's primal and adjoint loops run as
 * one persistent kernel (one workgroup of 1024 threads per compute unit, all
 * resident at once) captured in a HIP graph with a kernel that resets its
 * counters, replayed until every instance has stopped; rounds_per_launch
 * rounds per replay (0 = 4096).  In every round each running instance
 * takes its own next piece of work from one shared work-list -- a fused LDS
 * tile sweep of up to the tile steps per launch (solid_lbm_batch_set_tile_steps;
 * periodic instances are tiled too), a single step (its residual-check step,
 * or the plain steps before its next check or its max_steps), or the
 * reduction of its residual after a check -- so the
 * instances keep their own step counters and check intervals and a stopped
 * instance takes no more work; a grid barrier ends each round.  Results equal
 * the host-driven launches' bit for bit (same node arithmetic).  A barrier
 * that waits for more than a few seconds (workgroups not co-resident) ends
 * the launch with SLBM_EHIP instead of hanging.  Off by default; the
 * no-allocation variant always uses the host-driven launches. */
int solid_lbm_batch_set_persistent(slbm_batch *batch, int32_t on, int32_t rounds_per_launch);

/* Progress report of long batch solves, as solid_lbm_set_progress for one
 * context: fn(user, phase, step, residual) is called on the calling thread
 * from inside the batch solves when a check has been read back and at least
 * every_s seconds have passed since the last report; phase 0 = primal,
 * 1 = adjoint.  Host-driven launches report the time step of the check
 * read back and the largest residual among the instances still running then
 * that have completed a check (no report before the first such check; checks are read one behind, so that step can pass the last instance's
 * final step by up to two check intervals); persistent
 * launches report the rounds run and residual -1 (not read back).  fn = NULL
 * turns reports off.  The callback must not call into the library with the
 * same batch. */
int solid_lbm_batch_set_progress(slbm_batch *batch, slbm_progress_fn fn, void *user, double every_s);

/* Graph replays (persistent launches) and rounds of the last persistent solve half. */
int solid_lbm_batch_persistent_stats(const slbm_batch *batch, int64_t *launches, int64_t *rounds);

/* The context of instance i (owned by the batch) for solid_lbm_get_field and
 * the other per-context calls; NULL if i is out of range. */
slbm_ctx *solid_lbm_batch_instance(slbm_batch *batch, int32_t i);

const char *solid_lbm_batch_last_error(const slbm_batch *batch);
void solid_lbm_batch_destroy(slbm_batch *batch);

#ifdef __cplusplus
}
#endif
#endif /* SOLID_LBM_H */
