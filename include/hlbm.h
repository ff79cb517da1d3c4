/*
 * hlbm.h -- C ABI of the MI355X (gfx950) HLBM mean-flow adjoint library.
 *
 * The library computes, on one GPU, the data-parallel hot path of the method
 * of Ito et al., "Mean-Flow Adjoint Sensitivity Analysis of Unsteady Flow
 * Around Porous Cylinders Using a Homogenized Lattice Boltzmann Method":
 *
 *   primal HLBM sweep (Sec. 2, Eq. hlbm, or the HRRLBM collision of Eq.
 *   HRRLBM; optional Smagorinsky closure, Eqs. sgsStress/turbVisc/tauEff)
 *   ->  FP64 tracking average of the flow (Sec. 3.3, Eq. averageObjective)
 *   ->  adjoint LBM sweep on the frozen (mean) flow (Sec. 3.2-3.3, Eqs.
 *   adjoint_steady/adjoint_unsteady)  ->  gradient assembly dJ/dd over the
 *   porosity field (Eqs. gradients_steady/gradients_unsteady), for the drag
 *   (J_FFA, Eq. obj_ffa; J_MEA, Eq. obj_mea) and dissipation (J_DISS, Eq.
 *   obj_diss) objectives (Sec. 4); and the forward tangent of the transient
 *   (App. C).
 *
 * The call sequence follows the paper's problem statement (Sec. 3.1: minimise
 * J(alpha, f) subject to the lattice Boltzmann residual G(alpha, f) = 0, and
 * return dJ/dalpha) and the three phases of its Algorithm 1 (primal, adjoint,
 * gradient assembly).  The control variable is the lattice porosity d of
 * Sec. 2.1 (d = 1 fluid, d = 0 solid; d = 1 - dx^2 tau nu / K).
 *
 * Conventions
 *  - Lattice units: dx = dt = 1, c_s^2 = 1/3.  Cell index
 *    cell = x + nx*(y + ny*z).  Population arrays exchanged through this ABI
 *    use the canonical layout value[i*n + cell] with the direction order
 *      D2Q9 : 0 rest; 1..4 = (1,0),(0,1),(1,1),(-1,1); 5..8 their negatives
 *      D3Q19: 0 rest; 1..9 = (1,0,0),(0,1,0),(0,0,1),(1,1,0),(1,-1,0),
 *             (1,0,1),(1,0,-1),(0,1,1),(0,1,-1); 10..18 their negatives.
 *  - Every call returns hlbm_status (0 = HLBM_OK).  On error nothing is
 *    enqueued; hlbm_last_error() gives a thread-local message.
 *  - Ownership: the caller owns every buffer it passes; set_* calls copy,
 *    get_* calls write into caller memory.  The handle owns all device memory
 *    it allocates until hlbm_destroy.
 *  - Memory kind: arguments typed `const double*`/`double*` with an
 *    `hlbm_mem` flag are host pointers (HLBM_MEM_HOST) or device pointers on
 *    the lattice's device (HLBM_MEM_DEVICE), e.g. a PyTorch tensor's
 *    data_ptr().  All exchanged values are FP64 whatever the precision form.
 *  - Streams: every kernel is enqueued on desc.stream (a hipStream_t; NULL is
 *    the null stream).  Calls that return values to the host synchronise that
 *    stream; all others are asynchronous.
 *  - Threads: one host thread per handle at a time; different handles may be
 *    used from different threads.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hlbm_lattice_s* hlbm_lattice;

typedef enum {
  HLBM_OK = 0,
  HLBM_W_NOT_CONVERGED = 1, /* iteration limit reached; outputs valid */
  HLBM_E_INVALID = -1,      /* bad argument (size, range, NaN, null) */
  HLBM_E_OOM = -2,          /* device allocation failed */
  HLBM_E_STATE = -3,        /* call order violated (e.g. adjoint before objective) */
  HLBM_E_DIVERGED = -4,     /* non-finite state or residual, or a growing adjoint
                               residual; outputs undefined */
  HLBM_E_DEVICE = -5        /* HIP runtime error */
} hlbm_status;

typedef enum { HLBM_D2Q9 = 0, HLBM_D3Q19 = 1 } hlbm_stencil;

/* Precision forms.  FP64: FP64 storage and arithmetic.  FP32: FP32 storage
 * and arithmetic.  FP16S: FP32 arithmetic, populations stored as binary16
 * values of f_i - w_i.  In every form the window accumulators, objective and
 * gradient reductions and the adjoint residual are FP64. */
typedef enum { HLBM_FP64 = 0, HLBM_FP32 = 1, HLBM_FP16S = 2 } hlbm_precision;

/* Boundary kinds per axis.  WALLS: halfway bounce-back at -1/2 and n-1/2.
 * INLET_OUTLET (x only): column x = 0 is an equilibrium velocity inlet
 * f = f^eq(1, u_in(y)) (not collided); column x = nx-1 is a pressure outlet
 * whose missing populations come from a virtual column holding
 * f^eq(1, u of the last column) (density 1 as the paper's p_out = 0, zero-
 * gradient velocity).  Walls take precedence at corners. */
typedef enum { HLBM_BC_PERIODIC = 0, HLBM_BC_WALLS = 1, HLBM_BC_INLET_OUTLET = 2 } hlbm_bc;
typedef enum { HLBM_INLET_UNIFORM = 1, HLBM_INLET_PARABOLIC = 2 } hlbm_inlet;

/* Objectives (Sec. 4).  FFA: far-field drag over a plane, Eq. obj_ffa, with
 * p = rho/3.  DISS: viscous + porous dissipation over a box, Eq. obj_diss,
 * S = -Pi/(2 tau0 c_s^2) from the non-equilibrium part with respect to
 * f^eq(rho, u), nu/K = (1 - d)/tau0.  MOMENTUM: sum of j_x (test objective).
 * MEA: drag by momentum exchange on the cylinder's surface nodes, Eq.
 * obj_mea (see hlbm_set_objective). */
typedef enum { HLBM_OBJ_FFA = 0, HLBM_OBJ_DISS = 1, HLBM_OBJ_MOMENTUM = 2, HLBM_OBJ_MEA = 3 } hlbm_objective;

/* Treatment of the Smagorinsky closure in the adjoint (Sec. 5.4).  FROZEN:
 * frozen-turbulence assumption, relaxation time tau_adj + (mean tau_eff -
 * tau0) held constant.  DIFFERENTIATED: tau_eff(fbar) with tau0 -> tau_adj and
 * the extra (1/tau_eff)^2 dtau_eff/df f^neq term (needs the window to track
 * mean populations, desc.track_mean_populations = 1). */
typedef enum { HLBM_TURB_FROZEN = 0, HLBM_TURB_DIFFERENTIATED = 1 } hlbm_turb;

/* Adjoint source.  STEADY: Jacobians and dJ/df at the current primal state
 * (Eq. adjoint_steady).  MEAN: Jacobians at the window-mean state and the
 * window mean of dJ/df, dJ/dd (Eqs. adjoint_unsteady, gradients_unsteady). */
typedef enum { HLBM_SOURCE_STEADY = 0, HLBM_SOURCE_MEAN = 1 } hlbm_source;

typedef enum { HLBM_MEM_HOST = 0, HLBM_MEM_DEVICE = 1 } hlbm_mem;

typedef enum { HLBM_NOISE_NONE = 0, HLBM_NOISE_RIM = 1, HLBM_NOISE_BOX = 2 } hlbm_noise;

/* Fields for hlbm_get_field (n values each, or 3n for vectors, component-
 * major).  RHO/U: current state.  MEAN_RHO/MEAN_U: window means.
 * POROSITY: d.  MEAN_TAU: window mean of tau_eff. */
typedef enum {
  HLBM_FIELD_RHO = 0,
  HLBM_FIELD_U = 1,
  HLBM_FIELD_MEAN_RHO = 2,
  HLBM_FIELD_MEAN_U = 3,
  HLBM_FIELD_POROSITY = 4,
  HLBM_FIELD_MEAN_TAU = 5
} hlbm_field;

/* Collision model.  BGK: the HLBM-BGK collision toward f^eq(rho, d u) (Sec.
 * 2.1, Eq. hlbm).  HRR: the homogenized recursive regularized collision of
 * Sec. 2.2 (Eq. HRRLBM): C = f^eq + (1 - 1/tau_eff) f^(1) with the third-
 * order Hermite equilibrium at (rho, d u) and the regularized non-
 * equilibrium part (Hermite coefficients a1 = (1 - d) j, a2 projected, a3
 * recursive from d u and a2), third order restricted to the components
 * H_aab (a != b) the velocity set supports.  Either takes the Smagorinsky
 * closure (smagorinsky_cs > 0). */
typedef enum { HLBM_COLL_BGK = 0, HLBM_COLL_HRR = 1 } hlbm_collision;

/* Cache hints of the sweeps: the population loads and stores of both AA
 * steps of the D2Q9 primal sweep (with or without the window statistics),
 * of the even step of the D3Q19 primal sweep (its odd step reuses the lines
 * of the neighbouring xy layer) and of the even step of the adjoint sweep;
 * the window sums of every window step and the adjoint's frozen per-cell
 * data in both adjoint steps (data of the cell's own, read once a sweep).
 * AUTO: streaming (nontemporal) hints when the populations and the porosity
 * exceed 256 MiB, the size of the MI355X Infinity Cache, plain accesses
 * otherwise (a lattice that stays in that cache from one step to the next
 * is 5-20 % slower with the hints, a larger D2Q9 one 5-20 % faster (adjoint
 * 4-5 %), D3Q19 1-2 %).  PLAIN and STREAMING force either.  Results are
 * bitwise identical under every policy, for either collision.  Every other
 * kernel uses plain accesses. */
typedef enum { HLBM_CACHE_AUTO = 0, HLBM_CACHE_PLAIN = 1, HLBM_CACHE_STREAMING = 2 } hlbm_cache_policy;

typedef struct {
  uint32_t struct_size;   /* sizeof(hlbm_desc) */
  int32_t stencil;        /* hlbm_stencil */
  int32_t precision;      /* hlbm_precision */
  int32_t nx, ny, nz;     /* nz = 1 for D2Q9; nx >= 2 */
  double tau;             /* molecular relaxation time tau0 > 1/2 (nu = (tau0 - 1/2)/3) */
  double smagorinsky_cs;  /* Cs >= 0; 0 disables the closure */
  int32_t bc_x, bc_y, bc_z;   /* hlbm_bc; y and z may not be INLET_OUTLET */
  int32_t inlet_profile;  /* hlbm_inlet (used with bc_x = INLET_OUTLET) */
  double u_in;            /* uniform inflow speed or parabola maximum */
  double force[3];        /* constant body force 3 w_i xi_i.G added after collision (tests) */
  int32_t track_mean_populations; /* 1: the window also accumulates full mean populations */
  int32_t collision;      /* hlbm_collision */
  int32_t cache_policy;   /* hlbm_cache_policy */
  void* stream;           /* hipStream_t or NULL */
} hlbm_desc;

typedef struct {
  uint32_t struct_size;   /* sizeof(hlbm_adjoint_opts) */
  int32_t source;         /* hlbm_source */
  double tau_adj;         /* adjoint relaxation time (Sec. 5.4 regularisation); <= 0: tau0 */
  int32_t turb;           /* hlbm_turb (ignored without the closure) */
  int64_t max_iters;      /* iterations (rounded up to an even number) */
  double tol;             /* stop when max|phi_k - phi_(k-M)| <= tol max|phi_k|; 0 = run max_iters */
  int64_t check_every;    /* M (rounded up to even), default 100 */
  int32_t restart;        /* 1: start from phi = 0 and re-freeze the Jacobian data */
} hlbm_adjoint_opts;

typedef struct {
  int64_t iters;          /* iterations performed by this call */
  double residual;        /* last relative residual (or -1 if never checked) */
} hlbm_adjoint_report;

/* ---- lifetime ------------------------------------------------------------ */

/* Allocate a lattice: populations (SoA, planes padded to 256 B), porosity,
 * outlet buffers.  Porosity starts at 1, populations at rest equilibrium.
 * Errors: INVALID (sizes, tau <= 1/2, Cs < 0, bad enums), OOM, DEVICE. */
hlbm_status hlbm_create(const hlbm_desc* desc, hlbm_lattice* out);
/* Free every device buffer of the handle (synchronises its stream). */
void hlbm_destroy(hlbm_lattice lat);
/* Device bytes a lattice of this descriptor holds at most for one query:
 * populations, porosity, outlet values, reduction partials and the steady-
 * check snapshot; the objective's region buffers for region_cells cells of
 * kind `objective` (0 cells: no objective); with_window != 0 the FP64 window
 * sums; with_adjoint != 0 the adjoint populations, frozen data, gradient data
 * and residual snapshot.  A velocity probe and the forward tangent's buffers
 * are not included.  Equals hlbm_device_bytes after such a query (primal
 * with steady checks and window, adjoint with residual checks, gradient).
 * Errors: INVALID (descriptor, region_cells outside [0, n], kind). */
hlbm_status hlbm_footprint_bytes(const hlbm_desc* desc, int with_window, int with_adjoint,
                                 int64_t region_cells, int32_t objective, uint64_t* bytes);
/* Device bytes the handle holds now (every buffer it has allocated). */
hlbm_status hlbm_device_bytes(hlbm_lattice lat, uint64_t* bytes);

/* ---- geometry and initial state (rows a1, a2) --------------------------- */

/* Copy a porosity field d[n]; every value must be finite and in [0, 1]
 * (checked on the host for host input, on the device for device input). */
hlbm_status hlbm_set_porosity(hlbm_lattice lat, const double* d, int64_t n, int32_t mem);
/* The same as hlbm_set_porosity with device input, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): it calls no allocating routine.  d[n] is
 * device memory on the lattice's device.  The validation flag lives in 4
 * bytes of a 256-byte library-owned device array, one per GPU, held until the
 * process ends; each call clears it first.  Calls that overlap on one GPU
 * (concurrent streams or threads) race on that flag.  Errors: INVALID (size,
 * or a value outside [0, 1] or not finite: the field then holds the rejected
 * values), STATE, DEVICE. */
hlbm_status hlbm_set_porosity_noalloc(hlbm_lattice lat, const double* d, int64_t n);
/* Build d on the device for a cylinder of diameter D centred at (xc, yc),
 * axis along z: solid fraction chi = 1 for r <= R-1, (1 + cos(pi(r-R+1)/2))/2
 * for R-1 < r < R+1, 0 beyond; d = 1 - chi (Sec. 5.1: d = 0 in the cylinder).
 * noise[n] (may be NULL) holds caller-drawn values: RIM adds them to d where
 * 0 < chi < 1, BOX adds them to chi where |x-xc|, |y-yc| <= box_half; both
 * clamp to [0, 1].  d_solid in [0, 1) is the porosity inside a permeable
 * cylinder (Sec. 2.1: d = 1 - dx^2 tau nu / K for permeability K; the
 * validation cases of Sec. 5.2 use K = 1e-6 m^2): the final field is
 * 1 - (1 - d)(1 - d_solid), i.e. d unchanged for d_solid = 0.
 * Errors: INVALID (non-finite centre, D <= 0, d_solid outside [0, 1), bad
 * noise mode or length), DEVICE. */
hlbm_status hlbm_build_cylinder(hlbm_lattice lat, double xc, double yc, double D,
                                const double* noise, int64_t n, int32_t mem,
                                int32_t noise_mode, double box_half, double d_solid);
/* f_i = f_i^eq(rho0, d u) with u[3n] (component-major) or, if u is NULL, the
 * inlet profile continued into the domain (INLET_OUTLET) or rest.  Resets the
 * step parity, the window and the adjoint. */
hlbm_status hlbm_init_equilibrium(hlbm_lattice lat, double rho0, const double* u, int64_t n,
                                  int32_t mem);
hlbm_status hlbm_set_populations(hlbm_lattice lat, const double* f, int64_t n_values,
                                 int32_t mem);
hlbm_status hlbm_get_populations(hlbm_lattice lat, double* f, int64_t n_values, int32_t mem);

/* ---- objective (row a6) -------------------------------------------------- */

/* Objective over the inclusive box lo..hi (a one-cell-thick plane for FFA).
 * With INLET_OUTLET the box may not touch column 0.  u0, p0: FFA reference
 * velocity and pressure (p0 = 1/3 for rho = 1).
 * HLBM_OBJ_MEA (Sec. 4 Eq. obj_mea, drag by momentum exchange on the
 * surface nodes, n = e_x): u0 carries the surface area A (the perimeter in
 * 2D; must be > 0), p0 is unused.  The surface nodes are the box cells with
 * d < 1/2 and a lattice neighbour with d >= 1/2, kept one cell away from the
 * box faces on axes the box does not span completely; they follow later
 * porosity changes.  J_MEA is linear in f: its adjoint source is constant
 * and dJ/dd = 0 (the surface set is piecewise constant in d). */
hlbm_status hlbm_set_objective(hlbm_lattice lat, int32_t kind, const int32_t lo[3],
                               const int32_t hi[3], double u0, double p0);

/* ---- primal and window (rows a3, a4, a5) --------------------------------- */

/* Advance n_steps collide-and-stream steps (in-place AA pattern).  If
 * accumulate != 0 every step adds its pre-collision state to the FP64 window
 * (rho, j, optional f, tau_eff, objective terms and dJ/df, dJ/dd
 * coefficients).  If steady_tol > 0, every check_every steps the call stops
 * once max|u(t) - u(t - check_every)| <= steady_tol max|u|.  *steps_done (may
 * be NULL) receives the steps taken.  Returns DIVERGED on a non-finite check,
 * W_NOT_CONVERGED if steady_tol > 0 was not met.  FP32 and FP16 lattices
 * add the window values of each group of four consecutive steps to the FP64
 * sums in one pass (the first three steps leave their FP32 values in
 * pending slots; the same additions in the same order); when the call
 * returns, every step taken is in the sums. */
hlbm_status hlbm_run_primal(hlbm_lattice lat, int64_t n_steps, int32_t accumulate,
                            double steady_tol, int64_t check_every, int64_t* steps_done);
hlbm_status hlbm_window_reset(hlbm_lattice lat);
hlbm_status hlbm_window_count(hlbm_lattice lat, int64_t* samples);
/* which = 0: J of the current state; which = 1: window mean of J. */
hlbm_status hlbm_get_objective(hlbm_lattice lat, int32_t which, double* J);

/* ---- forward tangent (App. C) -------------------------------------------- */

/* The exact transient sensitivity of the instantaneous objective along a
 * porosity direction v (App. C, where it diverges for the unsteady flow):
 * advances n_steps primal steps from the current state together with
 * fdot = (df/dd) v, seeded fdot = 0 at the call (the current state is taken
 * as independent of d), and every record_every steps writes J(t) and
 * dJ(t)/dd . v = dJ/df . fdot + dJ/dd v to out[2r], out[2r + 1] (host
 * memory, floor(n_steps / record_every) pairs).  v[n] is host or device
 * memory per mem.  The primal state, parity and step count advance as with
 * hlbm_run_primal (no window accumulation, no probe).  FP64 lattices
 * without the Smagorinsky closure.  Errors: INVALID (precision, closure,
 * sizes, null output), STATE (no objective), OOM, DEVICE. */
hlbm_status hlbm_run_tangent(hlbm_lattice lat, const double* v, int64_t n, int32_t mem,
                             int64_t n_steps, int64_t record_every, double* out);

/* ---- adjoint and gradient (rows a7, a8, a9) ------------------------------ */

/* Freeze the Jacobian data (row a7) and iterate the adjoint sweep (row a8)
 * until its variables are steady (Algorithm 1).  With tol > 0, every
 * check_every iterations the relative residual max|phi_k - phi_(k-M)| /
 * max|phi_k| is formed in FP64: at most tol ends the call with OK; a
 * non-finite value, or a residual above 1e3 times the smallest residual of
 * this call, ends it with DIVERGED (outputs undefined); max_iters without
 * either gives W_NOT_CONVERGED (outputs valid, report->residual the last
 * residual).  tol = 0 runs max_iters iterations and checks nothing.
 * Returns STATE without an objective (or without a window for MEAN, or
 * without tracked mean populations for the differentiated closure or for a
 * MEAN source with the HRR collision, whose frozen data include the mean
 * second moments). */
hlbm_status hlbm_solve_adjoint(hlbm_lattice lat, const hlbm_adjoint_opts* opts,
                               hlbm_adjoint_report* report);
/* dJ/dd[n] (FP64), 0 on the inlet column (row a9). */
hlbm_status hlbm_get_gradient(hlbm_lattice lat, double* g, int64_t n, int32_t mem);
/* Adjoint populations phi on post-collision slots, canonical layout (q*n). */
hlbm_status hlbm_get_adjoint(hlbm_lattice lat, double* phi, int64_t n_values, int32_t mem);

/* ---- fields, timing, errors ---------------------------------------------- */

hlbm_status hlbm_get_field(hlbm_lattice lat, int32_t field, double* out, int64_t n_values,
                           int32_t mem);
hlbm_status hlbm_synchronize(hlbm_lattice lat);
/* Sweep timing by HIP events on the lattice's stream.  With every > 0, the
 * sweeps of each kind are timed in blocks of up to `every` back-to-back
 * launches: an event is recorded before the first and after the last launch
 * of a block, and a block ends with the caller's run of consecutive sweeps
 * (hlbm_run_primal's steps between steady checks, hlbm_solve_adjoint's
 * iterations between residual checks), so the time per launch is the sweep's
 * duration in a steady stream of launches, dispatch gaps included.  The events
 * are read back lazily: timing adds no host synchronization to a run.
 * every = 0 switches it off; every call clears the statistics.  kind: 0
 * primal sweep, 1 primal step with window accumulation (sweep plus the
 * region pass of a small objective region), 2 adjoint sweep.
 * hlbm_profile_get returns the mean time per launch in microseconds and the
 * number of launches timed (blocks finished so far). */
hlbm_status hlbm_profile_enable(hlbm_lattice lat, int32_t every);
hlbm_status hlbm_profile_get(hlbm_lattice lat, int32_t kind, double* mean_us, int64_t* sampled);
/* Velocity probe: every primal step records u_y of cell (x, y, z) (the
 * pre-collision state of that step) into a device ring of `capacity` values
 * (capacity 0 removes the probe).  hlbm_get_probe copies the last
 * min(steps, capacity) values, oldest first, and their count. */
hlbm_status hlbm_set_probe(hlbm_lattice lat, int32_t x, int32_t y, int32_t z, int64_t capacity);
hlbm_status hlbm_get_probe(hlbm_lattice lat, double* out, int64_t capacity, int64_t* count);
/* Algorithmic bytes per lattice update of the primal sweep (accumulate = 0 or
 * 1) and of the adjoint sweep for this lattice's configuration.  A window
 * step of an FP32 or FP16 lattice is counted as the mean over a group of
 * four steps: its FP64 sums are read and written once per group, the first
 * three steps leaving their values as FP32 for the fourth (see
 * hlbm_run_primal). */
hlbm_status hlbm_bytes_per_update(hlbm_lattice lat, double* primal, double* primal_window,
                                  double* adjoint);
/* Bandwidth probe (a measurement, not a step of the method): n_launches
 * back-to-back launches of a kernel that moves exactly the bytes of a plain
 * primal sweep -- it reads every population slot and the porosity of each
 * cell and writes the populations back unchanged -- on the same workgroups,
 * tile order and addressing, with no arithmetic.  pattern 0: each cell's own
 * slots (the even AA step's accesses); 1: interior cells read and write the
 * odd step's upstream neighbour slots; 2: the two-array pull pattern, the
 * alternative to the in-place propagation -- interior cells read slot i of
 * their upstream cell x - xi_i and every cell writes its own slots to a
 * second population array (allocated for the call and freed before it
 * returns) with nontemporal hints.  streaming != 0: nontemporal hints on
 * every population access (patterns 0 and 1).  *us_per_launch receives the
 * mean time per launch (HIP events on the lattice's stream around the
 * launches; synchronises that stream).  The lattice state is unchanged.
 * Errors: INVALID (pattern, n_launches < 1, null output), OOM (pattern 2),
 * DEVICE. */
hlbm_status hlbm_copy_probe(hlbm_lattice lat, int32_t pattern, int32_t streaming, int64_t n_launches,
                            double* us_per_launch);
/* Changes the relaxation time, Smagorinsky constant and inflow speed of an
 * existing lattice (same validity rules as hlbm_create); the state, window
 * and adjoint are kept but the adjoint must be prepared again.  Lets a caller
 * reuse a resident lattice of the same shape for a new query. */
hlbm_status hlbm_reconfigure(hlbm_lattice lat, double tau, double smagorinsky_cs, double u_in);

/* ---- groups: many small lattices in one packed launch per step --------- */

/* A group steps several lattices of one stencil and precision with a single
 * kernel launch per step (and per phase kind), each member running exactly
 * the per-cell code of its own sweep, so a member's results do not depend on
 * the other members.  Used by the request scheduler to fill the GPU with
 * small lattices; every launch goes to the group's stream. */
typedef struct hlbm_group_s* hlbm_group;
typedef enum {
  HLBM_GROUP_PRIMAL = 0,         /* primal step */
  HLBM_GROUP_PRIMAL_WINDOW = 1,  /* primal step with window accumulation */
  HLBM_GROUP_ADJOINT = 2         /* adjoint iteration (adjoint already prepared) */
} hlbm_group_mode;

hlbm_status hlbm_group_create(void* stream, hlbm_group* out);
void hlbm_group_destroy(hlbm_group g);
/* Sets the members (the lattices stay owned by the caller) and what each does
 * per step.  Synchronises every member's own stream.  Members must share
 * stencil, precision and collision model; ADJOINT members need a prepared adjoint
 * (hlbm_solve_adjoint with max_iters = 0).  Until the next hlbm_group_set the
 * members may not be advanced by any other call (hlbm_group_step returns
 * E_STATE for a member that was).  count = 0 empties it. */
hlbm_status hlbm_group_set(hlbm_group g, const hlbm_lattice* lats, const int32_t* modes, int32_t count);
/* Advances every member by n steps / iterations (asynchronous).  On a group
 * with its own stream (not the null stream), a run of n >= 16 steps is
 * launched as one HIP graph of kernel nodes, captured once and replayed while
 * the members, their modes and n repeat (one host launch per run instead of
 * one per kernel); otherwise, or if capture fails, one launch per step. */
hlbm_status hlbm_group_step(hlbm_group g, int64_t n);
hlbm_status hlbm_group_synchronize(hlbm_group g);

const char* hlbm_status_string(hlbm_status s);
const char* hlbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
