/*
 * hlbm_oracle.h -- plain FP64 CPU oracle of the HLBM mean-flow adjoint path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * What it computes (Ito et al., "Mean-Flow Adjoint Sensitivity Analysis of
 * Unsteady Flow Around Porous Cylinders Using a Homogenized Lattice Boltzmann
 * Method"):
 *   - the HLBM-BGK primal step (Sec. 2.1, Eq. hlbm and the equilibrium with
 *     the porosity-scaled velocity), optionally with the Smagorinsky effective
 *     relaxation time (Sec. 2.2, Eqs. sgsStress, turbVisc, tauEff);
 *   - the tracking average over a window (Sec. 3.3, Eq. averageObjective);
 *   - the objectives J_FFA and J_DISS and their partial derivatives (Sec. 4,
 *     Eqs. obj_ffa, obj_diss);
 *   - the steady and mean-flow adjoint iterations (Sec. 3.2-3.3, Eqs.
 *     adjoint_steady, adjoint_unsteady) and the gradient assembly (Eqs.
 *     gradients_steady, gradients_unsteady), with the Smagorinsky closure
 *     either differentiated (Sec. 5.4, the dC/df expression with the
 *     (1/tau_eff)^2 term) or frozen (frozen-turbulence assumption, Sec. 5.4).
 *
 * The mean-flow gradient of the nonlinear objectives (J_FFA, J_DISS) on a
 * changing flow has no closed-form ground truth as a whole; it is pinned by
 * parts in the tests: per-cell Jacobians by finite differences, window means
 * as plain means on a changing flow, the window-mean source dJ/df and dJ/dd
 * by central differences of the per-cell objective at every sampled state,
 * the whole path against the steady adjoint on a steady flow and, for the
 * linear J_MEA, against the steady path at the mean state.
 *
 * Conventions: lattice units (dx = dt = 1, c_s^2 = 1/3).  Exchange arrays
 * use the "canonical" layout value[i*n + cell], cell = x + nx*(y + ny*z).
 * Internally the oracle keeps populations cell-major (f[cell*q + i]).
 */
#ifndef HLBM_ORACLE_H
#define HLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_WALLS = 1, ORC_BC_INLET_OUTLET = 2 };
enum { ORC_INLET_UNIFORM = 1, ORC_INLET_PARABOLIC = 2 };
enum { ORC_OBJ_FFA = 0, ORC_OBJ_DISS = 1, ORC_OBJ_MOMENTUM = 2, ORC_OBJ_MEA = 3 };
enum { ORC_TURB_FROZEN = 0, ORC_TURB_DIFFERENTIATED = 1 };
enum { ORC_NOISE_NONE = 0, ORC_NOISE_RIM = 1, ORC_NOISE_BOX = 2 };
enum { ORC_COLL_BGK = 0, ORC_COLL_HRR = 1 };

typedef struct {
  int stencil;        /* ORC_D2Q9 or ORC_D3Q19 */
  int nx, ny, nz;     /* nz = 1 for D2Q9 */
  double tau;         /* molecular relaxation time tau0 (> 1/2) */
  double cs;          /* Smagorinsky constant; 0 gives plain BGK */
  int bc_x;           /* ORC_BC_*: periodic, walls, or an equilibrium inlet at x=0 plus a
                         pressure outlet (density 1, zero-gradient velocity) at x=nx-1 */
  int bc_y, bc_z;     /* ORC_BC_PERIODIC or ORC_BC_WALLS (halfway bounce-back) */
  int inlet_profile;  /* ORC_INLET_UNIFORM or ORC_INLET_PARABOLIC (parabolic in y) */
  double u_in;        /* uniform inflow speed, or parabola maximum */
  double force[3];    /* constant body force added after collision (tests only) */
  int collision;      /* ORC_COLL_BGK (Eq. hlbm) or ORC_COLL_HRR (Eq. HRRLBM) */
} orc_params;

typedef struct orc_lattice orc_lattice;

orc_lattice* orc_create(const orc_params* p);
void orc_destroy(orc_lattice* L);
int orc_q(const orc_lattice* L);
long orc_n(const orc_lattice* L);

/* Porosity field d (d = 1 fluid, d = 0 solid). */
int orc_set_porosity(orc_lattice* L, const double* d);
int orc_get_porosity(const orc_lattice* L, double* d);
/* Cylinder of diameter D centred at (xc, yc), axis along z, cosine ramp over
 * [R-1, R+1]; noise (one value per cell, drawn by the caller) is applied per
 * noise_mode: RIM adds it to d on cells with 0 < chi < 1, BOX adds it to chi
 * on cells with |x-xc|,|y-yc| <= box_half; both clamp to [0,1].  A permeable
 * cylinder (Sec. 2.1, d = 1 - dx^2 tau nu / K inside) has porosity d_solid
 * in its core: d <- 1 - (1 - d)(1 - d_solid). */
int orc_build_cylinder(orc_lattice* L, double xc, double yc, double D,
                       const double* noise, int noise_mode, double box_half, double d_solid);

/* f_i = f_i^eq(rho0, d*u); u is 3*n component-major or NULL (NULL: the inlet
 * profile continued into the domain for inlet/outlet channels, else 0). */
int orc_init_equilibrium(orc_lattice* L, double rho0, const double* u);
int orc_set_populations(orc_lattice* L, const double* f);
int orc_get_populations(const orc_lattice* L, double* f);
int orc_step(orc_lattice* L, long nsteps);
/* Steady run: stops once max|u(t)-u(t-check)| <= tol*max|u| (checked every
 * check_every steps) or after max_steps; returns the steps taken. */
long orc_run_steady(orc_lattice* L, long max_steps, double tol, long check_every);
int orc_moments(const orc_lattice* L, double* rho, double* u /* 3*n */);

/* Objective region: inclusive box lo..hi.  For ORC_OBJ_MEA (drag by the
 * momentum exchange algorithm, Sec. 4 Eq. obj_mea) u0 carries the surface
 * area A (the perimeter in 2D) and the surface set is the box cells (away
 * from the box faces on axes the box does not span completely) with d < 1/2
 * and a lattice neighbour with d >= 1/2. */
int orc_set_objective(orc_lattice* L, int kind, const int* lo, const int* hi,
                      double u0, double p0);
double orc_objective(const orc_lattice* L);
/* J_MEA surface flags (1 on surface cells) and dJ_MEA/df ([i*n + c]). */
int orc_mea_surface(const orc_lattice* L, unsigned char* flags);
int orc_mea_source(const orc_lattice* L, double* g);

/* Tracking average (window) of the post-stream state. */
void orc_window_reset(orc_lattice* L);
void orc_window_sample(orc_lattice* L);
long orc_window_count(const orc_lattice* L);
double orc_window_objective(const orc_lattice* L);
int orc_window_mean_populations(const orc_lattice* L, double* fbar);

/* Adjoint.  source: 0 = current state (steady adjoint), 1 = window means
 * (mean-flow adjoint).  tau_adj <= 0 means tau0. */
int orc_adjoint_prepare(orc_lattice* L, int source, double tau_adj, int turb);
void orc_adjoint_reset(orc_lattice* L);
int orc_adjoint_iterate(orc_lattice* L, long iters);
/* Iterates until max|phi^k - phi^(k-check)| <= tol*max|phi^k| or max_iters;
 * returns the iterations done, writes the last relative residual. */
long orc_adjoint_solve(orc_lattice* L, long max_iters, double tol, long check_every,
                       double* residual);
int orc_get_adjoint(const orc_lattice* L, double* phi);
int orc_gradient(const orc_lattice* L, double* g);

/* Forward tangent (App. C): fdot = (df/dd) v along the primal trajectory.
 * seed: fdot = 0 at the current state; step: advances f and fdot together;
 * objective: dJ(t)/dd . v of the current objective at the current state. */
int orc_tangent_seed(orc_lattice* L);
/* HRRLBM per-cell maps (Eq. HRRLBM): collision, dC/df and dC/dd (complex
 * steps; turb FROZEN holds tau_frozen). */
void orc_hrr_collide_cell(int stencil, const double* f, double d, double tau0, double cs,
                          const double* force, double* out);
void orc_hrr_jacobian_cell(int stencil, const double* f, double d, double tau_a, double cs, int turb,
                           double tau_frozen, double* A);
void orc_hrr_dcdd_cell(int stencil, const double* f, double d, double tau_a, double cs, int turb,
                       double tau_frozen, double* out);
int orc_tangent_step(orc_lattice* L, const double* v, long nsteps);
double orc_tangent_objective(const orc_lattice* L, const double* v);
int orc_get_tangent(const orc_lattice* L, double* fdot);

/* Per-cell building blocks (exposed for the pin tests). */
void orc_stencil(int stencil, int* q, int* c /* 3*q */, double* w, int* opp);
void orc_equilibrium(int stencil, double rho, const double* v, double* feq);
double orc_tau_eff(int stencil, const double* f, double tau0, double cs);
void orc_collide_cell(int stencil, const double* f, double d, double tau0, double cs,
                      const double* force, double* out);
void orc_jacobian_cell(int stencil, const double* f, double d, double tau_a, double cs,
                       int turb, double tau_frozen, double* A /* A[j*q+i] = dC_j/df_i */);
void orc_dcdd_cell(int stencil, const double* f, double d, double tau_used, double* out);
double orc_objective_cell(int stencil, int kind, const double* f, double d, double tau0,
                          double u0, double p0);
void orc_dJdf_cell(int stencil, int kind, const double* f, double d, double tau0,
                   double u0, double p0, double* out);
double orc_dJdd_cell(int stencil, int kind, const double* f, double d, double tau0);
/* Outlet virtual values V_i = f_i^eq(1, u) of a last-column cell and their
 * Jacobian B[j*q+i] = dV_j/df_i. */
void orc_outlet_values_cell(int stencil, const double* f, double* out);
void orc_outlet_jacobian_cell(int stencil, const double* f, double* B);
/* Adjoint values on the outlet's virtual slots (canonical layout). */
int orc_get_adjoint_virtual(const orc_lattice* L, double* phiv);
/* Streaming map S ((post-collision values, virtual values) -> state values)
 * and its transpose, on canonical-layout arrays; pinned inlet slots receive 0. */
int orc_apply_stream(const orc_lattice* L, const double* in, const double* vin, double* out);
int orc_apply_stream_transpose(const orc_lattice* L, const double* in, double* out,
                               double* vout);

#ifdef __cplusplus
}
#endif
#endif
