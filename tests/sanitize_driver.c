/* Drives every entry point of the test oracle once on tiny lattices, for the
 * AddressSanitizer / UndefinedBehaviorSanitizer build of tests/test_sanitizers.py
 * (host code only).  Exit status 0 and no sanitizer report are the pass. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "hlbm_oracle.h"

static void exercise(int stencil, int collision, double cs, int bcy, int objective) {
  orc_params p = {0};
  p.stencil = stencil;
  p.nx = 14;
  p.ny = 9;
  p.nz = stencil == ORC_D2Q9 ? 1 : 5;
  p.tau = 0.62;
  p.cs = cs;
  p.bc_x = ORC_BC_INLET_OUTLET;
  p.bc_y = bcy;
  p.bc_z = ORC_BC_PERIODIC;
  p.inlet_profile = ORC_INLET_PARABOLIC;
  p.u_in = 0.04;
  p.collision = collision;
  orc_lattice* L = orc_create(&p);
  if (!L) {
    fprintf(stderr, "create failed\n");
    exit(2);
  }
  const long n = orc_n(L);
  const int q = orc_q(L);
  double* noise = calloc(n, sizeof(double));
  double* d = calloc(n, sizeof(double));
  double* f = calloc(n * q, sizeof(double));
  double* g = calloc(n * q, sizeof(double));
  double* v = calloc(n * q, sizeof(double));
  double* u = calloc(3 * n, sizeof(double));
  double* rho = calloc(n, sizeof(double));
  unsigned char* flags = calloc(n, 1);
  for (long c = 0; c < n; ++c) noise[c] = 0.01 * (double)((c * 7919) % 13) / 13.0;
  orc_build_cylinder(L, 5.0, 4.0, 4.0, noise, ORC_NOISE_BOX, 3.0, 0.0);
  orc_get_porosity(L, d);
  orc_set_porosity(L, d);
  orc_init_equilibrium(L, 1.0, NULL);
  int lo[3] = {2, 0, 0}, hi[3] = {11, p.ny - 1, p.nz - 1};
  orc_set_objective(L, objective, lo, hi, objective == ORC_OBJ_MEA ? 12.0 : 0.04, 1.0 / 3.0);
  orc_step(L, 20);
  orc_run_steady(L, 40, 1e-30, 10);
  orc_moments(L, rho, u);
  orc_get_populations(L, f);
  orc_set_populations(L, f);
  (void)orc_objective(L);
  orc_mea_surface(L, flags);
  orc_mea_source(L, g);
  orc_window_reset(L);
  for (int k = 0; k < 6; ++k) {
    orc_window_sample(L);
    orc_step(L, 1);
  }
  (void)orc_window_count(L);
  (void)orc_window_objective(L);
  orc_window_mean_populations(L, g);
  for (int source = 0; source < 2; ++source)
    for (int turb = 0; turb < 2; ++turb) {
      orc_adjoint_prepare(L, source, source ? 0.6 : 0.0, turb);
      orc_adjoint_iterate(L, 5);
      double res = 0.0;
      orc_adjoint_solve(L, 10, 1e-30, 2, &res);
      orc_get_adjoint(L, g);
      orc_get_adjoint_virtual(L, v);
      orc_gradient(L, d);
      orc_adjoint_reset(L);
    }
  orc_apply_stream(L, f, v, g);
  orc_apply_stream_transpose(L, g, f, v);
  if (collision == ORC_COLL_BGK && cs == 0.0) {
    for (long c = 0; c < n; ++c) u[c] = (c % 3 == 0) ? 1.0 : 0.0;
    orc_tangent_seed(L);
    orc_tangent_step(L, u, 4);
    (void)orc_tangent_objective(L, u);
    orc_get_tangent(L, g);
  }
  /* per-cell maps */
  int qq, cc[57], opp[19];
  double w[19], fc[19], out[19], A[361], B[361], vel[3] = {0.03, -0.01, 0.005};
  orc_stencil(stencil, &qq, cc, w, opp);
  orc_equilibrium(stencil, 1.01, vel, fc);
  for (int i = 0; i < qq; ++i) fc[i] *= 1.0 + 0.01 * (i % 5);
  (void)orc_tau_eff(stencil, fc, 0.6, 0.1);
  orc_collide_cell(stencil, fc, 0.7, 0.6, cs, NULL, out);
  orc_jacobian_cell(stencil, fc, 0.7, 0.6, cs, ORC_TURB_DIFFERENTIATED, 0.65, A);
  orc_dcdd_cell(stencil, fc, 0.7, 0.6, out);
  orc_hrr_collide_cell(stencil, fc, 0.7, 0.6, cs, NULL, out);
  orc_hrr_jacobian_cell(stencil, fc, 0.7, 0.6, cs, ORC_TURB_FROZEN, 0.65, A);
  orc_hrr_dcdd_cell(stencil, fc, 0.7, 0.6, cs, ORC_TURB_DIFFERENTIATED, 0.65, out);
  for (int kind = 0; kind < 3; ++kind) {
    (void)orc_objective_cell(stencil, kind, fc, 0.7, 0.6, 0.04, 1.0 / 3.0);
    orc_dJdf_cell(stencil, kind, fc, 0.7, 0.6, 0.04, 1.0 / 3.0, out);
    (void)orc_dJdd_cell(stencil, kind, fc, 0.7, 0.6);
  }
  orc_outlet_values_cell(stencil, fc, out);
  orc_outlet_jacobian_cell(stencil, fc, B);
  free(noise); free(d); free(f); free(g); free(v); free(u); free(rho); free(flags);
  orc_destroy(L);
}

int main(void) {
  for (int stencil = 0; stencil < 2; ++stencil)
    for (int collision = 0; collision < 2; ++collision) {
      exercise(stencil, collision, 0.0, ORC_BC_WALLS, ORC_OBJ_DISS);
      exercise(stencil, collision, 0.12, ORC_BC_PERIODIC, ORC_OBJ_FFA);
      exercise(stencil, collision, 0.0, ORC_BC_WALLS, ORC_OBJ_MEA);
    }
  printf("ok\n");
  return 0;
}
