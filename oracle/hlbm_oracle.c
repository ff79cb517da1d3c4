/*
 * hlbm_oracle.c -- plain FP64 CPU oracle of the HLBM mean-flow adjoint path.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library.
 *
 * Deliberately slow and literal: two population arrays (state f, post-
 * collision fpost), an explicit streaming table src[state slot] -> post-
 * collision slot and its explicit transpose, and a full q x q Jacobian per
 * cell written out with the chain rule.  Built with -O2 -ffp-contract=off.
 * OpenMP only splits independent per-cell loops; every reduction is serial.
 *
 * Readings of the paper where it is silent (numbered as in the design notes):
 *  - the equilibrium of the collision uses the porosity-scaled velocity
 *    d*u with u = j/rho of the pre-collision state (Sec. 2.1);
 *  - the strain rate of the Smagorinsky closure and of J_DISS comes from the
 *    non-equilibrium part with respect to f^eq(rho, u) (Sec. 2.2, Sec. 4.3);
 *  - the implicit Smagorinsky relation tau = tau0 + 3 Cs^2 |S(tau)| with
 *    |S| = sqrt(2 S:S) and S = -Pi/(2 tau c_s^2) is solved in closed form;
 *  - nu/K of J_DISS is (1-d)/tau0, from d = 1 - dx^2 tau nu / K (Sec. 2.1);
 *  - the window mean divides by the number of samples t_e - t_s + 1;
 *  - the adjoint variable phi lives on post-collision slots: lambda =
 *    (dC/df)^T phi - dJ/df at each cell, then phi = S^T lambda (Eq.
 *    adjoint_steady read as "collide at x, then move against xi_i");
 *  - frozen turbulence keeps tau_adj + (mean tau_eff - tau0) constant;
 *    the differentiated closure uses tau_eff(fbar) with tau0 -> tau_adj.
 */
#include "hlbm_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 19

struct orc_lattice {
  orc_params p;
  int q;
  long n;
  int c[QMAX][3];
  double w[QMAX];
  int opp[QMAX];
  double* d;      /* [n] */
  double* f;      /* [n*q] state (post-stream, pre-collision) */
  double* fpost;  /* [n*q] post-collision */
  double* vpost;  /* [n*q] outlet virtual-column values (outlet cells only) */
  long* src;      /* [n*q] state slot -> source: >= 0 fpost slot, -1 pinned inlet,
                     <= -2 vpost slot -(src+2) */
  long* dst;      /* [n*q] fpost slot -> state slot fed by it, or -1 (transpose of src) */
  long* vdst;     /* [n*q] vpost slot -> state slot fed by it, or -1 */
  /* objective */
  int obj_kind, obj_set;
  int lo[3], hi[3];
  double u0, p0;
  /* window */
  long nsamp;
  double* fsum;     /* [n*q] */
  double* gsum;     /* [n*q] sum of dJ/df */
  double* dJdd_sum; /* [n] */
  double* tau_sum;  /* [n] sum of tau_eff */
  double Jsum;
  /* adjoint */
  int adj_ready;
  double* jac;   /* [n*q*q] collision Jacobian dC_j/df_i */
  double* vjac;  /* [n*q*q] outlet Jacobian dV_j/df_i (outlet cells only) */
  double* dcdd;  /* [n*q] */
  double* gsrc;  /* [n*q] adjoint source dJ/df (mean or steady) */
  double* dJdd;  /* [n] explicit dJ/dd */
  double* phi;   /* [n*q] adjoint on post-collision slots */
  double* phiv;  /* [n*q] adjoint on outlet virtual slots */
  double* lam;   /* [n*q] */
  /* forward tangent fdot = (df/dd) v (App. C) */
  double* fdot;  /* [n*q] */
  double* tpost; /* [n*q] post-collision tangent */
  double* tvpost;/* [n*q] outlet virtual-column tangent */
};

/* ------------------------------------------------------------------------ */
/* Velocity sets (Sec. 2.1: D2Q9 and D3Q19).                                 */
/* ------------------------------------------------------------------------ */

void orc_stencil(int stencil, int* q, int* c, double* w, int* opp) {
  if (stencil == ORC_D2Q9) {
    static const int v[9][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}, {-1, 1},
                                {-1, 0}, {0, -1}, {-1, -1}, {1, -1}};
    *q = 9;
    for (int i = 0; i < 9; ++i) {
      c[3 * i + 0] = v[i][0];
      c[3 * i + 1] = v[i][1];
      c[3 * i + 2] = 0;
      int s = abs(v[i][0]) + abs(v[i][1]);
      w[i] = (s == 0) ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
      opp[i] = (i == 0) ? 0 : (i <= 4 ? i + 4 : i - 4);
    }
  } else {
    static const int v[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0},
                                 {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};
    *q = 19;
    for (int i = 0; i < 10; ++i)
      for (int a = 0; a < 3; ++a) c[3 * i + a] = v[i][a];
    for (int i = 1; i < 10; ++i)
      for (int a = 0; a < 3; ++a) c[3 * (i + 9) + a] = -v[i][a];
    for (int i = 0; i < 19; ++i) {
      int s = abs(c[3 * i]) + abs(c[3 * i + 1]) + abs(c[3 * i + 2]);
      w[i] = (s == 0) ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
      opp[i] = (i == 0) ? 0 : (i <= 9 ? i + 9 : i - 9);
    }
  }
}

typedef struct {
  int q, dim;
  int c[QMAX][3];
  double w[QMAX];
} stencil_t;

static stencil_t get_stencil(int stencil) {
  stencil_t s;
  int cc[3 * QMAX], opp[QMAX];
  orc_stencil(stencil, &s.q, cc, s.w, opp);
  s.dim = (stencil == ORC_D2Q9) ? 2 : 3;
  for (int i = 0; i < s.q; ++i)
    for (int a = 0; a < 3; ++a) s.c[i][a] = cc[3 * i + a];
  return s;
}

/* ------------------------------------------------------------------------ */
/* Moments and equilibrium (Sec. 2.1: f^eq, rho = sum f, u = sum xi f / rho) */
/* ------------------------------------------------------------------------ */

static void moments(const stencil_t* s, const double* f, double* rho, double j[3]) {
  double r = 0.0;
  j[0] = j[1] = j[2] = 0.0;
  for (int i = 0; i < s->q; ++i) {
    r += f[i];
    for (int a = 0; a < 3; ++a) j[a] += s->c[i][a] * f[i];
  }
  *rho = r;
}

/* f_i^eq(rho, v) = w_i rho (1 + xi.v/cs2 + (xi.v)^2/(2 cs2^2) - v.v/(2 cs2)), cs2 = 1/3 */
void orc_equilibrium(int stencil, double rho, const double* v, double* feq) {
  stencil_t s = get_stencil(stencil);
  double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  for (int i = 0; i < s.q; ++i) {
    double cv = s.c[i][0] * v[0] + s.c[i][1] * v[1] + s.c[i][2] * v[2];
    feq[i] = s.w[i] * rho * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
  }
}

/* Non-equilibrium momentum flux with respect to f^eq(rho, u):
 * Pi_ab = sum_i xi_ia xi_ib f_i - rho/3 delta_ab - j_a j_b / rho.
 * Evaluated as sum_i xi_ia xi_ib (f_i - w_i) - (rho - 1)/3 delta_ab - j_a j_b / rho,
 * the same number by sum_i w_i = 1 and sum_i w_i xi_ia xi_ib = delta_ab / 3,
 * without cancelling two O(1/3) terms. */
static void neq_flux(const stencil_t* s, const double* f, double Pi[3][3]) {
  double rho, j[3], drho = 0.0;
  moments(s, f, &rho, j);
  for (int i = 0; i < s->q; ++i) drho += f[i] - s->w[i];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Pi[a][b] = 0.0;
  for (int a = 0; a < s->dim; ++a)
    for (int b = 0; b < s->dim; ++b) {
      double m = 0.0;
      for (int i = 0; i < s->q; ++i) m += s->c[i][a] * s->c[i][b] * (f[i] - s->w[i]);
      Pi[a][b] = m - (a == b ? drho / 3.0 : 0.0) - j[a] * j[b] / rho;
    }
}

static double frob(double Pi[3][3]) {
  double ss = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) ss += Pi[a][b] * Pi[a][b];
  return sqrt(ss);
}

/* Smagorinsky effective relaxation time (Eqs. turbVisc, tauEff):
 * tau = tau0 + 3 nu_t, nu_t = Cs^2 |S|, |S| = sqrt(2 S:S), S = -3 Pi / (2 tau);
 * hence tau^2 - tau0 tau - (9 Cs^2 / sqrt 2) |Pi| = 0, positive root. */
static double tau_eff_s(const stencil_t* s, const double* f, double tau0, double cs) {
  if (cs == 0.0) return tau0;
  double Pi[3][3];
  neq_flux(s, f, Pi);
  double P = frob(Pi);
  return 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * P));
}

double orc_tau_eff(int stencil, const double* f, double tau0, double cs) {
  stencil_t s = get_stencil(stencil);
  return tau_eff_s(&s, f, tau0, cs);
}

/* ------------------------------------------------------------------------ */
/* Collision (Eq. hlbm): f*_i = f_i - (f_i - f_i^eq(rho, d u)) / tau_eff      */
/* plus a constant body force 3 w_i xi_i.G (tests only).                     */
/* ------------------------------------------------------------------------ */

static void collide_s(const stencil_t* s, const double* f, double d, double tau0, double cs,
                      const double* force, double* out) {
  double rho, j[3], ut[3], feq[QMAX];
  moments(s, f, &rho, j);
  for (int a = 0; a < 3; ++a) ut[a] = d * (j[a] / rho);
  double tau = tau_eff_s(s, f, tau0, cs);
  double vv = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  for (int i = 0; i < s->q; ++i) {
    double cv = s->c[i][0] * ut[0] + s->c[i][1] * ut[1] + s->c[i][2] * ut[2];
    feq[i] = s->w[i] * rho * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
  }
  for (int i = 0; i < s->q; ++i) {
    double fi = f[i] - (f[i] - feq[i]) / tau;
    if (force) {
      double cG = s->c[i][0] * force[0] + s->c[i][1] * force[1] + s->c[i][2] * force[2];
      fi += 3.0 * s->w[i] * cG;
    }
    out[i] = fi;
  }
}

void orc_collide_cell(int stencil, const double* f, double d, double tau0, double cs,
                      const double* force, double* out) {
  stencil_t s = get_stencil(stencil);
  collide_s(&s, f, d, tau0, cs, force, out);
}

/* ------------------------------------------------------------------------ */
/* Jacobian dC_j/df_i of the collision, written out with the chain rule      */
/* (Sec. 5.4: dC_j/df_i including the (1/tau)^2 dtau/df_i f^neq_j term).     */
/* ------------------------------------------------------------------------ */

/* d Pi_ab / d f_i = xi_ia xi_ib - delta_ab/3 - (xi_ia j_b + j_a xi_ib)/rho + j_a j_b / rho^2 */
static double dPi_df(const stencil_t* s, int i, int a, int b, double rho, const double* j) {
  return s->c[i][a] * s->c[i][b] - (a == b ? 1.0 / 3.0 : 0.0) -
         (s->c[i][a] * j[b] + j[a] * s->c[i][b]) / rho + j[a] * j[b] / (rho * rho);
}

static void jacobian_s(const stencil_t* s, const double* f, double d, double tau_a, double cs,
                       int turb, double tau_frozen, double* A) {
  int q = s->q;
  double rho, j[3], u[3], ut[3], feq[QMAX];
  moments(s, f, &rho, j);
  for (int a = 0; a < 3; ++a) {
    u[a] = j[a] / rho;
    ut[a] = d * u[a];
  }
  double vv = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  for (int k = 0; k < q; ++k) {
    double cv = s->c[k][0] * ut[0] + s->c[k][1] * ut[1] + s->c[k][2] * ut[2];
    feq[k] = s->w[k] * rho * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
  }
  double tau;
  int differentiated = (cs != 0.0 && turb == ORC_TURB_DIFFERENTIATED);
  if (cs == 0.0)
    tau = tau_a;
  else if (differentiated)
    tau = tau_eff_s(s, f, tau_a, cs);
  else
    tau = tau_frozen;

  /* dtau/df_i for the differentiated closure: tau = (tau_a + sqrt(tau_a^2 + k P))/2,
   * k = 18 sqrt2 Cs^2, P = |Pi|; dtau/df_i = k / (4 sqrt(tau_a^2 + k P)) dP/df_i,
   * dP/df_i = sum_ab Pi_ab dPi_ab/df_i / P (taken as 0 where P = 0). */
  double dtau[QMAX];
  for (int i = 0; i < q; ++i) dtau[i] = 0.0;
  if (differentiated) {
    double Pi[3][3];
    neq_flux(s, f, Pi);
    double P = frob(Pi);
    if (P > 0.0) {
      double k = 18.0 * sqrt(2.0) * cs * cs;
      double pre = k / (4.0 * sqrt(tau_a * tau_a + k * P));
      for (int i = 0; i < q; ++i) {
        double dP = 0.0;
        for (int a = 0; a < s->dim; ++a)
          for (int b = 0; b < s->dim; ++b) dP += Pi[a][b] * dPi_df(s, i, a, b, rho, j);
        dtau[i] = pre * dP / P;
      }
    }
  }

  for (int jj = 0; jj < q; ++jj) {
    /* f^eq_j = rho * phi_j(ut), phi_j = w_j (1 + 3 xi.ut + 4.5 (xi.ut)^2 - 1.5 ut.ut);
     * d phi_j / d ut_a = w_j (3 xi_a + 9 (xi.ut) xi_a - 3 ut_a);
     * d ut_a / d f_i = d (xi_ia - u_a) / rho. */
    double cv = s->c[jj][0] * ut[0] + s->c[jj][1] * ut[1] + s->c[jj][2] * ut[2];
    double dphi[3];
    for (int a = 0; a < 3; ++a)
      dphi[a] = s->w[jj] * (3.0 * s->c[jj][a] + 9.0 * cv * s->c[jj][a] - 3.0 * ut[a]);
    for (int i = 0; i < q; ++i) {
      double dfeq = feq[jj] / rho;
      for (int a = 0; a < 3; ++a) dfeq += rho * dphi[a] * d * (s->c[i][a] - u[a]) / rho;
      double val = (jj == i ? 1.0 : 0.0) - ((jj == i ? 1.0 : 0.0) - dfeq) / tau;
      val += (f[jj] - feq[jj]) / (tau * tau) * dtau[i];
      A[jj * q + i] = val;
    }
  }
}

void orc_jacobian_cell(int stencil, const double* f, double d, double tau_a, double cs, int turb,
                       double tau_frozen, double* A) {
  stencil_t s = get_stencil(stencil);
  jacobian_s(&s, f, d, tau_a, cs, turb, tau_frozen, A);
}

/* dC_j/dd = (1/tau) d f^eq_j / d d = (1/tau) rho sum_a dphi_j/d ut_a * u_a */
static void dcdd_s(const stencil_t* s, const double* f, double d, double tau_used, double* out) {
  double rho, j[3], u[3], ut[3];
  moments(s, f, &rho, j);
  for (int a = 0; a < 3; ++a) {
    u[a] = j[a] / rho;
    ut[a] = d * u[a];
  }
  for (int jj = 0; jj < s->q; ++jj) {
    double cv = s->c[jj][0] * ut[0] + s->c[jj][1] * ut[1] + s->c[jj][2] * ut[2];
    double acc = 0.0;
    for (int a = 0; a < 3; ++a)
      acc += s->w[jj] * (3.0 * s->c[jj][a] + 9.0 * cv * s->c[jj][a] - 3.0 * ut[a]) * u[a];
    out[jj] = rho * acc / tau_used;
  }
}

void orc_dcdd_cell(int stencil, const double* f, double d, double tau_used, double* out) {
  stencil_t s = get_stencil(stencil);
  dcdd_s(&s, f, d, tau_used, out);
}

/* ------------------------------------------------------------------------ */
/* HRRLBM collision (Sec. 2.2, Eq. HRRLBM), read as:                         */
/*   C_i = f_i^eq + (1 - 1/tau_eff) f_i^(1)                                  */
/*   f_i^eq  = w_i [rho + 3 xi_i.rho u~ + (9/2) H2_i:rho u~u~                 */
/*                  + (9/2) H3_i:rho u~u~u~],  u~ = d u                       */
/*   f_i^(1) = w_i [3 xi_i.a1 + (9/2) H2_i:a2 + (9/2) H3_i:a3]                */
/* with the Hermite coefficients of the non-equilibrium part f - f^eq:       */
/*   a0 = 0, a1 = j - rho u~ = (1 - d) j, a2 = sum_i H2_i f_i - rho u~u~      */
/*   (projections), a3_abg = u~_a a2_bg + u~_b a2_ag + u~_g a2_ab (recursive),*/
/* H2_i = xi_i xi_i - I/3, and the third order restricted to the components  */
/* H_aab = xi_b (xi_a^2 - 1/3), a != b, that the velocity set supports (each */
/* enters H3:a with multiplicity 3).  tau_eff: the Smagorinsky closure on    */
/* Pi of f^eq(rho, u) as for BGK.  Complex arithmetic: the exact Jacobian    */
/* dC/df and dC/dd follow by complex-step differentiation.                   */
/* ------------------------------------------------------------------------ */

static const int H3_TYPES_2D[2][2] = {{0, 1}, {1, 0}};
static const int H3_TYPES_3D[6][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 2}, {2, 0}, {2, 1}};

/* freeze: 0 -> tau_eff from the closure (or tau0 without it); 1 -> tau_frozen */
static void hrr_collide_z(const stencil_t* s, const double complex* f, double complex d, double tau0,
                          double cs, int freeze, double tau_frozen, const double* force,
                          double complex* out) {
  const int q = s->q, D = s->dim;
  double complex drho = 0.0, j[3] = {0.0, 0.0, 0.0}, S[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) S[a][b] = 0.0;
  for (int i = 0; i < q; ++i) {
    double complex g = f[i] - s->w[i]; /* shifted: sum w = 1, sum w xi xi = I/3 */
    drho += g;
    for (int a = 0; a < 3; ++a) j[a] += s->c[i][a] * f[i];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) S[a][b] += s->c[i][a] * s->c[i][b] * g;
  }
  double complex rho = 1.0 + drho, u[3], ut[3];
  for (int a = 0; a < 3; ++a) {
    u[a] = j[a] / rho;
    ut[a] = d * u[a];
  }
  double complex tau = tau0;
  if (freeze) {
    tau = tau_frozen;
  } else if (cs > 0.0) {
    double complex P2 = 0.0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) {
        double complex Pi = S[a][b] - (a == b ? drho / 3.0 : 0.0) - j[a] * j[b] / rho;
        P2 += Pi * Pi;
      }
    /* |Pi| = 0: no strain, tau_eff = tau0 and no derivative (as for BGK) */
    double complex P = (creal(P2) > 0.0) ? csqrt(P2) : 0.0;
    tau = 0.5 * (tau0 + csqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * P));
  }
  double complex a2[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      a2[a][b] = (a < D && b < D) ? S[a][b] - (a == b ? drho / 3.0 : 0.0) - rho * ut[a] * ut[b] : 0.0;
  const int nt = (D == 2) ? 2 : 6;
  const int(*T)[2] = (D == 2) ? H3_TYPES_2D : H3_TYPES_3D;
  for (int i = 0; i < q; ++i) {
    const int* c = s->c[i];
    double complex cu = 0.0, cj = 0.0, tt = 0.0;
    for (int a = 0; a < D; ++a) {
      cu += c[a] * ut[a];
      cj += c[a] * j[a];
      tt += ut[a] * ut[a];
    }
    double complex e2 = rho * (cu * cu - tt / 3.0), e3 = 0.0, n2 = 0.0, n3 = 0.0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) n2 += (c[a] * c[b] - (a == b ? 1.0 / 3.0 : 0.0)) * a2[a][b];
    for (int t = 0; t < nt; ++t) {
      const int a = T[t][0], b = T[t][1];
      const double H = c[b] * (c[a] * c[a] - 1.0 / 3.0);
      e3 += 3.0 * H * rho * ut[a] * ut[a] * ut[b];
      n3 += 3.0 * H * (2.0 * ut[a] * a2[a][b] + ut[b] * a2[a][a]);
    }
    double complex feq = s->w[i] * (rho + 3.0 * rho * cu + 4.5 * e2 + 4.5 * e3);
    double complex f1 = s->w[i] * (3.0 * (1.0 - d) * cj + 4.5 * n2 + 4.5 * n3);
    double complex v = feq + (1.0 - 1.0 / tau) * f1;
    if (force) v += 3.0 * s->w[i] * (c[0] * force[0] + c[1] * force[1] + c[2] * force[2]);
    out[i] = v;
  }
}

static void hrr_collide_s(const stencil_t* s, const double* f, double d, double tau0, double cs,
                          const double* force, double* out) {
  double complex fz[QMAX] = {0}, oz[QMAX] = {0};
  for (int i = 0; i < s->q; ++i) fz[i] = f[i];
  hrr_collide_z(s, fz, d, tau0, cs, 0, 0.0, force, oz);
  for (int i = 0; i < s->q; ++i) out[i] = creal(oz[i]);
}

#define CSTEP 1e-30

/* A[j*q + i] = dC_j/df_i by complex steps f_i + i h (turb FROZEN: tau_frozen). */
static void hrr_jacobian_s(const stencil_t* s, const double* f, double d, double tau_a, double cs,
                           int turb, double tau_frozen, double* A) {
  const int q = s->q;
  const int freeze = (cs > 0.0 && turb == ORC_TURB_FROZEN);
  double complex fz[QMAX] = {0}, oz[QMAX] = {0};
  for (int i = 0; i < q; ++i) {
    for (int k = 0; k < q; ++k) fz[k] = f[k];
    fz[i] = CMPLX(f[i], CSTEP);
    hrr_collide_z(s, fz, d, tau_a, cs, freeze, tau_frozen, NULL, oz);
    for (int jj = 0; jj < q; ++jj) A[jj * q + i] = cimag(oz[jj]) / CSTEP;
  }
}

/* dC_j/dd by a complex step in d (tau_eff does not depend on d). */
static void hrr_dcdd_s(const stencil_t* s, const double* f, double d, double tau_a, double cs,
                       int freeze, double tau_frozen, double* out) {
  double complex fz[QMAX] = {0}, oz[QMAX] = {0};
  for (int i = 0; i < s->q; ++i) fz[i] = f[i];
  hrr_collide_z(s, fz, CMPLX(d, CSTEP), tau_a, cs, freeze, tau_frozen, NULL, oz);
  for (int jj = 0; jj < s->q; ++jj) out[jj] = cimag(oz[jj]) / CSTEP;
}

void orc_hrr_collide_cell(int stencil, const double* f, double d, double tau0, double cs,
                          const double* force, double* out) {
  stencil_t s = get_stencil(stencil);
  hrr_collide_s(&s, f, d, tau0, cs, force, out);
}

void orc_hrr_jacobian_cell(int stencil, const double* f, double d, double tau_a, double cs, int turb,
                           double tau_frozen, double* A) {
  stencil_t s = get_stencil(stencil);
  hrr_jacobian_s(&s, f, d, tau_a, cs, turb, tau_frozen, A);
}

void orc_hrr_dcdd_cell(int stencil, const double* f, double d, double tau_a, double cs, int turb,
                       double tau_frozen, double* out) {
  stencil_t s = get_stencil(stencil);
  hrr_dcdd_s(&s, f, d, tau_a, cs, cs > 0.0 && turb == ORC_TURB_FROZEN, tau_frozen, out);
}

/* ------------------------------------------------------------------------ */
/* Objectives (Sec. 4) per cell and their partial derivatives.               */
/*  FFA  (Eq. obj_ffa):  rho (u_x u0 - u_x^2) + p0 - p,  p = rho/3           */
/*  DISS (Eq. obj_diss): 2 nu S:S + (nu/K) u.u,  S = -Pi/(2 tau0 cs2),       */
/*                       nu = (tau0 - 1/2)/3,  nu/K = (1-d)/tau0             */
/*  MOMENTUM (test):     j_x                                                 */
/* ------------------------------------------------------------------------ */

static double objective_cell_s(const stencil_t* s, int kind, const double* f, double d,
                               double tau0, double u0, double p0) {
  double rho, j[3];
  moments(s, f, &rho, j);
  if (kind == ORC_OBJ_FFA) {
    double ux = j[0] / rho;
    return rho * (ux * u0 - ux * ux) + (p0 - rho / 3.0);
  }
  if (kind == ORC_OBJ_DISS) {
    double Pi[3][3];
    neq_flux(s, f, Pi);
    double nu = (tau0 - 0.5) / 3.0;
    double SS = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double S = -Pi[a][b] / (2.0 * tau0 / 3.0);
        SS += S * S;
      }
    double uu = 0.0;
    for (int a = 0; a < 3; ++a) uu += (j[a] / rho) * (j[a] / rho);
    return 2.0 * nu * SS + (1.0 - d) / tau0 * uu;
  }
  return j[0];
}

double orc_objective_cell(int stencil, int kind, const double* f, double d, double tau0,
                          double u0, double p0) {
  stencil_t s = get_stencil(stencil);
  return objective_cell_s(&s, kind, f, d, tau0, u0, p0);
}

static void dJdf_s(const stencil_t* s, int kind, const double* f, double d, double tau0,
                   double u0, double p0, double* out) {
  (void)p0;
  double rho, j[3];
  moments(s, f, &rho, j);
  if (kind == ORC_OBJ_FFA) {
    /* J = j_x u0 - j_x^2/rho + p0 - rho/3 */
    for (int i = 0; i < s->q; ++i)
      out[i] = s->c[i][0] * u0 - 2.0 * j[0] * s->c[i][0] / rho + j[0] * j[0] / (rho * rho) -
               1.0 / 3.0;
    return;
  }
  if (kind == ORC_OBJ_DISS) {
    /* J = (2 nu / (2 tau0/3)^2) Pi:Pi + ((1-d)/tau0) j.j / rho^2 */
    double Pi[3][3];
    neq_flux(s, f, Pi);
    double nu = (tau0 - 0.5) / 3.0;
    double cS = 2.0 * nu / ((2.0 * tau0 / 3.0) * (2.0 * tau0 / 3.0));
    double cD = (1.0 - d) / tau0;
    for (int i = 0; i < s->q; ++i) {
      double acc = 0.0;
      for (int a = 0; a < s->dim; ++a)
        for (int b = 0; b < s->dim; ++b) acc += 2.0 * Pi[a][b] * dPi_df(s, i, a, b, rho, j);
      double duu = 0.0;
      for (int a = 0; a < 3; ++a)
        duu += 2.0 * (j[a] / rho) * (s->c[i][a] / rho - j[a] / (rho * rho));
      out[i] = cS * acc + cD * duu;
    }
    return;
  }
  for (int i = 0; i < s->q; ++i) out[i] = s->c[i][0];
}

void orc_dJdf_cell(int stencil, int kind, const double* f, double d, double tau0, double u0,
                   double p0, double* out) {
  stencil_t s = get_stencil(stencil);
  dJdf_s(&s, kind, f, d, tau0, u0, p0, out);
}

static double dJdd_s(const stencil_t* s, int kind, const double* f, double d, double tau0) {
  (void)d;
  if (kind != ORC_OBJ_DISS) return 0.0;
  double rho, j[3];
  moments(s, f, &rho, j);
  double uu = 0.0;
  for (int a = 0; a < 3; ++a) uu += (j[a] / rho) * (j[a] / rho);
  return -uu / tau0;
}

double orc_dJdd_cell(int stencil, int kind, const double* f, double d, double tau0) {
  stencil_t s = get_stencil(stencil);
  return dJdd_s(&s, kind, f, d, tau0);
}

/* ------------------------------------------------------------------------ */
/* Outlet: a pressure outlet (density 1, as the paper's p_out) whose         */
/* velocity has zero gradient.  A virtual column x = nx holds the values     */
/* V_i = f_i^eq(1, u) with u the velocity of the last column; the missing    */
/* populations of the last column stream in from it.                        */
/* ------------------------------------------------------------------------ */

static void outlet_values_s(const stencil_t* s, const double* f, double* out) {
  double rho, j[3], u[3];
  moments(s, f, &rho, j);
  for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < s->q; ++i) {
    double cu = s->c[i][0] * u[0] + s->c[i][1] * u[1] + s->c[i][2] * u[2];
    out[i] = s->w[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* dV_j/df_i = w_j (3 xi_j + 9 (xi_j.u) xi_j - 3 u) . (xi_i - u) / rho */
static void outlet_jacobian_s(const stencil_t* s, const double* f, double* B) {
  int q = s->q;
  double rho, j[3], u[3];
  moments(s, f, &rho, j);
  for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
  for (int jj = 0; jj < q; ++jj) {
    double cu = s->c[jj][0] * u[0] + s->c[jj][1] * u[1] + s->c[jj][2] * u[2];
    for (int i = 0; i < q; ++i) {
      double acc = 0.0;
      for (int a = 0; a < 3; ++a)
        acc += s->w[jj] * (3.0 * s->c[jj][a] + 9.0 * cu * s->c[jj][a] - 3.0 * u[a]) *
               (s->c[i][a] - u[a]) / rho;
      B[jj * q + i] = acc;
    }
  }
}

void orc_outlet_values_cell(int stencil, const double* f, double* out) {
  stencil_t s = get_stencil(stencil);
  outlet_values_s(&s, f, out);
}

void orc_outlet_jacobian_cell(int stencil, const double* f, double* B) {
  stencil_t s = get_stencil(stencil);
  outlet_jacobian_s(&s, f, B);
}

/* ------------------------------------------------------------------------ */
/* Lattice: geometry, streaming table, inlet.                                */
/* ------------------------------------------------------------------------ */

static stencil_t lat_stencil(const orc_lattice* L) { return get_stencil(L->p.stencil); }

static long cell_index(const orc_lattice* L, int x, int y, int z) {
  return (long)x + (long)L->p.nx * ((long)y + (long)L->p.ny * (long)z);
}

static void cell_coords(const orc_lattice* L, long c, int* x, int* y, int* z) {
  *x = (int)(c % L->p.nx);
  long r = c / L->p.nx;
  *y = (int)(r % L->p.ny);
  *z = (int)(r / L->p.ny);
}

static int is_inlet(const orc_lattice* L, long c) {
  return L->p.bc_x == ORC_BC_INLET_OUTLET && (c % L->p.nx) == 0;
}

static int is_outlet(const orc_lattice* L, long c) {
  return L->p.bc_x == ORC_BC_INLET_OUTLET && (c % L->p.nx) == L->p.nx - 1;
}

/* Inlet velocity profile u_in(y) (parabola vanishing at the halfway walls). */
static double inlet_u(const orc_lattice* L, int y) {
  if (L->p.inlet_profile == ORC_INLET_PARABOLIC) {
    double H = (double)L->p.ny;
    return 4.0 * L->p.u_in * (y + 0.5) * (H - 0.5 - y) / (H * H);
  }
  return L->p.u_in;
}

static void inlet_feq(const orc_lattice* L, long c, double* feq) {
  int x, y, z;
  cell_coords(L, c, &x, &y, &z);
  double v[3] = {inlet_u(L, y), 0.0, 0.0};
  orc_equilibrium(L->p.stencil, 1.0, v, feq);
}

/* Streaming with halfway bounce-back walls, periodic axes, a pinned
 * equilibrium inlet column x = 0 and the outlet above at x = nx-1.
 * Bounce-back takes precedence where a source crosses a wall. */
static void build_stream_table(orc_lattice* L) {
  stencil_t s = lat_stencil(L);
  int q = s.q;
  int n3[3] = {L->p.nx, L->p.ny, L->p.nz};
  int bc[3] = {L->p.bc_x, L->p.bc_y, L->p.bc_z};
  for (long c = 0; c < L->n; ++c) {
    int x[3];
    cell_coords(L, c, &x[0], &x[1], &x[2]);
    for (int i = 0; i < q; ++i) {
      long slot = c * q + i;
      if (is_inlet(L, c)) {
        L->src[slot] = -1;
        continue;
      }
      int sp[3];
      int bounce = 0, outlet = 0;
      for (int a = 0; a < 3; ++a) {
        sp[a] = x[a] - s.c[i][a];
        if (sp[a] < 0 || sp[a] >= n3[a]) {
          if (bc[a] == ORC_BC_PERIODIC)
            sp[a] = (sp[a] + n3[a]) % n3[a];
          else if (bc[a] == ORC_BC_WALLS)
            bounce = 1;
          else /* inlet/outlet axis (x only); sp < 0 only for the inlet column */
            outlet = (sp[a] >= n3[a]);
        }
      }
      if (bounce)
        L->src[slot] = c * q + L->opp[i];
      else if (outlet) /* virtual column nx, fed by the last column at (sp_y, sp_z) */
        L->src[slot] = -2 - (cell_index(L, n3[0] - 1, sp[1], sp[2]) * q + i);
      else
        L->src[slot] = cell_index(L, sp[0], sp[1], sp[2]) * q + i;
    }
  }
  /* explicit transpose */
  for (long k = 0; k < L->n * q; ++k) {
    L->dst[k] = -1;
    L->vdst[k] = -1;
  }
  for (long slot = 0; slot < L->n * q; ++slot) {
    long sidx = L->src[slot];
    if (sidx >= 0)
      L->dst[sidx] = slot;
    else if (sidx <= -2)
      L->vdst[-2 - sidx] = slot;
  }
}

orc_lattice* orc_create(const orc_params* p) {
  if (!p || !(p->tau > 0.5) || p->nx < 2 || p->ny < 1 || p->nz < 1) return NULL;
  if (p->stencil != ORC_D2Q9 && p->stencil != ORC_D3Q19) return NULL;
  if (p->stencil == ORC_D2Q9 && p->nz != 1) return NULL;
  if (p->bc_y == ORC_BC_INLET_OUTLET || p->bc_z == ORC_BC_INLET_OUTLET) return NULL;
  if (p->collision != ORC_COLL_BGK && p->collision != ORC_COLL_HRR) return NULL;
  orc_lattice* L = (orc_lattice*)calloc(1, sizeof(orc_lattice));
  L->p = *p;
  if (L->p.stencil == ORC_D2Q9) L->p.bc_z = ORC_BC_PERIODIC;
  int cc[3 * QMAX];
  orc_stencil(p->stencil, &L->q, cc, L->w, L->opp);
  for (int i = 0; i < L->q; ++i)
    for (int a = 0; a < 3; ++a) L->c[i][a] = cc[3 * i + a];
  L->n = (long)p->nx * p->ny * p->nz;
  long nq = L->n * L->q;
  L->d = (double*)malloc(sizeof(double) * L->n);
  L->f = (double*)calloc(nq, sizeof(double));
  L->fpost = (double*)calloc(nq, sizeof(double));
  L->vpost = (double*)calloc(nq, sizeof(double));
  L->src = (long*)malloc(sizeof(long) * nq);
  L->dst = (long*)malloc(sizeof(long) * nq);
  L->vdst = (long*)malloc(sizeof(long) * nq);
  L->fsum = (double*)calloc(nq, sizeof(double));
  L->gsum = (double*)calloc(nq, sizeof(double));
  L->dJdd_sum = (double*)calloc(L->n, sizeof(double));
  L->tau_sum = (double*)calloc(L->n, sizeof(double));
  for (long c = 0; c < L->n; ++c) L->d[c] = 1.0;
  build_stream_table(L);
  orc_init_equilibrium(L, 1.0, NULL);
  return L;
}

void orc_destroy(orc_lattice* L) {
  if (!L) return;
  free(L->d); free(L->f); free(L->fpost); free(L->vpost);
  free(L->src); free(L->dst); free(L->vdst);
  free(L->fsum); free(L->gsum); free(L->dJdd_sum); free(L->tau_sum);
  free(L->jac); free(L->vjac); free(L->dcdd); free(L->gsrc); free(L->dJdd);
  free(L->fdot); free(L->tpost); free(L->tvpost);
  free(L->phi); free(L->phiv); free(L->lam);
  free(L);
}

int orc_q(const orc_lattice* L) { return L->q; }
long orc_n(const orc_lattice* L) { return L->n; }

int orc_set_porosity(orc_lattice* L, const double* d) {
  for (long c = 0; c < L->n; ++c) {
    if (!(d[c] >= 0.0 && d[c] <= 1.0)) return -1;
  }
  memcpy(L->d, d, sizeof(double) * L->n);
  L->adj_ready = 0;
  return 0;
}

int orc_get_porosity(const orc_lattice* L, double* d) {
  memcpy(d, L->d, sizeof(double) * L->n);
  return 0;
}

/* Porous cylinder: solid fraction chi = 1 inside r <= R-1, half-cosine ramp
 * chi = (1 + cos(pi (r - R + 1)/2))/2 on R-1 < r < R+1, 0 outside; d = 1 - chi
 * (Sec. 5.1: d = 0 in the cylinder, d = 1 in the fluid). */
int orc_build_cylinder(orc_lattice* L, double xc, double yc, double D, const double* noise,
                       int noise_mode, double box_half, double d_solid) {
  const double pi = 3.14159265358979323846;
  double R = 0.5 * D;
  for (long c = 0; c < L->n; ++c) {
    int x, y, z;
    cell_coords(L, c, &x, &y, &z);
    double dx = x - xc, dy = y - yc;
    double r = sqrt(dx * dx + dy * dy);
    double chi;
    if (r <= R - 1.0)
      chi = 1.0;
    else if (r >= R + 1.0)
      chi = 0.0;
    else
      chi = 0.5 * (1.0 + cos(pi * (r - R + 1.0) / 2.0));
    double d = 1.0 - chi;
    if (noise && noise_mode == ORC_NOISE_RIM && chi > 0.0 && chi < 1.0) {
      d += noise[c];
      if (d < 0.0) d = 0.0;
      if (d > 1.0) d = 1.0;
    } else if (noise && noise_mode == ORC_NOISE_BOX && fabs(dx) <= box_half &&
               fabs(dy) <= box_half) {
      double ch = chi + noise[c];
      if (ch < 0.0) ch = 0.0;
      if (ch > 1.0) ch = 1.0;
      d = 1.0 - ch;
    }
    /* permeable cylinder: porosity d_solid where chi = 1 (d_solid = 0 leaves
       d untouched) */
    if (d_solid != 0.0) d = 1.0 - (1.0 - d) * (1.0 - d_solid);
    L->d[c] = d;
  }
  L->adj_ready = 0;
  return 0;
}

int orc_init_equilibrium(orc_lattice* L, double rho0, const double* u) {
  int q = L->q;
  for (long c = 0; c < L->n; ++c) {
    double* fc = L->f + c * q;
    if (is_inlet(L, c)) {
      inlet_feq(L, c, fc);
      continue;
    }
    int x, y, z;
    cell_coords(L, c, &x, &y, &z);
    double v[3] = {0.0, 0.0, 0.0};
    if (u) {
      for (int a = 0; a < 3; ++a) v[a] = u[a * L->n + c];
    } else if (L->p.bc_x == ORC_BC_INLET_OUTLET) {
      v[0] = inlet_u(L, y);
    }
    for (int a = 0; a < 3; ++a) v[a] *= L->d[c];
    orc_equilibrium(L->p.stencil, rho0, v, fc);
  }
  return 0;
}

int orc_set_populations(orc_lattice* L, const double* f) {
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < L->q; ++i) L->f[c * L->q + i] = f[(long)i * L->n + c];
  return 0;
}

int orc_get_populations(const orc_lattice* L, double* f) {
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < L->q; ++i) f[(long)i * L->n + c] = L->f[c * L->q + i];
  return 0;
}

/* One time step: collide every cell into fpost (and the outlet cells'
 * virtual values into vpost), then pull every state slot through the table. */
static void step_once(orc_lattice* L) {
  stencil_t s = lat_stencil(L);
  int q = s.q;
  const double* force = L->p.force;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < L->n; ++c) {
    if (is_inlet(L, c)) {
      inlet_feq(L, c, L->fpost + c * q);
      continue;
    }
    if (L->p.collision == ORC_COLL_HRR)
      hrr_collide_s(&s, L->f + c * q, L->d[c], L->p.tau, L->p.cs, force, L->fpost + c * q);
    else
      collide_s(&s, L->f + c * q, L->d[c], L->p.tau, L->p.cs, force, L->fpost + c * q);
    if (is_outlet(L, c)) outlet_values_s(&s, L->f + c * q, L->vpost + c * q);
  }
#pragma omp parallel for schedule(static)
  for (long c = 0; c < L->n; ++c) {
    if (is_inlet(L, c)) {
      inlet_feq(L, c, L->f + c * q);
      continue;
    }
    for (int i = 0; i < q; ++i) {
      long sidx = L->src[c * q + i];
      L->f[c * q + i] = (sidx >= 0) ? L->fpost[sidx] : L->vpost[-2 - sidx];
    }
  }
}

int orc_step(orc_lattice* L, long nsteps) {
  for (long t = 0; t < nsteps; ++t) step_once(L);
  return 0;
}

int orc_moments(const orc_lattice* L, double* rho, double* u) {
  stencil_t s = lat_stencil(L);
  for (long c = 0; c < L->n; ++c) {
    double r, j[3];
    moments(&s, L->f + c * s.q, &r, j);
    if (rho) rho[c] = r;
    if (u)
      for (int a = 0; a < 3; ++a) u[a * L->n + c] = j[a] / r;
  }
  return 0;
}

long orc_run_steady(orc_lattice* L, long max_steps, double tol, long check_every) {
  long n = L->n;
  double* uprev = (double*)malloc(sizeof(double) * 3 * n);
  double* ucur = (double*)malloc(sizeof(double) * 3 * n);
  orc_moments(L, NULL, uprev);
  long t = 0;
  if (check_every < 1) check_every = 1;
  while (t < max_steps) {
    long k = check_every;
    if (t + k > max_steps) k = max_steps - t;
    orc_step(L, k);
    t += k;
    orc_moments(L, NULL, ucur);
    double dmax = 0.0, umax = 0.0;
    for (long m = 0; m < 3 * n; ++m) {
      double dd = fabs(ucur[m] - uprev[m]);
      if (dd > dmax) dmax = dd;
      if (fabs(ucur[m]) > umax) umax = fabs(ucur[m]);
    }
    memcpy(uprev, ucur, sizeof(double) * 3 * n);
    if (dmax <= tol * umax) break;
  }
  free(uprev);
  free(ucur);
  return t;
}

/* ------------------------------------------------------------------------ */
/* Objective over the region and the tracking average (Sec. 3.3).            */
/* ------------------------------------------------------------------------ */

static int in_region(const orc_lattice* L, long c) {
  int x[3];
  cell_coords(L, c, &x[0], &x[1], &x[2]);
  for (int a = 0; a < 3; ++a)
    if (x[a] < L->lo[a] || x[a] > L->hi[a]) return 0;
  return 1;
}

int orc_set_objective(orc_lattice* L, int kind, const int* lo, const int* hi, double u0,
                      double p0) {
  int n3[3] = {L->p.nx, L->p.ny, L->p.nz};
  if (kind < ORC_OBJ_FFA || kind > ORC_OBJ_MEA) return -1;
  if (kind == ORC_OBJ_MEA && !(u0 > 0.0)) return -1; /* u0 = surface area A */
  for (int a = 0; a < 3; ++a) {
    if (lo[a] < 0 || hi[a] >= n3[a] || lo[a] > hi[a]) return -1;
  }
  if (L->p.bc_x == ORC_BC_INLET_OUTLET && lo[0] < 1) return -1; /* inlet column is not state */
  L->obj_kind = kind;
  for (int a = 0; a < 3; ++a) {
    L->lo[a] = lo[a];
    L->hi[a] = hi[a];
  }
  L->u0 = u0;
  L->p0 = p0;
  L->obj_set = 1;
  L->adj_ready = 0;
  return 0;
}

/* Lattice neighbour x + xi_i (periodic axes wrap), or -1 when that position
 * is not a lattice cell (across a wall, beyond either x end). */
static long lattice_neighbour(const orc_lattice* L, long c, int i) {
  int n3[3] = {L->p.nx, L->p.ny, L->p.nz};
  int bc[3] = {L->p.bc_x, L->p.bc_y, L->p.bc_z};
  int x[3];
  cell_coords(L, c, &x[0], &x[1], &x[2]);
  for (int a = 0; a < 3; ++a) {
    x[a] += L->c[i][a];
    if (x[a] < 0 || x[a] >= n3[a]) {
      if (bc[a] != ORC_BC_PERIODIC) return -1;
      x[a] = (x[a] + n3[a]) % n3[a];
    }
  }
  return cell_index(L, x[0], x[1], x[2]);
}

/* Surface node set of J_MEA (Sec. 4): the cylinder's boundary nodes, read
 * for a porosity field as cells with d < 1/2 that have a lattice neighbour
 * with d >= 1/2, taken inside the objective box and one cell away from its
 * faces (on axes the box does not span completely), so that every
 * neighbour the functional reads lies in the box as well. */
static int mea_surface(const orc_lattice* L, long c) {
  int n3[3] = {L->p.nx, L->p.ny, L->p.nz};
  int x[3];
  cell_coords(L, c, &x[0], &x[1], &x[2]);
  for (int a = 0; a < 3; ++a) {
    int lo = L->lo[a], hi = L->hi[a];
    if (!(lo == 0 && hi == n3[a] - 1)) {
      lo += 1;
      hi -= 1;
    }
    if (x[a] < lo || x[a] > hi) return 0;
  }
  if (L->d[c] >= 0.5) return 0;
  for (int i = 1; i < L->q; ++i) {
    long nb = lattice_neighbour(L, c, i);
    if (nb >= 0 && L->d[nb] >= 0.5) return 1;
  }
  return 0;
}

/* J_MEA = (1/A) sum_{x in surface} sum_i xi_i,x (f_i(x + xi_i) - f_opp(i)(x)),
 * the x component (n = e_x) of the momentum exchanged across the surface
 * (Sec. 4, Eq. obj_mea), on the post-stream state; a neighbour that is not
 * a lattice cell contributes nothing. */
static double mea_objective(const orc_lattice* L) {
  int q = L->q;
  double J = 0.0;
  for (long c = 0; c < L->n; ++c) {
    if (!mea_surface(L, c)) continue;
    for (int i = 0; i < q; ++i) {
      long nb = lattice_neighbour(L, c, i);
      double fi = (nb >= 0) ? L->f[nb * q + i] : 0.0;
      J += L->c[i][0] * (fi - L->f[c * q + L->opp[i]]);
    }
  }
  return J / L->u0;
}

/* dJ_MEA/df: J is linear in f; every term xi_i,x f_i(x + xi_i) / A and
 * -xi_i,x f_opp(i)(x) / A adds its coefficient to the slot it reads.
 * g is slot-major [c*q + i]. */
static void mea_source_slots(const orc_lattice* L, double* g) {
  int q = L->q;
  memset(g, 0, sizeof(double) * L->n * q);
  for (long c = 0; c < L->n; ++c) {
    if (!mea_surface(L, c)) continue;
    for (int i = 0; i < q; ++i) {
      long nb = lattice_neighbour(L, c, i);
      if (nb >= 0) g[nb * q + i] += L->c[i][0] / L->u0;
      g[c * q + L->opp[i]] -= L->c[i][0] / L->u0;
    }
  }
}

int orc_mea_surface(const orc_lattice* L, unsigned char* flags) {
  if (!L->obj_set) return -1;
  for (long c = 0; c < L->n; ++c) flags[c] = (unsigned char)mea_surface(L, c);
  return 0;
}

int orc_mea_source(const orc_lattice* L, double* g) {
  if (!L->obj_set || L->obj_kind != ORC_OBJ_MEA) return -1;
  double* t = (double*)malloc(sizeof(double) * L->n * L->q);
  mea_source_slots(L, t);
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < L->q; ++i) g[(long)i * L->n + c] = t[c * L->q + i];
  free(t);
  return 0;
}

double orc_objective(const orc_lattice* L) {
  if (L->obj_kind == ORC_OBJ_MEA) return mea_objective(L);
  stencil_t s = lat_stencil(L);
  double J = 0.0;
  for (long c = 0; c < L->n; ++c)
    if (in_region(L, c))
      J += objective_cell_s(&s, L->obj_kind, L->f + c * s.q, L->d[c], L->p.tau, L->u0, L->p0);
  return J;
}

void orc_window_reset(orc_lattice* L) {
  long nq = L->n * L->q;
  memset(L->fsum, 0, sizeof(double) * nq);
  memset(L->gsum, 0, sizeof(double) * nq);
  memset(L->dJdd_sum, 0, sizeof(double) * L->n);
  memset(L->tau_sum, 0, sizeof(double) * L->n);
  L->Jsum = 0.0;
  L->nsamp = 0;
}

/* One sample t of the window: f(., t), J(t), dJ/df(t), dJ/dd(t), tau_eff(t). */
void orc_window_sample(orc_lattice* L) {
  stencil_t s = lat_stencil(L);
  int q = s.q;
  double g[QMAX];
  const int mea = L->obj_set && L->obj_kind == ORC_OBJ_MEA;
  if (mea) { /* dJ_MEA/df is constant; dJ_MEA/dd = 0 */
    double* t = (double*)malloc(sizeof(double) * L->n * q);
    mea_source_slots(L, t);
    for (long k = 0; k < L->n * q; ++k) L->gsum[k] += t[k];
    free(t);
  }
  for (long c = 0; c < L->n; ++c) {
    const double* fc = L->f + c * q;
    for (int i = 0; i < q; ++i) L->fsum[c * q + i] += fc[i];
    L->tau_sum[c] += tau_eff_s(&s, fc, L->p.tau, L->p.cs);
    if (L->obj_set && !mea && in_region(L, c)) {
      dJdf_s(&s, L->obj_kind, fc, L->d[c], L->p.tau, L->u0, L->p0, g);
      for (int i = 0; i < q; ++i) L->gsum[c * q + i] += g[i];
      L->dJdd_sum[c] += dJdd_s(&s, L->obj_kind, fc, L->d[c], L->p.tau);
    }
  }
  if (L->obj_set) L->Jsum += orc_objective(L);
  L->nsamp += 1;
}

long orc_window_count(const orc_lattice* L) { return L->nsamp; }

double orc_window_objective(const orc_lattice* L) {
  return L->nsamp ? L->Jsum / (double)L->nsamp : 0.0;
}

int orc_window_mean_populations(const orc_lattice* L, double* fbar) {
  if (!L->nsamp) return -1;
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < L->q; ++i)
      fbar[(long)i * L->n + c] = L->fsum[c * L->q + i] / (double)L->nsamp;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint (Eqs. adjoint_steady / adjoint_unsteady) and gradient (Eqs.       */
/* gradients_steady / gradients_unsteady).                                   */
/* ------------------------------------------------------------------------ */

int orc_adjoint_prepare(orc_lattice* L, int source, double tau_adj, int turb) {
  if (!L->obj_set) return -1;
  if (source == 1 && L->nsamp == 0) return -1;
  stencil_t s = lat_stencil(L);
  int q = s.q;
  long nq = L->n * q;
  double tau0 = L->p.tau;
  double ta = (tau_adj > 0.0) ? tau_adj : tau0;
  if (!L->jac) {
    L->jac = (double*)malloc(sizeof(double) * nq * q);
    L->vjac = (double*)calloc(nq * q, sizeof(double));
    L->dcdd = (double*)malloc(sizeof(double) * nq);
    L->gsrc = (double*)malloc(sizeof(double) * nq);
    L->dJdd = (double*)malloc(sizeof(double) * L->n);
    L->phi = (double*)calloc(nq, sizeof(double));
    L->phiv = (double*)calloc(nq, sizeof(double));
    L->lam = (double*)calloc(nq, sizeof(double));
  }
  double inv = (source == 1) ? 1.0 / (double)L->nsamp : 1.0;
  const int mea = L->obj_kind == ORC_OBJ_MEA;
  double* gmea = NULL;
  if (mea) {
    gmea = (double*)malloc(sizeof(double) * nq);
    if (source == 1)
      for (long k = 0; k < nq; ++k) gmea[k] = L->gsum[k] * inv;
    else
      mea_source_slots(L, gmea);
  }
#pragma omp parallel for schedule(static)
  for (long c = 0; c < L->n; ++c) {
    double fs[QMAX];
    double* A = L->jac + c * q * q;
    if (is_inlet(L, c)) {
      for (int k = 0; k < q * q; ++k) A[k] = 0.0;
      for (int i = 0; i < q; ++i) {
        L->dcdd[c * q + i] = 0.0;
        L->gsrc[c * q + i] = 0.0;
      }
      L->dJdd[c] = 0.0;
      continue;
    }
    for (int i = 0; i < q; ++i)
      fs[i] = (source == 1) ? L->fsum[c * q + i] * inv : L->f[c * q + i];
    double tau_mean = (source == 1) ? L->tau_sum[c] * inv : tau_eff_s(&s, fs, tau0, L->p.cs);
    double tau_frozen = ta + (tau_mean - tau0);
    const int hrr = (L->p.collision == ORC_COLL_HRR);
    if (hrr)
      hrr_jacobian_s(&s, fs, L->d[c], ta, L->p.cs, turb, tau_frozen, A);
    else
      jacobian_s(&s, fs, L->d[c], ta, L->p.cs, turb, tau_frozen, A);
    if (is_outlet(L, c)) outlet_jacobian_s(&s, fs, L->vjac + c * q * q);
    double tau_used;
    if (L->p.cs == 0.0)
      tau_used = ta;
    else if (turb == ORC_TURB_DIFFERENTIATED)
      tau_used = tau_eff_s(&s, fs, ta, L->p.cs);
    else
      tau_used = tau_frozen;
    if (hrr)
      hrr_dcdd_s(&s, fs, L->d[c], ta, L->p.cs, L->p.cs > 0.0 && turb == ORC_TURB_FROZEN, tau_frozen,
                 L->dcdd + c * q);
    else
      dcdd_s(&s, fs, L->d[c], tau_used, L->dcdd + c * q);
    if (mea) { /* a source on the surface cells and their neighbours */
      for (int i = 0; i < q; ++i) L->gsrc[c * q + i] = gmea[c * q + i];
      L->dJdd[c] = 0.0;
    } else if (in_region(L, c)) {
      if (source == 1) {
        for (int i = 0; i < q; ++i) L->gsrc[c * q + i] = L->gsum[c * q + i] * inv;
        L->dJdd[c] = L->dJdd_sum[c] * inv;
      } else {
        dJdf_s(&s, L->obj_kind, fs, L->d[c], tau0, L->u0, L->p0, L->gsrc + c * q);
        L->dJdd[c] = dJdd_s(&s, L->obj_kind, fs, L->d[c], tau0);
      }
    } else {
      for (int i = 0; i < q; ++i) L->gsrc[c * q + i] = 0.0;
      L->dJdd[c] = 0.0;
    }
  }
  free(gmea);
  L->adj_ready = 1;
  orc_adjoint_reset(L);
  return 0;
}

void orc_adjoint_reset(orc_lattice* L) {
  if (L->phi) memset(L->phi, 0, sizeof(double) * L->n * L->q);
  if (L->phiv) memset(L->phiv, 0, sizeof(double) * L->n * L->q);
}

/* lambda_i(x) = sum_j dC_j/df_i(x) phi_j(x) + sum_j dV_j/df_i(x) phiv_j(x) - dJ/df_i(x)
 * (the second sum only on outlet cells); then (phi, phiv) = S^T lambda. */
static void adjoint_once(orc_lattice* L) {
  int q = L->q;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < L->n; ++c) {
    const double* A = L->jac + c * q * q;
    const double* ph = L->phi + c * q;
    int out = is_outlet(L, c);
    const double* B = L->vjac + c * q * q;
    const double* pv = L->phiv + c * q;
    for (int i = 0; i < q; ++i) {
      double acc = 0.0;
      for (int jj = 0; jj < q; ++jj) acc += A[jj * q + i] * ph[jj];
      if (out)
        for (int jj = 0; jj < q; ++jj) acc += B[jj * q + i] * pv[jj];
      L->lam[c * q + i] = acc - L->gsrc[c * q + i];
    }
  }
#pragma omp parallel for schedule(static)
  for (long slot = 0; slot < L->n * q; ++slot) {
    L->phi[slot] = (L->dst[slot] >= 0) ? L->lam[L->dst[slot]] : 0.0;
    L->phiv[slot] = (L->vdst[slot] >= 0) ? L->lam[L->vdst[slot]] : 0.0;
  }
}

int orc_adjoint_iterate(orc_lattice* L, long iters) {
  if (!L->adj_ready) return -1;
  for (long k = 0; k < iters; ++k) adjoint_once(L);
  return 0;
}

long orc_adjoint_solve(orc_lattice* L, long max_iters, double tol, long check_every,
                       double* residual) {
  if (!L->adj_ready) return -1;
  long nq = L->n * L->q;
  double* snap = (double*)malloc(sizeof(double) * nq);
  memcpy(snap, L->phi, sizeof(double) * nq);
  if (check_every < 1) check_every = 1;
  long k = 0;
  double res = INFINITY;
  while (k < max_iters) {
    long m = check_every;
    if (k + m > max_iters) m = max_iters - k;
    orc_adjoint_iterate(L, m);
    k += m;
    double dmax = 0.0, pmax = 0.0;
    for (long s = 0; s < nq; ++s) {
      double dd = fabs(L->phi[s] - snap[s]);
      if (dd > dmax) dmax = dd;
      if (fabs(L->phi[s]) > pmax) pmax = fabs(L->phi[s]);
    }
    memcpy(snap, L->phi, sizeof(double) * nq);
    res = (pmax > 0.0) ? dmax / pmax : dmax;
    if (!isfinite(res)) break;
    if (res <= tol) break;
  }
  free(snap);
  if (residual) *residual = res;
  return k;
}

int orc_get_adjoint(const orc_lattice* L, double* phi) {
  if (!L->phi) return -1;
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < L->q; ++i) phi[(long)i * L->n + c] = L->phi[c * L->q + i];
  return 0;
}

int orc_get_adjoint_virtual(const orc_lattice* L, double* phiv) {
  if (!L->phiv) return -1;
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < L->q; ++i) phiv[(long)i * L->n + c] = L->phiv[c * L->q + i];
  return 0;
}

/* dJ/dd(x) = dJ/dd(x) - sum_i phi_i(x) dC_i/dd(x)  (the outlet values V do not
 * depend on d). */
int orc_gradient(const orc_lattice* L, double* g) {
  if (!L->adj_ready) return -1;
  int q = L->q;
  for (long c = 0; c < L->n; ++c) {
    double acc = 0.0;
    for (int i = 0; i < q; ++i) acc += L->phi[c * q + i] * L->dcdd[c * q + i];
    g[c] = L->dJdd[c] - acc;
  }
  return 0;
}

/* S: (post-collision values, outlet virtual values) -> state values; pinned
 * inlet slots get 0. */
int orc_apply_stream(const orc_lattice* L, const double* in, const double* vin, double* out) {
  int q = L->q;
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < q; ++i) {
      long sidx = L->src[c * q + i];
      double v = 0.0;
      if (sidx >= 0)
        v = in[(sidx % q) * L->n + sidx / q];
      else if (sidx <= -2)
        v = vin[((-2 - sidx) % q) * L->n + (-2 - sidx) / q];
      out[(long)i * L->n + c] = v;
    }
  return 0;
}

int orc_apply_stream_transpose(const orc_lattice* L, const double* in, double* out,
                               double* vout) {
  int q = L->q;
  for (long slot = 0; slot < L->n * q; ++slot) {
    long c = slot / q;
    int i = (int)(slot % q);
    long ds = L->dst[slot], vs = L->vdst[slot];
    out[(long)i * L->n + c] = (ds >= 0) ? in[(ds % q) * L->n + ds / q] : 0.0;
    vout[(long)i * L->n + c] = (vs >= 0) ? in[(vs % q) * L->n + vs / q] : 0.0;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Forward tangent (App. C): the directional derivative fdot = (df/dd) v of  */
/* the primal trajectory, carried along with it from fdot = 0 at the seeding */
/* moment.  Each step: fdot* = (dC/df) fdot + (dC/dd) v at every collided    */
/* cell, the outlet's virtual values get (dV/df) fdot, the pinned inlet 0,   */
/* then the same streaming map as f.  dJ(t)/dd . v = sum dJ/df . fdot +      */
/* dJ/dd v.  The closure enters through its exact Jacobian (tau_eff depends  */
/* on f, not on d).                                                          */
/* ------------------------------------------------------------------------ */

int orc_tangent_seed(orc_lattice* L) {
  long nq = L->n * L->q;
  if (!L->fdot) {
    L->fdot = (double*)calloc(nq, sizeof(double));
    L->tpost = (double*)calloc(nq, sizeof(double));
    L->tvpost = (double*)calloc(nq, sizeof(double));
  }
  memset(L->fdot, 0, sizeof(double) * nq);
  return 0;
}

int orc_tangent_step(orc_lattice* L, const double* v, long nsteps) {
  if (!L->fdot) return -1;
  stencil_t s = lat_stencil(L);
  int q = s.q;
  for (long t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static)
    for (long c = 0; c < L->n; ++c) {
      double A[QMAX * QMAX], B[QMAX * QMAX], dc[QMAX];
      const double* fc = L->f + c * q;
      const double* td = L->fdot + c * q;
      if (is_inlet(L, c)) {
        for (int i = 0; i < q; ++i) L->tpost[c * q + i] = 0.0;
        continue;
      }
      if (L->p.collision == ORC_COLL_HRR) {
        hrr_jacobian_s(&s, fc, L->d[c], L->p.tau, L->p.cs, ORC_TURB_DIFFERENTIATED, 0.0, A);
        hrr_dcdd_s(&s, fc, L->d[c], L->p.tau, L->p.cs, 0, 0.0, dc);
      } else {
        jacobian_s(&s, fc, L->d[c], L->p.tau, L->p.cs, ORC_TURB_DIFFERENTIATED, 0.0, A);
        dcdd_s(&s, fc, L->d[c], tau_eff_s(&s, fc, L->p.tau, L->p.cs), dc);
      }
      for (int jj = 0; jj < q; ++jj) {
        double acc = dc[jj] * v[c];
        for (int i = 0; i < q; ++i) acc += A[jj * q + i] * td[i];
        L->tpost[c * q + jj] = acc;
      }
      if (is_outlet(L, c)) {
        outlet_jacobian_s(&s, fc, B);
        for (int jj = 0; jj < q; ++jj) {
          double acc = 0.0;
          for (int i = 0; i < q; ++i) acc += B[jj * q + i] * td[i];
          L->tvpost[c * q + jj] = acc;
        }
      }
    }
    step_once(L);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < L->n; ++c) {
      for (int i = 0; i < q; ++i) {
        long sidx = L->src[c * q + i];
        double val;
        if (sidx >= 0)
          val = L->tpost[sidx];
        else if (sidx == -1)
          val = 0.0; /* pinned inlet */
        else
          val = L->tvpost[-2 - sidx];
        L->fdot[c * q + i] = val;
      }
    }
  }
  return 0;
}

double orc_tangent_objective(const orc_lattice* L, const double* v) {
  if (!L->fdot || !L->obj_set) return 0.0;
  stencil_t s = lat_stencil(L);
  int q = s.q;
  double acc = 0.0;
  if (L->obj_kind == ORC_OBJ_MEA) {
    double* g = (double*)malloc(sizeof(double) * L->n * q);
    mea_source_slots(L, g);
    for (long k = 0; k < L->n * q; ++k) acc += g[k] * L->fdot[k];
    free(g);
    return acc;
  }
  double g[QMAX];
  for (long c = 0; c < L->n; ++c) {
    if (!in_region(L, c)) continue;
    const double* fc = L->f + c * q;
    dJdf_s(&s, L->obj_kind, fc, L->d[c], L->p.tau, L->u0, L->p0, g);
    for (int i = 0; i < q; ++i) acc += g[i] * L->fdot[c * q + i];
    acc += dJdd_s(&s, L->obj_kind, fc, L->d[c], L->p.tau) * v[c];
  }
  return acc;
}

int orc_get_tangent(const orc_lattice* L, double* fdot) {
  if (!L->fdot) return -1;
  for (long c = 0; c < L->n; ++c)
    for (int i = 0; i < L->q; ++i) fdot[(long)i * L->n + c] = L->fdot[c * L->q + i];
  return 0;
}
