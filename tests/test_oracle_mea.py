"""Pins of the oracle's momentum-exchange drag J_MEA (Sec. 4, Eq. obj_mea).

- the surface node set of a cylinder lies on its rim (R - sqrt(2) < r < R)
  and inherits the geometry's mirror symmetry;
- a uniform equilibrium state gives the closed form J = 2 N_s rho u_x / A
  (each surface node exchanges sum_i xi_i,x (f_i - f_opp(i)) = 2 j_x);
- J is linear in f and dJ/df is its exact gradient: J(f + e) - J(f) = <g, e>;
- the steady adjoint gradient of J_MEA against central differences of the
  converged J on a tiny channel (relative error < 1e-6).
"""
import math

import numpy as np
import pytest

import oracle as O


def _lattice(nx=40, ny=24, xc=12.0, yc=11.5, D=8.0, box=((4, 2, 0), (20, 21, 0)), **kw):
    p = O.Params(nx=nx, ny=ny, **{**dict(tau=0.8, u_in=0.04), **kw})
    L = O.Lattice(p)
    L.build_cylinder(xc, yc, D)
    L.init_equilibrium()
    L.set_objective(O.OBJ_MEA, box[0], box[1], u0=math.pi * D)
    return L


def test_surface_set_on_the_rim_and_symmetric():
    L = _lattice()
    fl = L.mea_surface().reshape(24, 40)
    y, x = np.nonzero(fl)
    r = np.hypot(x - 12.0, y - 11.5)
    assert len(r) > 16
    assert np.all(r < 4.0) and np.all(r > 4.0 - math.sqrt(2.0))
    assert np.array_equal(fl, fl[::-1, :])  # mirror y -> 23 - y about y_c = 11.5


def test_uniform_equilibrium_closed_form():
    L = _lattice(bc_x=O.BC_PERIODIC, bc_y=O.BC_PERIODIC)
    ux, uy = 0.03, -0.01
    feq = O.equilibrium(O.D2Q9, 1.0, (ux, uy))
    L.set_populations(np.repeat(feq[:, None], L.n, axis=1))
    ns = int(L.mea_surface().sum())
    A = math.pi * 8.0
    assert abs(L.objective() - 2.0 * ns * ux / A) < 1e-15


def test_source_is_the_exact_gradient():
    rng = np.random.default_rng(5)
    L = _lattice()
    L.step(200)
    f = L.populations()
    J0 = L.objective()
    g = L.mea_source()
    e = 1e-6 * rng.standard_normal(f.shape)
    L.set_populations(f + e)
    assert abs(L.objective() - J0 - float((g * e).sum())) < 1e-15


def _solve(L, d, f_start=None):
    L.set_porosity(d)
    if f_start is None:
        L.init_equilibrium()
    else:
        L.set_populations(f_start)
    L.run_steady(200000, 1e-14, 100)
    return L.objective()


def test_steady_gradient_matches_finite_differences():
    L = _lattice(nx=24, ny=12, xc=7.0, yc=5.5, D=4.0, box=((2, 0, 0), (13, 11, 0)), tau=0.8, u_in=0.05)
    nx = L.p.nx
    d0 = L.porosity()
    J0 = _solve(L, d0)
    f0 = L.populations()
    L.adjoint_prepare(0, 0.0, O.TURB_DIFFERENTIATED)
    k, res = L.adjoint_solve(200000, 1e-14, 100)
    assert res < 1e-14
    g = L.gradient()
    h = 1e-4
    for (x, y) in [(5, 4), (8, 6), (6, 3), (12, 9)]:
        c = x + nx * y
        assert abs(d0[c] - 0.5) > 4 * h  # the surface set does not change
        if 2 * h < d0[c] < 1 - 2 * h:
            dp, dm = d0.copy(), d0.copy()
            dp[c] += h
            dm[c] -= h
            fd = (_solve(L, dp, f0) - _solve(L, dm, f0)) / (2 * h)
        else:
            s = -1.0 if d0[c] > 0.5 else 1.0
            d1, d2 = d0.copy(), d0.copy()
            d1[c] += s * h
            d2[c] += 2 * s * h
            fd = s * (-3 * J0 + 4 * _solve(L, d1, f0) - _solve(L, d2, f0)) / (2 * h)
        assert abs(g[c] - fd) < 1e-6 * abs(fd), ((x, y), g[c], fd)
