"""Pins of the oracle's HRRLBM collision (Sec. 2.2, Eq. HRRLBM) and its
complex-step Jacobians.

- mass is conserved; momentum is conserved for d = 1 and decays by
  (1 - (1 - d)/tau) per step otherwise (the HLBM porous term, as for BGK);
- the collision depends on f only through rho, j and sum xi xi f (the
  regularization discards the rest);
- a third-order Hermite equilibrium at d = 1 is a fixed point;
- the complex-step dC/df and dC/dd equal central finite differences, with and
  without the closure, frozen or differentiated;
- a steady 3D channel flow with the HRR collision and the closure: the steady
  adjoint gradient against central differences of the converged J.
"""
import numpy as np
import pytest

import oracle as O


def _rand_f(kind, rng, amp=0.08):
    _, w, _ = O.stencil(kind)
    return w * (1.0 + amp * rng.uniform(-1, 1, len(w)))


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("cs", [0.0, 0.15])
def test_conservation_and_porous_decay(kind, cs):
    rng = np.random.default_rng(2)
    c, _, _ = O.stencil(kind)
    for d in (1.0, 0.6):
        f = _rand_f(kind, rng)
        out = O.hrr_collide_cell(kind, f, d, 0.7, cs)
        assert abs(out.sum() - f.sum()) < 1e-15
        tau = O.tau_eff(kind, f, 0.7, cs)
        j0, j1 = c.T @ f, c.T @ out
        assert np.abs(j1 - (1.0 - (1.0 - d) / tau) * j0).max() < 1e-15


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_depends_only_on_rho_j_and_second_moments(kind):
    rng = np.random.default_rng(3)
    c, w, _ = O.stencil(kind)
    f = _rand_f(kind, rng)
    # a perturbation with zero mass, momentum and second moments
    M = np.vstack([np.ones(len(w)), c.T] + [c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)])
    _, _, vt = np.linalg.svd(M)
    g = vt[-1] * 1e-3
    assert np.abs(M @ g).max() < 1e-15
    a = O.hrr_collide_cell(kind, f, 0.8, 0.6, 0.1)
    b = O.hrr_collide_cell(kind, f + g, 0.8, 0.6, 0.1)
    assert np.abs(a - b).max() < 1e-15


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_third_order_equilibrium_is_a_fixed_point(kind):
    u = np.array([0.04, -0.03, 0.02 if kind == O.D3Q19 else 0.0])
    f0 = O.hrr_collide_cell(kind, O.equilibrium(kind, 1.02, u), 1.0, 0.6)  # f^eq(rho, u) of the scheme
    f1 = O.hrr_collide_cell(kind, f0, 1.0, 0.6)
    assert np.abs(f1 - f0).max() < 1e-15


def _fd_jac(fun, f, h=1e-6):
    cols = []
    for i in range(len(f)):
        e = np.zeros(len(f))
        e[i] = h
        cols.append((fun(f + e) - fun(f - e)) / (2 * h))
    return np.array(cols).T


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("cs,turb", [(0.0, O.TURB_DIFFERENTIATED), (0.15, O.TURB_DIFFERENTIATED),
                                     (0.15, O.TURB_FROZEN)])
def test_complex_step_jacobians_match_finite_differences(kind, cs, turb):
    rng = np.random.default_rng(4)
    f = _rand_f(kind, rng)
    d, ta, tf = 0.7, 0.62, 0.66
    A = O.hrr_jacobian_cell(kind, f, d, ta, cs, turb, tf)
    if turb == O.TURB_FROZEN and cs > 0:
        # frozen: the collision with tau held at tf, i.e. BGK-free HRR at tau0 = tf without closure
        fun = lambda x: O.hrr_collide_cell(kind, x, d, tf, 0.0)  # noqa: E731
    else:
        fun = lambda x: O.hrr_collide_cell(kind, x, d, ta, cs)  # noqa: E731
    assert np.abs(A - _fd_jac(fun, f)).max() < 1e-8
    g = O.hrr_dcdd_cell(kind, f, d, ta, cs, turb, tf)
    h = 1e-6
    if turb == O.TURB_FROZEN and cs > 0:
        fd = (O.hrr_collide_cell(kind, f, d + h, tf) - O.hrr_collide_cell(kind, f, d - h, tf)) / (2 * h)
    else:
        fd = (O.hrr_collide_cell(kind, f, d + h, ta, cs) - O.hrr_collide_cell(kind, f, d - h, ta, cs)) / (2 * h)
    assert np.abs(g - fd).max() < 1e-8


def _solve(L, d, f_start=None):
    L.set_porosity(d)
    if f_start is None:
        L.init_equilibrium()
    else:
        L.set_populations(f_start)
    L.run_steady(200000, 1e-14, 100)
    return L.objective()


@pytest.mark.parametrize("cs", [0.0, 0.1])
def test_hrr_steady_gradient_matches_finite_differences(cs):
    p = O.Params(stencil=O.D3Q19, nx=24, ny=12, nz=5, tau=0.7, cs=cs, u_in=0.04, bc_z=O.BC_PERIODIC,
                 collision=O.COLL_HRR)
    L = O.Lattice(p)
    L.build_cylinder(7.0, 5.5, 4.0)
    L.set_objective(O.OBJ_DISS, (2, 0, 0), (20, 11, 4))
    d0 = L.porosity()
    J0 = _solve(L, d0)
    f0 = L.populations()
    L.adjoint_prepare(0, 0.0, O.TURB_DIFFERENTIATED)
    k, res = L.adjoint_solve(200000, 1e-14, 100)
    assert res < 1e-14
    g = L.gradient()
    nx, ny = 24, 12
    for (x, y, z) in [(5, 4, 2), (8, 6, 0), (12, 9, 3)]:
        c = x + nx * (y + ny * z)
        h = 1e-4
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
        assert abs(g[c] - fd) < 1e-6 * abs(fd), ((x, y, z), g[c], fd)
