"""Pins of the oracle's HRRLBM collision (Sec. 2.2, Eq. HRRLBM) and its
complex-step Jacobians.

- mass is conserved; momentum is conserved for d = 1 and decays by
  (1 - (1 - d)/tau) per step otherwise (the HLBM porous term, as for BGK);
- the collision depends on f only through rho, j and sum xi xi f (the
  regularization discards the rest);
- a third-order Hermite equilibrium at d = 1 is a fixed point;
- the post-collision second moment is exactly
  rho/3 I + rho u~u~ + (1 - 1/tau_eff) a2, a2 = sum xi xi f - rho/3 I - rho u~u~
  (the regularized non-equilibrium part relaxes by 1 - 1/tau_eff);
- the collision output is a Hermite series with the coefficients Eq. HRRLBM
  names: rho, rho u~ + (1 - 1/tau)(1 - d) j, rho u~u~ + (1 - 1/tau) a2, and on
  the supported third-order components rho u~_a^2 u~_b + (1 - 1/tau)
  (2 u~_a a2_ab + u~_b a2_aa) (the recursive a3);
- plane Poiseuille flow with the HRR collision: second differences of u_x
  equal -G/nu exactly (the viscosity nu = (tau - 1/2)/3 of the relaxed
  second moment);
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


def _state(kind, f, d):
    c, w, _ = O.stencil(kind)
    rho = f.sum()
    ut = d * (c.T @ f) / rho
    a2 = np.einsum("i,ia,ib->ab", f, c, c) - rho / 3.0 * np.eye(3) - rho * np.outer(ut, ut)
    return c, w, rho, ut, a2


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("cs", [0.0, 0.15])
def test_second_moment_relaxes_exactly(kind, cs):
    rng = np.random.default_rng(11)
    D = 2 if kind == O.D2Q9 else 3
    for d in (1.0, 0.65, 0.0):
        f = _rand_f(kind, rng)
        c, w, rho, ut, a2 = _state(kind, f, d)
        tau = O.tau_eff(kind, f, 0.62, cs)
        out = O.hrr_collide_cell(kind, f, d, 0.62, cs)
        M2 = np.einsum("i,ia,ib->ab", out, c, c)
        want = rho / 3.0 * np.eye(3) + rho * np.outer(ut, ut) + (1.0 - 1.0 / tau) * a2
        assert np.abs(M2 - want)[:D, :D].max() < 1e-15
        assert abs(a2[:D, :D]).max() > 1e-3  # a genuine non-equilibrium part


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_output_is_the_regularized_hermite_series(kind):
    """Fits the post-collision populations with the Hermite basis
    {1, xi, H2, supported H_aab} (weighted by w_i, cs^2 = 1/3) and checks the
    fitted coefficients against the HRRLBM relations."""
    rng = np.random.default_rng(12)
    D = 2 if kind == O.D2Q9 else 3
    pairs = [(0, 1), (1, 0)] if D == 2 else [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)]
    sym = [(a, b) for a in range(D) for b in range(a, D)]
    for d in (1.0, 0.7):
        f = _rand_f(kind, rng)
        c, w, rho, ut, a2 = _state(kind, f, d)
        tau = 0.58
        out = O.hrr_collide_cell(kind, f, d, tau, 0.0)
        cols = [w]
        cols += [w * 3.0 * c[:, a] for a in range(D)]
        cols += [w * 4.5 * (2.0 - (a == b)) * (c[:, a] * c[:, b] - (a == b) / 3.0) for a, b in sym]
        cols += [w * 13.5 * c[:, b] * (c[:, a] ** 2 - 1.0 / 3.0) for a, b in pairs]
        B = np.array(cols).T
        coef, *_ = np.linalg.lstsq(B, out, rcond=None)
        assert np.abs(B @ coef - out).max() < 1e-15  # the output lies in the span
        om = 1.0 - 1.0 / tau
        j = c.T @ f
        want = [rho] + [rho * ut[a] + om * (1.0 - d) * j[a] for a in range(D)]
        want += [rho * ut[a] * ut[b] + om * a2[a, b] for a, b in sym]
        want += [rho * ut[a] ** 2 * ut[b] + om * (2.0 * ut[a] * a2[a, b] + ut[b] * a2[a, a]) for a, b in pairs]
        assert np.abs(coef - np.array(want)).max() < 1e-14


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.3])
def test_hrr_poiseuille_curvature_exact(tau):
    H, G = 16, 1e-6
    p = O.Params(nx=3, ny=H, tau=tau, bc_x=O.BC_PERIODIC, bc_y=O.BC_WALLS, force=(G, 0.0, 0.0),
                 collision=O.COLL_HRR)
    L = O.Lattice(p)
    nu = (tau - 0.5) / 3.0
    y = np.repeat(np.arange(H), 3)
    u0 = np.zeros((3, L.n))
    u0[0] = G / (2 * nu) * (y + 0.5) * (H - 0.5 - y)  # start near the solution (only shortens the run)
    L.init_equilibrium(u=u0)
    L.run_steady(400000, 1e-15, 500)
    ux = L.moments()[1][0].reshape(H, 3)[:, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    assert np.abs(d2 * nu / G + 1.0).max() < 1e-9


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
