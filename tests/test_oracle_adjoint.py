"""Pins of the oracle's adjoint path.

- the per-cell Jacobians dC/df (BGK-HLBM, differentiated Smagorinsky, frozen
  turbulence), dC/dd, dV/df of the outlet and the objective partials dJ/df,
  dJ/dd (Sec. 3.2, Sec. 4, Sec. 5.4) against central finite differences of
  the per-cell maps;
- the streaming map and its transpose by the dot-product identity, and the
  stream table against the time step;
- the full steady adjoint gradient (Eqs. adjoint_steady, gradients_steady)
  against central finite differences of J(f*(d)) on a tiny channel,
  relative error < 1e-6, for J_FFA, J_DISS and the differentiated closure;
- the forced periodic Darcy box, where dJ/dd = G tau / (1 - d)^2 per cell
  for J = sum j_x (closed form);
- the mean-flow path on a steady flow reduces to the steady adjoint (Sec.
  3.3), a symmetric geometry gives a symmetric gradient (Sec. 5.3), and the
  frozen-turbulence and differentiated variants coincide when Cs = 0.
"""
import numpy as np
import pytest

import oracle as O


def _rand_f(kind, rng, amp=0.08):
    _, w, _ = O.stencil(kind)
    return w * (1.0 + amp * rng.uniform(-1, 1, len(w)))


def _fd_jac(fun, f, h=1e-6):
    q = len(f)
    cols = []
    for i in range(q):
        e = np.zeros(q)
        e[i] = h
        cols.append((fun(f + e) - fun(f - e)) / (2 * h))
    return np.array(cols).T  # [j, i] = d out_j / d f_i


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("cs", [0.0, 0.17])
def test_collision_jacobian_fd(kind, cs):
    rng = np.random.default_rng(11)
    for _ in range(4):
        f = _rand_f(kind, rng)
        d, tau = rng.uniform(0.05, 0.95), rng.uniform(0.51, 1.2)
        A = O.jacobian_cell(kind, f, d, tau, cs, O.TURB_DIFFERENTIATED)
        Afd = _fd_jac(lambda g: O.collide_cell(kind, g, d, tau, cs), f)
        assert np.abs(A - Afd).max() < 1e-8 * max(1.0, np.abs(A).max())


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_frozen_jacobian_is_constant_tau_bgk(kind):
    rng = np.random.default_rng(12)
    f = _rand_f(kind, rng)
    A = O.jacobian_cell(kind, f, 0.4, 0.6, 0.2, O.TURB_FROZEN, tau_frozen=0.73)
    Afd = _fd_jac(lambda g: O.collide_cell(kind, g, 0.4, 0.73, 0.0), f)
    assert np.abs(A - Afd).max() < 1e-8


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_frozen_equals_differentiated_without_closure(kind):
    rng = np.random.default_rng(13)
    f = _rand_f(kind, rng)
    a = O.jacobian_cell(kind, f, 0.4, 0.6, 0.0, O.TURB_FROZEN, tau_frozen=0.6)
    b = O.jacobian_cell(kind, f, 0.4, 0.6, 0.0, O.TURB_DIFFERENTIATED)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_dcdd_fd(kind):
    rng = np.random.default_rng(14)
    for cs in (0.0, 0.15):
        f = _rand_f(kind, rng)
        d, tau = 0.37, 0.66
        tau_used = O.tau_eff(kind, f, tau, cs)
        g = O.dcdd_cell(kind, f, d, tau_used)
        h = 1e-6
        fd = (O.collide_cell(kind, f, d + h, tau, cs) - O.collide_cell(kind, f, d - h, tau, cs)) / (2 * h)
        assert np.abs(g - fd).max() < 1e-9


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_outlet_jacobian_fd(kind):
    rng = np.random.default_rng(15)
    f = _rand_f(kind, rng)
    B = O.outlet_jacobian_cell(kind, f)
    Bfd = _fd_jac(lambda g: O.outlet_values_cell(kind, g), f)
    assert np.abs(B - Bfd).max() < 1e-8


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("obj", [O.OBJ_FFA, O.OBJ_DISS, O.OBJ_MOMENTUM])
def test_objective_partials_fd(kind, obj):
    rng = np.random.default_rng(16)
    for _ in range(3):
        f = _rand_f(kind, rng)
        d, tau, u0 = rng.uniform(0, 1), rng.uniform(0.51, 1.0), 0.04
        g = O.dJdf_cell(kind, obj, f, d, tau, u0)
        h = 1e-6
        fd = np.array([(O.objective_cell(kind, obj, f + h * e, d, tau, u0)
                        - O.objective_cell(kind, obj, f - h * e, d, tau, u0)) / (2 * h)
                       for e in np.eye(len(f))])
        assert np.abs(g - fd).max() < 1e-9 * max(1.0, np.abs(g).max())
        gd = O.dJdd_cell(kind, obj, f, d, tau)
        fdd = (O.objective_cell(kind, obj, f, d + h, tau, u0) - O.objective_cell(kind, obj, f, d - h, tau, u0)) / (2 * h)
        assert abs(gd - fdd) < 1e-9


def test_objective_values_closed_form():
    """J_FFA at equilibrium: rho (u0 ux - ux^2) + p0 - rho/3; J_DISS at
    equilibrium: only the porous part (1-d)/tau0 |u|^2 (no strain)."""
    u = np.array([0.03, 0.01, 0.0])
    f = O.equilibrium(O.D2Q9, 1.02, u)
    J = O.objective_cell(O.D2Q9, O.OBJ_FFA, f, 1.0, 0.8, u0=0.05, p0=1 / 3)
    assert abs(J - (1.02 * (0.05 * 0.03 - 0.03 ** 2) + 1 / 3 - 1.02 / 3)) < 1e-16
    Jd = O.objective_cell(O.D2Q9, O.OBJ_DISS, f, 0.3, 0.8)
    assert abs(Jd - 0.7 / 0.8 * (u @ u)) < 1e-16


CHANNEL = dict(nx=24, ny=12, tau=0.8, u_in=0.05)


def _channel(stencil=O.D2Q9, nz=1, **kw):
    p = O.Params(stencil=stencil, nz=nz, **{**CHANNEL, **kw})
    L = O.Lattice(p)
    L.build_cylinder(7.0, 5.5, 4.0)
    return L


@pytest.mark.parametrize("stencil,nz,bcy", [(O.D2Q9, 1, O.BC_WALLS), (O.D2Q9, 1, O.BC_PERIODIC),
                                            (O.D3Q19, 4, O.BC_WALLS)])
def test_stream_transpose_dot_product(stencil, nz, bcy):
    rng = np.random.default_rng(17)
    L = _channel(stencil, nz, bc_y=bcy, bc_z=O.BC_WALLS if stencil == O.D3Q19 else O.BC_PERIODIC)
    x = rng.standard_normal((L.q, L.n))
    xv = rng.standard_normal((L.q, L.n))
    y = rng.standard_normal((L.q, L.n))
    Sx = L.apply_stream(x, xv)
    ty, tvy = L.apply_stream_transpose(y)
    lhs = (y * Sx).sum()
    rhs = (ty * x).sum() + (tvy * xv).sum()
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)
    # every state slot outside the pinned inlet column has exactly one source
    ones = L.apply_stream(np.ones((L.q, L.n)), np.ones((L.q, L.n)))
    col = np.arange(L.n) % L.p.nx
    assert np.all(ones[:, col > 0] == 1.0) and np.all(ones[:, col == 0] == 0.0)


def test_stream_table_matches_step():
    """One oracle step equals S applied to the per-cell collisions and the
    outlet virtual values (pinned inlet column excluded)."""
    rng = np.random.default_rng(18)
    L = _channel(tau=0.7)
    L.init_equilibrium()
    L.step(50)
    f = L.populations()
    d = L.porosity()
    post = np.array([O.collide_cell(O.D2Q9, f[:, c], d[c], 0.7) for c in range(L.n)]).T
    virt = np.array([O.outlet_values_cell(O.D2Q9, f[:, c]) for c in range(L.n)]).T
    ref = L.apply_stream(post, virt)
    L.step(1)
    col = np.arange(L.n) % L.p.nx
    assert np.abs(L.populations()[:, col > 0] - ref[:, col > 0]).max() < 1e-16


def _solve(L, d, f_start=None):
    L.set_porosity(d)
    if f_start is None:
        L.init_equilibrium()
    else:  # warm start from the unperturbed steady state
        L.set_populations(f_start)
    L.run_steady(200000, 1e-14, 100)  # 1e-15 sits below the round-off floor
    return L.objective()


FD_CELLS = [(5, 4), (8, 6), (6, 3), (12, 9)]


@pytest.mark.parametrize("obj,cs", [(O.OBJ_FFA, 0.0), (O.OBJ_DISS, 0.0), (O.OBJ_FFA, 0.1),
                                    (O.OBJ_DISS, 0.12)])
def test_steady_gradient_matches_finite_differences(obj, cs):
    L = _channel(cs=cs)
    nx, ny = L.p.nx, L.p.ny
    if obj == O.OBJ_FFA:
        L.set_objective(obj, (16, 0, 0), (16, ny - 1, 0), u0=0.05)
    else:
        L.set_objective(obj, (2, 0, 0), (20, ny - 1, 0))
    d0 = L.porosity()
    J0 = _solve(L, d0)
    f0 = L.populations()
    L.adjoint_prepare(0, 0.0, O.TURB_DIFFERENTIATED)
    k, res = L.adjoint_solve(200000, 1e-14, 100)
    assert res < 1e-14
    g = L.gradient()
    for (x, y) in FD_CELLS:
        c = x + nx * y
        h = 1e-4
        if 2 * h < d0[c] < 1 - 2 * h:
            dp, dm = d0.copy(), d0.copy()
            dp[c] += h
            dm[c] -= h
            fd = (_solve(L, dp, f0) - _solve(L, dm, f0)) / (2 * h)
        else:  # d = 1 or 0: one-sided second-order difference inside [0, 1]
            s = -1.0 if d0[c] > 0.5 else 1.0
            d1, d2 = d0.copy(), d0.copy()
            d1[c] += s * h
            d2[c] += 2 * s * h
            fd = s * (-3 * J0 + 4 * _solve(L, d1, f0) - _solve(L, d2, f0)) / (2 * h)
        assert abs(g[c] - fd) < 1e-6 * abs(fd), ((x, y), g[c], fd)


@pytest.mark.parametrize("d,tau", [(0.6, 0.8), (0.3, 0.55)])
def test_darcy_gradient_closed_form(d, tau):
    G = 2e-5
    p = O.Params(nx=6, ny=5, tau=tau, bc_x=O.BC_PERIODIC, bc_y=O.BC_PERIODIC, force=(G, 0, 0))
    L = O.Lattice(p)
    L.set_porosity(np.full(L.n, d))
    L.init_equilibrium()
    L.step(4000)
    L.set_objective(O.OBJ_MOMENTUM, (0, 0, 0), (5, 4, 0))
    L.adjoint_prepare(0)
    L.adjoint_solve(100000, 1e-15, 100)
    g = L.gradient()
    assert np.abs(g / (G * tau / (1 - d) ** 2) - 1).max() < 1e-10


def test_meanflow_on_steady_flow_equals_steady_adjoint():
    L = _channel()
    ny = L.p.ny
    L.set_objective(O.OBJ_DISS, (2, 0, 0), (20, ny - 1, 0))
    L.init_equilibrium()
    L.run_steady(200000, 1e-14, 100)
    L.adjoint_prepare(0)
    L.adjoint_iterate(3000)
    g_steady = L.gradient()
    L.window_reset()
    for _ in range(16):
        L.step(1)
        L.window_sample()
    J = L.objective()
    assert abs(L.window_objective() - J) < 1e-13 * abs(J)
    L.adjoint_prepare(1)
    L.adjoint_iterate(3000)
    g_mean = L.gradient()
    assert np.abs(g_mean - g_steady).max() < 1e-11 * np.abs(g_steady).max()


@pytest.mark.parametrize("obj", [O.OBJ_FFA, O.OBJ_DISS])
def test_symmetric_geometry_gives_symmetric_gradient(obj):
    p = O.Params(nx=30, ny=13, tau=0.7, u_in=0.04)
    L = O.Lattice(p)
    L.build_cylinder(8.0, 6.0, 5.0)
    if obj == O.OBJ_FFA:
        L.set_objective(obj, (20, 0, 0), (20, 12, 0), u0=0.04)
    else:
        L.set_objective(obj, (1, 0, 0), (25, 12, 0))
    L.init_equilibrium()
    L.run_steady(100000, 1e-14, 200)
    L.adjoint_prepare(0)
    L.adjoint_solve(100000, 1e-14, 200)
    g = L.gradient().reshape(13, 30)
    assert np.abs(g - g[::-1]).max() < 1e-10 * np.abs(g).max()
    assert np.abs(g).max() > 0


def test_adjoint_tau_default_is_tau0():
    L = _channel()
    L.set_objective(O.OBJ_FFA, (16, 0, 0), (16, 11, 0), u0=0.05)
    L.init_equilibrium()
    L.step(500)
    L.adjoint_prepare(0, 0.0)
    L.adjoint_iterate(100)
    a = L.gradient()
    L.adjoint_prepare(0, 0.8)
    L.adjoint_iterate(100)
    assert np.array_equal(a, L.gradient())


def test_gradient_zero_on_inlet_column():
    L = _channel()
    L.set_objective(O.OBJ_FFA, (16, 0, 0), (16, 11, 0), u0=0.05)
    L.init_equilibrium()
    L.step(300)
    L.adjoint_prepare(0)
    L.adjoint_iterate(200)
    g = L.gradient().reshape(12, 24)
    assert np.all(g[:, 0] == 0.0)
    assert np.abs(g[:, 1:]).max() > 0


def test_objective_region_rejects_inlet_column():
    L = _channel()
    with pytest.raises(ValueError):
        L.set_objective(O.OBJ_FFA, (0, 0, 0), (0, 11, 0))


@pytest.mark.parametrize("obj,bcz", [(O.OBJ_FFA, O.BC_PERIODIC), (O.OBJ_DISS, O.BC_WALLS)])
def test_steady_gradient_d3q19_matches_finite_differences(obj, bcz):
    """The laminar 3D case (D3Q19; periodic or bounce-back z walls): the steady
    adjoint gradient against central finite differences of the converged J."""
    L = _channel(O.D3Q19, 5, bc_z=bcz, u_in=0.04, tau=0.7)
    nx, ny, nz = L.p.nx, L.p.ny, L.p.nz
    if obj == O.OBJ_FFA:
        L.set_objective(obj, (16, 0, 0), (16, ny - 1, nz - 1), u0=0.04)
    else:
        L.set_objective(obj, (2, 0, 0), (20, ny - 1, nz - 1))
    d0 = L.porosity()
    J0 = _solve(L, d0)
    f0 = L.populations()
    L.adjoint_prepare(0, 0.0, O.TURB_DIFFERENTIATED)
    k, res = L.adjoint_solve(200000, 1e-14, 100)
    assert res < 1e-14
    g = L.gradient()
    for (x, y, z) in [(5, 4, 2), (8, 6, 0), (9, 5, 4)]:
        c = x + nx * (y + ny * z)
        h = 1e-4
        assert 2 * h < d0[c] < 1 - 2 * h or d0[c] in (0.0, 1.0)
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
