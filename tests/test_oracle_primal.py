"""Pins of the oracle's primal HLBM step against closed forms and invariants.

- mass conservation of BGK/HLBM collision + bounce-back/periodic streaming
  (Sec. 2.1, Eq. hlbm: the equilibrium carries the cell's own density);
- Darcy decay of a uniform periodic state, u_{n+1} = (1 - (1-d)/tau) u_n,
  and the forced Darcy balance j* = G tau / (1 - d): the per-step momentum
  loss of the porosity term is (1 - d)/tau = nu/K (Sec. 2.1, d = 1 - tau nu/K);
- plane Poiseuille flow with halfway bounce-back: second differences equal
  -G/nu exactly, nu = (tau - 1/2)/3 (Sec. 2.1, viscosity relation), and the
  error to the continuum parabola is a uniform slip (second-order in H);
- a forced channel filled with a uniform porous medium (Sec. 2.1, the
  Brinkman-type equation the HLBM recovers, Eq. btnse): the steady profile
  converges at second order to the continuum Brinkman solution
  u = (G K / nu) [1 - cosh(y / sqrt K) / cosh(H / (2 sqrt K))] with
  K = tau nu / (1 - d), the grid refined at a fixed Darcy number K / H^2;
- the Smagorinsky closure: tau_eff solves tau = tau0 + 3 Cs^2 |S(tau)|
  (Sec. 2.2, Eqs. turbVisc, tauEff) and Cs = 0 gives plain BGK.
"""
import numpy as np
import pytest

import oracle as O


def _random_state(L, rng, amp=0.02):
    c, w, _ = O.stencil(L.p.stencil)
    f = np.outer(w, np.ones(L.n)) * (1.0 + amp * rng.uniform(-1, 1, (L.q, L.n)))
    L.set_populations(f)


@pytest.mark.parametrize("kind,cs", [(O.D2Q9, 0.0), (O.D2Q9, 0.15), (O.D3Q19, 0.0), (O.D3Q19, 0.15)])
def test_mass_conservation_closed_box(kind, cs):
    rng = np.random.default_rng(7)
    nz = 1 if kind == O.D2Q9 else 6
    p = O.Params(stencil=kind, nx=12, ny=9, nz=nz, tau=0.62, cs=cs, bc_x=O.BC_WALLS,
                 bc_y=O.BC_WALLS, bc_z=O.BC_WALLS if kind == O.D3Q19 else O.BC_PERIODIC)
    L = O.Lattice(p)
    L.set_porosity(rng.uniform(0.0, 1.0, L.n))
    _random_state(L, rng)
    m0 = L.populations().sum()
    L.step(1000 if kind == O.D2Q9 else 300)
    m1 = L.populations().sum()
    assert abs(m1 - m0) / m0 < 1e-13


def test_mass_conservation_periodic():
    rng = np.random.default_rng(8)
    p = O.Params(nx=10, ny=7, tau=0.9, bc_x=O.BC_PERIODIC, bc_y=O.BC_PERIODIC)
    L = O.Lattice(p)
    L.set_porosity(rng.uniform(0.3, 1.0, L.n))
    _random_state(L, rng, 0.05)
    m0 = L.populations().sum()
    L.step(1000)
    assert abs(L.populations().sum() - m0) / m0 < 1e-13


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("d,tau", [(0.7, 0.8), (0.2, 0.53), (0.0, 1.4)])
def test_darcy_decay_uniform(kind, d, tau):
    nz = 1 if kind == O.D2Q9 else 3
    p = O.Params(stencil=kind, nx=5, ny=4, nz=nz, tau=tau, bc_x=O.BC_PERIODIC, bc_y=O.BC_PERIODIC)
    L = O.Lattice(p)
    L.set_porosity(np.full(L.n, d))
    u0 = np.array([0.03, -0.02, 0.01 if kind == O.D3Q19 else 0.0])
    # plain equilibrium at velocity u0 (not scaled by d)
    L.set_populations(np.outer(O.equilibrium(kind, 1.0, u0), np.ones(L.n)))
    g = 1.0 - (1.0 - d) / tau
    for n in range(1, 31):
        L.step(1)
        rho, u = L.moments()
        assert np.abs(rho - 1.0).max() < 1e-14
        assert np.abs(u - (g ** n) * u0[:, None]).max() < 1e-15 + 1e-13 * abs(g) ** n


@pytest.mark.parametrize("d,tau", [(0.6, 0.8), (0.9, 0.55)])
def test_forced_darcy_steady(d, tau):
    G = np.array([2e-5, -1e-5, 0.0])
    p = O.Params(nx=4, ny=3, tau=tau, bc_x=O.BC_PERIODIC, bc_y=O.BC_PERIODIC, force=tuple(G))
    L = O.Lattice(p)
    L.set_porosity(np.full(L.n, d))
    L.init_equilibrium()
    L.step(3000)
    rho, u = L.moments()
    jstar = G * tau / (1.0 - d)
    assert np.abs(rho * u - jstar[:, None]).max() < 1e-16


def _parabola(L, H, nx, G, nu):
    """Initial velocity field: the continuum parabola (only speeds up the run)."""
    y = np.repeat(np.arange(H), nx)
    u = np.zeros((3, L.n))
    u[0] = G / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    return u


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 1.3])
def test_poiseuille_curvature_exact(tau):
    H, G = 16, 1e-6
    p = O.Params(nx=3, ny=H, tau=tau, bc_x=O.BC_PERIODIC, bc_y=O.BC_WALLS, force=(G, 0.0, 0.0))
    L = O.Lattice(p)
    nu = (tau - 0.5) / 3.0
    L.init_equilibrium(u=_parabola(L, H, 3, G, nu))
    L.run_steady(400000, 1e-15, 500)
    _, u = L.moments()
    ux = u[0].reshape(H, 3)[:, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    assert np.abs(d2 * nu / G + 1.0).max() < 1e-9
    # the profile differs from the continuum parabola by a uniform slip only
    y = np.arange(H)
    ua = G / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    diff = ux - ua
    assert np.ptp(diff) < 1e-9 * ua.max()
    assert np.abs(ux[: H // 2] - ux[::-1][: H // 2]).max() < 1e-15


def test_poiseuille_second_order():
    """Relative error to the continuum profile falls as H^-2."""
    tau, G = 0.8, 1e-7
    errs = []
    for H in (8, 16, 32):
        p = O.Params(nx=3, ny=H, tau=tau, bc_x=O.BC_PERIODIC, force=(G, 0.0, 0.0))
        L = O.Lattice(p)
        nu = (tau - 0.5) / 3.0
        L.init_equilibrium(u=_parabola(L, H, 3, G, nu))
        L.run_steady(2000000, 1e-14, 1000)
        ux = L.moments()[1][0].reshape(H, 3)[:, 0]
        y = np.arange(H)
        ua = G / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
        errs.append(np.abs(ux - ua).max() / ua.max())
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(eoc - 2.0) < 0.05), eoc


def _brinkman_error(H, Da, tau, G):
    """Relative max error of the converged porous channel (walls at y = -1/2
    and H - 1/2, x periodic, uniform d) to the continuum Brinkman profile."""
    nu = (tau - 0.5) / 3.0
    K = Da * H * H
    d = 1.0 - tau * nu / K  # Sec. 2.1: d = 1 - dx^2 tau nu / K
    p = O.Params(nx=2, ny=H, tau=tau, bc_x=O.BC_PERIODIC, bc_y=O.BC_WALLS, force=(G, 0.0, 0.0))
    L = O.Lattice(p)
    L.set_porosity(np.full(L.n, d))
    y = np.arange(H) - (H - 1) / 2.0
    sk = np.sqrt(K)
    ua = G * K / nu * (1.0 - np.cosh(y / sk) / np.cosh(H / (2.0 * sk)))
    u0 = np.zeros((3, L.n))
    u0[0] = np.repeat(ua, 2)  # start from the continuum profile (only shortens the run)
    L.init_equilibrium(u=u0)
    L.run_steady(400000, 1e-12, 500)
    ux = L.moments()[1][0].reshape(H, 2)[:, 0]
    assert np.abs(ux - ux[::-1]).max() < 1e-12 * ua.max()
    return np.abs(ux - ua).max() / ua.max()


def test_brinkman_channel_second_order():
    """Darcy number 0.05 (H / sqrt K = 4.5: a flattened profile, far from the
    parabola), tau = 0.8, H = 16, 32, 64."""
    e = np.array([_brinkman_error(H, 0.05, 0.8, 1e-6) for H in (16, 32, 64)])
    eoc = np.log2(e[:-1] / e[1:])
    assert e[-1] < 1e-3, e
    assert eoc[0] > 1.75 and 1.85 < eoc[1] < 2.1, eoc


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_smagorinsky_tau_implicit(kind):
    rng = np.random.default_rng(3)
    c, w, _ = O.stencil(kind)
    dim = 2 if kind == O.D2Q9 else 3
    cc = c[:, :dim].astype(float)
    for _ in range(20):
        f = w * (1.0 + 0.1 * rng.uniform(-1, 1, len(w)))
        tau0, cs = rng.uniform(0.501, 0.9), rng.uniform(0.05, 0.3)
        t = O.tau_eff(kind, f, tau0, cs)
        rho = f.sum()
        j = f @ cc
        Pi = np.einsum("i,ia,ib->ab", f, cc, cc) - rho / 3 * np.eye(dim) - np.outer(j, j) / rho
        S = -Pi / (2 * t / 3.0)
        Smag = np.sqrt(2 * (S * S).sum())
        assert abs(t - (tau0 + 3 * cs * cs * Smag)) < 1e-14
        assert t > tau0
        assert O.tau_eff(kind, f, tau0, 0.0) == tau0


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_smagorinsky_zero_is_bgk(kind):
    rng = np.random.default_rng(4)
    _, w, _ = O.stencil(kind)
    f = w * (1 + 0.05 * rng.uniform(-1, 1, len(w)))
    a = O.collide_cell(kind, f, 0.7, 0.8, 0.0)
    b = O.collide_cell(kind, f, 0.7, 0.8, 1e-300)  # tiny constant takes the closure branch
    assert np.abs(a - b).max() < 1e-16


@pytest.mark.parametrize("kind", [O.D2Q9, O.D3Q19])
def test_collision_conserves_mass_and_relaxes_momentum(kind):
    """Sum of f* equals rho; momentum of f* is j - (1/tau)(j - rho d u) (BGK
    toward f^eq(rho, d u))."""
    rng = np.random.default_rng(5)
    c, w, _ = O.stencil(kind)
    for _ in range(10):
        f = w * (1 + 0.05 * rng.uniform(-1, 1, len(w)))
        d, tau = rng.uniform(0, 1), rng.uniform(0.52, 1.5)
        out = O.collide_cell(kind, f, d, tau)
        rho, j = f.sum(), f @ c
        assert abs(out.sum() - rho) < 1e-15
        assert np.abs(out @ c - (j - (j - d * j) / tau)).max() < 1e-16


def test_outlet_values():
    """Virtual outlet column: f^eq at density 1 and the cell's velocity."""
    rng = np.random.default_rng(6)
    for kind in (O.D2Q9, O.D3Q19):
        c, w, _ = O.stencil(kind)
        f = w * (1 + 0.05 * rng.uniform(-1, 1, len(w)))
        u = (f @ c) / f.sum()
        assert np.abs(O.outlet_values_cell(kind, f) - O.equilibrium(kind, 1.0, u)).max() < 1e-16


def test_cylinder_geometry():
    p = O.Params(nx=40, ny=21)
    L = O.Lattice(p)
    L.build_cylinder(12.0, 10.0, 10.0)
    d = L.porosity().reshape(21, 40)
    assert d[10, 12] == 0.0                       # centre is solid
    assert d[10, 12 + 4] == 0.0                   # r = R - 1
    assert abs(d[10, 12 + 5] - 0.5) < 1e-15       # r = R: half solid
    assert d[10, 12 + 6] == 1.0                   # r = R + 1
    assert np.array_equal(d, d[::-1, :])          # symmetric about y = 10
    assert d.min() == 0.0 and d.max() == 1.0


def test_cylinder_noise_modes():
    rng = np.random.default_rng(9)
    p = O.Params(nx=40, ny=21)
    L = O.Lattice(p)
    L.build_cylinder(12.0, 10.0, 10.0)
    d0 = L.porosity()
    noise = rng.uniform(-0.3, 0.3, L.n)
    L.build_cylinder(12.0, 10.0, 10.0, noise, O.NOISE_RIM)
    d1 = L.porosity()
    rim = (d0 > 0) & (d0 < 1)
    assert np.array_equal(d1[~rim], d0[~rim])
    assert np.allclose(d1[rim], np.clip(d0[rim] + noise[rim], 0, 1), atol=0, rtol=0)
    L.build_cylinder(12.0, 10.0, 10.0, np.abs(noise), O.NOISE_BOX, 3.0)
    d2 = L.porosity().reshape(21, 40)
    x, y = np.meshgrid(np.arange(40), np.arange(21))
    box = (np.abs(x - 12) <= 3) & (np.abs(y - 10) <= 3)
    chi = np.clip(1 - d0.reshape(21, 40) + np.abs(noise).reshape(21, 40), 0, 1)
    assert np.array_equal(d2[box], 1 - chi[box])
    assert np.array_equal(d2[~box], d0.reshape(21, 40)[~box])


def test_channel_pressure_outlet_keeps_flow():
    """With the equilibrium inlet and the density-1 outlet, a channel carries a
    steady flow with a linear pressure drop (no drift of the flow rate)."""
    p = O.Params(nx=64, ny=16, tau=0.8, u_in=0.05)
    L = O.Lattice(p)
    L.init_equilibrium()
    L.step(6000)
    r1, u1 = L.moments()
    L.step(2000)
    r2, u2 = L.moments()
    assert np.abs(u2 - u1).max() < 1e-6
    flux = (r2 * u2[0]).reshape(16, 64)[:, 1:].sum(axis=0)
    assert np.ptp(flux) < 1e-6 * flux.mean()
    rc = r2.reshape(16, 64)[8, 4:60]
    assert np.all(np.diff(rc) < 0)  # pressure falls along the channel
    assert np.ptp(np.diff(rc)) < 0.1 * abs(np.diff(rc).mean())  # entrance/exit effects only


def test_permeable_cylinder_porosity():
    """d_solid sets the porosity of the cylinder core (Sec. 2.1: d = 1 - dx^2
    tau nu / K), the ramp scales with 1 - d_solid, d_solid = 0 is the solid
    cylinder."""
    p = O.Params(nx=40, ny=30, tau=0.55)
    A, B = O.Lattice(p), O.Lattice(p)
    A.build_cylinder(15.0, 14.5, 12.0)
    B.build_cylinder(15.0, 14.5, 12.0, d_solid=0.792)
    a, b = A.porosity(), B.porosity()
    x, y = np.arange(40 * 30) % 40, np.arange(40 * 30) // 40
    r = np.hypot(x - 15.0, y - 14.5)
    assert np.all(a[r <= 5.0] == 0.0) and np.all(b[r <= 5.0] == 0.792)
    assert np.all(b[r >= 7.0] == 1.0) and np.all(a[r >= 7.0] == 1.0)
    ramp = (r > 5.0) & (r < 7.0)
    assert np.allclose(1.0 - b[ramp], (1.0 - a[ramp]) * (1.0 - 0.792), rtol=0, atol=1e-15)
