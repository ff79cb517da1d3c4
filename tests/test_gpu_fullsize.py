"""Parity at the full sizes of the workloads, through the same library and
sweep grid the benchmark times.

- Vortex street, 1100 x 410 D2Q9 FP64: the whole field against the oracle
  over the first 1000 steps from the seeded initial state; one
  AA step pair on the developed shedding wake (the oracle takes the GPU state
  after 20 000 steps); the mean-flow dissipation adjoint on a short window
  from that state (both sides start from the same state, TOL_MEAN as in the
  small adjoint tests: the DISS source amplifies window rounding ~1e3).
- LES, 768 x 384 x 128 D3Q19 with the Smagorinsky closure (the benchmark
  lattice), FP64, FP32 and FP16S storage: sampled cells after 6000 steps, when
  the inflow has passed five diameters beyond the cylinder and its wake and
  shear layers have formed (half the samples lie in the near wake, where the
  closure raises tau_eff).  The oracle evaluates the collision of every
  upstream cell of a sampled cell one by one, so a sampled post-stream
  population f_i(x, t+1) = C_i(f(x - xi_i, t)) is checked without running the
  oracle over 38 M cells.
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_31707_amd import inputs as I
from tests.pairs import rel_err, say

pytestmark = pytest.mark.gpu
TOL = 1e-12
TOL_MEAN = 1e-11


def H():
    from paper_2606_31707_amd import hlbm
    return hlbm


def oracle_for(w):
    p = O.Params(stencil=w.stencil, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs, bc_x=O.BC_INLET_OUTLET,
                 bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile, u_in=w.u_max)
    L = O.Lattice(p)
    L.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode, box_half=w.box_half)
    L.init_equilibrium(1.0, I.initial_velocity(w))
    L.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
    return L


def gpu_for(w, precision=0, track_mean=False):
    h = H()
    G = h.Lattice(stencil=w.stencil, precision=precision, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs,
                  bc_x=h.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile,
                  u_in=w.u_max, track_mean_populations=track_mean)
    G.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode, box_half=w.box_half)
    G.init_equilibrium(1.0, I.initial_velocity(w))
    G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
    return G


def state_cols(w):
    return (np.arange(w.n) % w.nx) > 0  # the inlet column is not a state


@pytest.fixture(scope="module")
def vortex():
    w = I.vortex_re100()
    return w, gpu_for(w)


def test_vortex_full_field_first_steps(vortex):
    w, G = vortex
    say("full size vortex: first steps")
    L = oracle_for(w)
    assert rel_err(G.porosity(), L.porosity()) < 1e-15
    m = state_cols(w)
    for n in (1, 40, 959):
        L.step(n)
        G.run_primal(n)
        e = rel_err(G.populations(), L.populations(), m)
        print(f"after {n} more steps: populations {e:.3e}", flush=True)
        assert e < TOL


def test_vortex_developed_wake_step_pair(vortex):
    w, G = vortex
    say("full size vortex: developed wake")
    G.init_equilibrium(1.0, None)
    G.run_primal(20001)  # odd count: the check starts on the odd AA step
    f0 = G.populations()
    uy = G.moments()[1][1]
    assert np.abs(uy).max() > 1e-3  # a developed, non-trivial flow
    L = oracle_for(w)
    L.set_populations(f0)
    m = state_cols(w)
    for _ in range(3):
        L.step(1)
        G.run_primal(1)
        e = rel_err(G.populations(), L.populations(), m)
        print(f"developed wake step: populations {e:.3e}", flush=True)
        assert e < TOL


def test_vortex_mean_flow_adjoint(vortex):
    w, G = vortex
    say("full size vortex: mean-flow adjoint")
    G.init_equilibrium(1.0, None)
    G.run_primal(20000)
    L = oracle_for(w)
    L.set_populations(G.populations())
    n = 20
    L.window_reset()
    for _ in range(n):
        L.window_sample()
        L.step(1)
    G.window_reset()
    G.run_primal(n, accumulate=True)
    Jg, Jl = G.window_objective(), L.window_objective()
    # J_DISS is a sum of non-negative terms: a relative bound is meaningful
    assert abs(Jg - Jl) <= TOL_MEAN * abs(Jl), (Jg, Jl)
    L.adjoint_prepare(1)
    L.adjoint_iterate(30)
    G.solve_adjoint(H().SOURCE_MEAN, max_iters=30)
    m = state_cols(w)
    e_phi = rel_err(G.adjoint(), L.adjoint(), m)
    e_g = rel_err(G.gradient(), L.gradient())
    print(f"full size mean adjoint: J {Jg:.12e} vs {Jl:.12e}; phi {e_phi:.3e}, gradient {e_g:.3e}", flush=True)
    assert e_phi < TOL_MEAN and e_g < TOL_MEAN


def sampled_cells(w, count, seed):
    """Cells away from the inlet/outlet columns (their upstream cells are
    collided lattice cells): a quarter on the periodic seams in y and z, half
    in the near wake x_c - D/2 .. x_c + 4 D, |y - y_c| <= 1.5 D."""
    rng = np.random.default_rng(seed)
    x = rng.integers(2, w.nx - 2, count)
    y = rng.integers(0, w.ny, count)
    z = rng.integers(0, w.nz, count)
    y[: count // 8] = 0
    y[count // 8: count // 4] = w.ny - 1
    z[count // 4: 3 * count // 8] = 0
    z[3 * count // 8: count // 2] = w.nz - 1
    h = count // 2
    x[h:] = rng.integers(int(w.xc - 0.5 * w.D), int(w.xc + 4 * w.D), count - h)
    y[h:] = rng.integers(int(w.yc - 1.5 * w.D), int(w.yc + 1.5 * w.D), count - h)
    return x, y, z


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_les_sampled_cells(precision):
    """One step on a developed 3D LES field: sampled post-stream populations
    against the oracle's per-cell collision of their upstream cells, from the
    same stored state.  FP64: 1e-12 of the population scale.  FP32 storage and
    arithmetic: 1e-6 of the scale (FP32 rounding of the update and of the
    stored value).  FP16S: the GPU's FP32 result is stored as binary16 of
    f_i - w_i, so each value may also differ by half a binary16 unit of
    f_i - w_i (2^-11 relative) from the exact collision."""
    w = I.les_re3900()
    say("full size les: sampled cells", precision)
    G = gpu_for(w, precision)
    G.run_primal(6000)
    f0 = G.populations()
    G.run_primal(1)
    f1 = G.populations()
    d = G.porosity()
    G.close()
    c3, w3, _ = O.stencil(O.D3Q19)
    cx, cy, cz = c3[:, 0], c3[:, 1], c3[:, 2]
    x, y, z = sampled_cells(w, 1600, 77)
    cache, taus = {}, []
    worst = 0.0
    scale = np.abs(f1).max()
    for a, b, c in zip(x, y, z):
        cell = a + w.nx * (b + w.ny * c)
        for i in range(19):
            ux, uy, uz = a - cx[i], (b - cy[i]) % w.ny, (c - cz[i]) % w.nz
            up = int(ux + w.nx * (uy + w.ny * uz))
            if up not in cache:
                cache[up] = O.collide_cell(O.D3Q19, f0[:, up], d[up], w.tau, w.cs)
                taus.append(O.tau_eff(O.D3Q19, f0[:, up], w.tau, w.cs))
            ref = cache[up][i]
            if precision == 0:
                bound = 1e-12 * scale
            elif precision == 1:
                bound = 1e-6 * scale
            else:
                bound = 2.0 ** -11 * abs(ref - w3[i]) + 1e-6 * scale
            worst = max(worst, abs(f1[i, cell] - ref) / bound)
    dtau = max(taus) - w.tau
    print(f"les sampled cells (precision {precision}): max error / bound {worst:.3e} over {len(x)} cells; "
          f"max tau_eff - tau0 {dtau:.3e} (tau0 - 1/2 = {w.tau - 0.5:.3e})", flush=True)
    assert worst < 1.0
    # the closure is active on the sampled cells: the eddy viscosity exceeds
    # a tenth of the molecular one somewhere
    assert dtau > 0.1 * (w.tau - 0.5)
