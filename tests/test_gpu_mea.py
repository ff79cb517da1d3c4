"""GPU parity of the momentum-exchange drag J_MEA (Sec. 4, Eq. obj_mea)
against the oracle: the surface-node objective (steady and window mean), the
steady and mean-flow adjoints with its constant source, and the gradient, in
2D and 3D.  Adjoint inputs are synchronised as in the other adjoint tests
(the GPU lattice takes the oracle's state)."""
import math

import numpy as np
import pytest

import oracle as O
from tests.pairs import Spec, make_gpu, make_oracle, rel_err, say, state_mask

pytestmark = pytest.mark.gpu
TOL = 1e-12


def H():
    from paper_2606_31707_amd import hlbm
    return hlbm


def spec(stencil=O.D2Q9):
    if stencil == O.D2Q9:
        return Spec(nx=120, ny=41, tau=0.56, u_in=0.05, cyl=(40.0, 20.0, 10.0),
                    obj=(O.OBJ_MEA, (30, 8, 0), (50, 32, 0), math.pi * 10.0))
    return Spec(stencil=O.D3Q19, nx=48, ny=20, nz=6, tau=0.6, u_in=0.05, bc_z=O.BC_PERIODIC,
                cyl=(16.0, 9.5, 8.0), obj=(O.OBJ_MEA, (9, 3, 0), (23, 16, 5), math.pi * 8.0 * 6))


def j_tol(L):
    """First-order effect of 1e-12 population errors on the linear J."""
    g = L.mea_source()
    return TOL * np.abs(g).sum() * np.abs(L.populations()).max()


@pytest.mark.parametrize("stencil", [O.D2Q9, O.D3Q19])
def test_mea_steady_objective_and_adjoint(stencil):
    s = spec(stencil)
    say("mea steady", stencil)
    L, G = make_oracle(s), make_gpu(s)
    L.step(600)
    G.set_populations(L.populations())
    assert L.mea_surface().sum() > 8
    Jl, Jg = L.objective(), G.objective(0)
    print(f"J_MEA {Jg:.15e} vs {Jl:.15e}", flush=True)
    assert abs(Jg - Jl) < j_tol(L)
    L.adjoint_prepare(0)
    L.adjoint_iterate(300)
    G.solve_adjoint(H().SOURCE_STEADY, max_iters=300)
    m = state_mask(s)
    e_phi = rel_err(G.adjoint(), L.adjoint(), m)
    e_g = rel_err(G.gradient(), L.gradient())
    print(f"mea adjoint parity: phi {e_phi:.3e} gradient {e_g:.3e}", flush=True)
    assert e_phi < TOL and e_g < TOL


def test_mea_mean_flow_and_porosity_change():
    """Window mean of J_MEA and the mean-flow adjoint; the surface set
    follows a new porosity field set after the objective."""
    s = spec()
    say("mea mean flow")
    L, G = make_oracle(s), make_gpu(s)
    d = L.porosity()
    d[40 + 120 * 14] = 0.3  # a new surface node on the rim
    L.set_porosity(d)
    G.set_porosity(d)
    L.step(400)
    G.set_populations(L.populations())
    n = 60
    L.window_reset()
    for _ in range(n):
        L.window_sample()
        L.step(1)
    G.window_reset()
    G.run_primal(n, accumulate=True)
    Jl, Jg = L.window_objective(), G.window_objective()
    assert abs(Jg - Jl) < 10 * j_tol(L), (Jg, Jl)
    L.adjoint_prepare(1, 0.6)
    L.adjoint_iterate(200)
    G.solve_adjoint(H().SOURCE_MEAN, tau_adj=0.6, max_iters=200)
    e_phi = rel_err(G.adjoint(), L.adjoint(), state_mask(s))
    e_g = rel_err(G.gradient(), L.gradient())
    print(f"mea mean adjoint parity: phi {e_phi:.3e} gradient {e_g:.3e}", flush=True)
    # J_MEA is linear in f (no Pi): the mean-flow bound is the steady one
    assert e_phi < 1e-12 and e_g < 1e-12
