"""GPU parity of the window statistics (Sec. 3, the running time average) for
objective regions of every size: a region of at most 1/8 of the lattice has
its objective terms accumulated by a separate pass over the region, a larger
one inside the sweep.  Both must give the oracle's window mean of J and its
mean-flow adjoint and gradient, for FFA, DISS and J_MEA, with either
collision, and for a region in the outlet and wall corner."""
import math

import numpy as np
import pytest

import oracle as O
from tests.pairs import Spec, make_gpu, make_oracle, objective_tol, rel_err, say, state_mask

pytestmark = pytest.mark.gpu
TOL = 1e-12       # drag objectives: no dependence on Pi
TOL_MEAN = 1e-11  # J_DISS and the closure read Pi (see test_gpu_parity_adjoint)
NX, NY = 120, 41

CASES = {
    # name: (kind, lo, hi, u0, collision, cs)
    "diss_small": (O.OBJ_DISS, (50, 10, 0), (60, 30, 0), 0.0, 0, 0.0),
    "diss_large": (O.OBJ_DISS, (2, 0, 0), (118, 40, 0), 0.0, 0, 0.0),
    "diss_outlet": (O.OBJ_DISS, (110, 0, 0), (119, 10, 0), 0.0, 0, 0.0),
    "ffa_plane": (O.OBJ_FFA, (90, 0, 0), (90, 40, 0), 0.05, 0, 0.0),
    "mea_small": (O.OBJ_MEA, (30, 8, 0), (50, 32, 0), math.pi * 10.0, 0, 0.0),
    "mea_large": (O.OBJ_MEA, (5, 2, 0), (110, 38, 0), math.pi * 10.0, 0, 0.0),
    "diss_small_hrr": (O.OBJ_DISS, (50, 10, 0), (60, 30, 0), 0.0, 1, 0.15),
    "diss_large_hrr": (O.OBJ_DISS, (2, 0, 0), (118, 40, 0), 0.0, 1, 0.15),
}
SMALL = {"diss_small", "diss_outlet", "ffa_plane", "mea_small", "diss_small_hrr"}


def H():
    from paper_2606_31707_amd import hlbm
    return hlbm


def region_cells(lo, hi):
    return (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1)


def test_cases_cover_both_paths():
    for name, (_, lo, hi, *_rest) in CASES.items():
        assert (region_cells(lo, hi) * 8 <= NX * NY) == (name in SMALL), name


@pytest.mark.parametrize("name", sorted(CASES))
def test_window_mean_and_mean_flow_adjoint(name):
    kind, lo, hi, u0, coll, cs = CASES[name]
    s = Spec(nx=NX, ny=NY, tau=0.56 if cs == 0 else 0.52, cs=cs, u_in=0.05, cyl=(40.0, 20.0, 10.0),
             obj=(kind, lo, hi, u0), collision=coll, track_mean=coll == 1)
    say("window region", name)
    L, G = make_oracle(s), make_gpu(s)
    L.step(400)
    G.set_populations(L.populations())
    if kind == O.OBJ_MEA:
        jtol = 1e-12 * np.abs(L.mea_source()).sum() * np.abs(L.populations()).max()
    else:
        jtol = objective_tol(L, s, kind, lo, hi, u0)
    n = 60
    L.window_reset()
    for _ in range(n):
        L.window_sample()
        L.step(1)
    G.window_reset()
    G.run_primal(n, accumulate=True)
    assert G.window_count() == n
    Jl, Jg = L.window_objective(), G.window_objective()
    print(f"{name}: window J {Jg:.15e} vs {Jl:.15e} (bound {10 * jtol:.3e})", flush=True)
    assert abs(Jg - Jl) < 10 * jtol
    assert rel_err(G.populations(), L.populations(), state_mask(s)) < 1e-12
    L.adjoint_prepare(1, 0.6)
    L.adjoint_iterate(200)
    G.solve_adjoint(H().SOURCE_MEAN, tau_adj=0.6, max_iters=200)
    e_phi = rel_err(G.adjoint(), L.adjoint(), state_mask(s))
    e_g = rel_err(G.gradient(), L.gradient())
    print(f"{name}: mean adjoint parity phi {e_phi:.3e} gradient {e_g:.3e}", flush=True)
    tol = TOL if kind in (O.OBJ_FFA, O.OBJ_MEA) else TOL_MEAN
    assert e_phi < tol and e_g < tol
