"""Race canary: the library built with another tile shape (64 x 4 instead of
128 x 2) and every sweep's workgroup order flipped (XCD-renumbered where the
default keeps the dispatch order, and the other way round) must give bitwise
the same per-cell results -- populations, window means, adjoint populations,
gradients -- in every precision and for both collisions, because every slot
is read and written by exactly one thread per step.  A dependence on
execution order (a race) would show as a difference.  Only block reductions
(J) may differ, by their summation order."""
import numpy as np
import pytest

import oracle as O
from tests.pairs import Spec, say

pytestmark = pytest.mark.gpu


def _libs():
    from paper_2606_31707_amd import hlbm as H
    return H, H.load_library(), H.open_library(H.CANARY_PATH)


CASES = {
    # name: (spec, precision, steps before the window, window, adjoint iterations, closure treatment)
    "d2q9_fp64_diss": (Spec(nx=203, ny=57, tau=0.56, u_in=0.05, cyl=(50.0, 28.0, 14.0),
                            obj=(O.OBJ_DISS, (2, 0, 0), (190, 56, 0), 0.05)), 0, 301, 64, 150, O.TURB_FROZEN),
    "d2q9_fp16s_ffa": (Spec(nx=203, ny=57, tau=0.56, u_in=0.05, cyl=(50.0, 28.0, 14.0),
                            obj=(O.OBJ_FFA, (120, 0, 0), (120, 56, 0), 0.05)), 2, 300, 63, 150, O.TURB_FROZEN),
    "d3q19_fp32_les": (Spec(stencil=1, nx=71, ny=22, nz=13, tau=0.505, cs=0.1, bc_y=0, bc_z=0, inlet_profile=1,
                            u_in=0.04, cyl=(20.0, 10.5, 8.0), track_mean=True,
                            obj=(O.OBJ_DISS, (3, 0, 0), (60, 21, 12), 0.04)), 1, 151, 40, 80,
                       O.TURB_DIFFERENTIATED),
    "d2q9_fp32_hrr": (Spec(nx=131, ny=45, tau=0.52, cs=0.1, u_in=0.05, cyl=(35.0, 22.0, 12.0), collision=1,
                           track_mean=True, obj=(O.OBJ_DISS, (2, 0, 0), (120, 44, 0), 0.05)), 1, 200, 50, 100,
                      O.TURB_FROZEN),
}


def _run(H, lib, s, prec, spin, win, iters, turb):
    G = H.Lattice(lib=lib, stencil=s.stencil, precision=prec, nx=s.nx, ny=s.ny, nz=s.nz, tau=s.tau, cs=s.cs,
                  bc_x=s.bc_x, bc_y=s.bc_y, bc_z=s.bc_z, inlet_profile=s.inlet_profile, u_in=s.u_in,
                  track_mean_populations=s.track_mean, collision=s.collision)
    G.build_cylinder(*s.cyl)
    G.init_equilibrium()
    kind, lo, hi, u0 = s.obj
    G.set_objective(kind, lo, hi, u0=u0)
    G.run_primal(spin)
    G.run_primal(win, accumulate=True)
    out = {"f": G.populations(), "mean_u": G.field(H.FIELD_MEAN_U), "mean_rho": G.field(H.FIELD_MEAN_RHO),
           "J": G.window_objective()}
    G.solve_adjoint(H.SOURCE_MEAN, tau_adj=0.6, turb=turb, max_iters=iters)
    out.update({"phi": G.adjoint(), "g": G.gradient()})
    G.close()
    return out


@pytest.mark.parametrize("name", sorted(CASES))
def test_other_tile_shape_and_order_give_the_same_results(name):
    H, main, canary = _libs()
    s, prec, spin, win, iters, turb = CASES[name]
    say("race canary", name)
    a = _run(H, main, s, prec, spin, win, iters, turb)
    b = _run(H, canary, s, prec, spin, win, iters, turb)
    for k in ("f", "mean_u", "mean_rho", "phi", "g"):
        assert np.array_equal(a[k], b[k]), k
    assert abs(a["J"] - b["J"]) <= 1e-12 * abs(a["J"])  # summation order of the block partials
