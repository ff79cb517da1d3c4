"""The device-memory footprint the serving admission uses: after a whole
query (primal with steady checks, window, adjoint with residual checks,
gradient) a lattice holds exactly hlbm_footprint_bytes of device memory, for
a dissipation query (a large objective box) and a J_MEA query (surface flags
and source)."""
import math

import pytest

import oracle as O
from tests.pairs import Spec, make_gpu, say

pytestmark = pytest.mark.gpu


def H():
    from paper_2606_31707_amd import hlbm
    return hlbm


@pytest.mark.parametrize("kind,stencil,prec", [(O.OBJ_DISS, 0, 1), (O.OBJ_MEA, 0, 0), (O.OBJ_DISS, 1, 2),
                                                (O.OBJ_FFA, 0, 0), (O.OBJ_FFA, 1, 1)])
def test_device_bytes_equal_the_footprint(kind, stencil, prec):
    """Large boxes (fused window terms), a J_MEA box, and drag planes (a
    region pass fed by the sweep's copy of the plane cells' state)."""
    if stencil == 0:
        s = Spec(nx=150, ny=41, tau=0.56, u_in=0.05, cyl=(40.0, 20.0, 10.0))
        lo, hi = {O.OBJ_DISS: ((2, 0, 0), (140, 40, 0)), O.OBJ_MEA: ((25, 5, 0), (55, 35, 0)),
                  O.OBJ_FFA: ((100, 0, 0), (100, 40, 0))}[kind]
    else:
        s = Spec(stencil=1, nx=48, ny=20, nz=8, tau=0.55, cs=0.1, bc_y=0, bc_z=0, inlet_profile=1, u_in=0.04,
                 cyl=(14.0, 9.5, 6.0))
        lo, hi = ((2, 0, 0), (40, 19, 7)) if kind == O.OBJ_DISS else ((36, 0, 0), (36, 19, 7))
    say("footprint", kind, stencil, prec)
    G = make_gpu(s, precision=prec)
    u0 = math.pi * 10.0 if kind == O.OBJ_MEA else 0.05
    G.set_objective(kind, lo, hi, u0=u0)
    G.run_primal(200, steady_tol=1e-12, check_every=50)
    G.run_primal(40, accumulate=True)
    G.solve_adjoint(H().SOURCE_MEAN, tau_adj=0.6, turb=H().TURB_FROZEN, max_iters=40, tol=1e-12, check_every=10)
    G.gradient()
    cells = (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1)
    fp = H().footprint_bytes(G.desc, True, True, cells, kind)
    used = G.device_bytes()
    print(f"footprint {fp} bytes, held {used} bytes", flush=True)
    assert used == fp
