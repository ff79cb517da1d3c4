"""Precision forms against the FP64 oracle: FP32 arithmetic with FP32 storage
and FP32 arithmetic with binary16 storage of f_i - w_i (FP16S).  Window
accumulators, objective and gradient reductions stay FP64 in both.  The
bounds below are the stated errors of each form, about three times the
measured ones (the kernels are deterministic, so these do not vary from run
to run): D2Q9 channel FP32 populations 5.3e-7, mean J 1.2e-5, gradient
1.3e-5; FP16S 8.5e-5, 3.9e-5, 4.4e-4; D3Q19 LES box populations FP32
4.9e-7, FP16S 2.1e-4."""
import numpy as np
import pytest

import oracle as O
from paper_2606_31707_amd import inputs as I
from tests.pairs import Spec, make_gpu, make_oracle, rel_err, say, state_mask

pytestmark = pytest.mark.gpu

# form: (populations after 1000 steps, mean J, gradient)
BOUNDS = {1: (1.6e-6, 3.5e-5, 4e-5), 2: (2.5e-4, 1.2e-4, 1.3e-3)}
# form: populations after 200 D3Q19 steps with the closure
BOUNDS_3D = {1: 1.5e-6, 2: 6e-4}


def channel(**kw):
    w = I.channel_re20()
    base = dict(stencil=0, nx=w.nx, ny=w.ny, tau=0.56, u_in=0.05, cyl=(w.xc, w.yc, w.D),
                obj=(O.OBJ_DISS, (2, 0, 0), (200, 40, 0), 0.05))
    base.update(kw)
    return Spec(**base)


@pytest.mark.parametrize("prec", [1, 2])
def test_precision_form_against_fp64_oracle(prec):
    s = channel()
    say("precision form", prec)
    L = make_oracle(s)
    G = make_gpu(s, precision=prec)
    L.step(1000)
    G.run_primal(1000)
    m = state_mask(s)
    e_f = rel_err(G.populations(), L.populations(), m)
    L.window_reset()
    for _ in range(200):
        L.window_sample()
        L.step(1)
    G.run_primal(200, accumulate=True)
    Jo, Jg = L.window_objective(), G.window_objective()
    e_J = abs(Jg - Jo) / abs(Jo)
    L.adjoint_prepare(1)
    L.adjoint_iterate(2000)
    G.solve_adjoint(1, max_iters=2000)
    e_g = rel_err(G.gradient(), L.gradient())
    go, gg = L.gradient(), G.gradient()
    cos = float(go @ gg / np.linalg.norm(go) / np.linalg.norm(gg))
    print(f"form {prec}: populations {e_f:.3e}, mean J {e_J:.3e}, gradient {e_g:.3e}, cosine {cos:.9f}",
          flush=True)
    bf, bJ, bg = BOUNDS[prec]
    assert e_f < bf and e_J < bJ and e_g < bg, (e_f, e_J, e_g)


@pytest.mark.parametrize("prec", [1, 2])
def test_d3q19_precision_forms(prec):
    rng = np.random.default_rng(41)
    n = 60 * 12 * 8
    u = np.zeros((3, n))
    u[0] = 0.04
    u += 0.004 * rng.uniform(-1, 1, (3, n))
    s = Spec(stencil=1, nx=60, ny=12, nz=8, tau=0.505, cs=0.1, bc_y=0, bc_z=0, inlet_profile=1, u_in=0.04,
             cyl=(18.0, 5.5, 6.0), init_u=u, obj=(O.OBJ_FFA, (40, 2, 0), (40, 9, 7), 0.04))
    say("d3q19 precision", prec)
    L = make_oracle(s)
    G = make_gpu(s, precision=prec)
    L.step(200)
    G.run_primal(200)
    e_f = rel_err(G.populations(), L.populations(), state_mask(s))
    print(f"d3q19 form {prec}: populations {e_f:.3e}", flush=True)
    assert e_f < BOUNDS_3D[prec]
