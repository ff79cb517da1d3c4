"""The sweep timing of the library (hlbm_profile_enable / hlbm_profile_get):
every launch of a timed run is counted once, blocks end with the caller's run
(steady checks, residual checks), a fresh enable clears the statistics, and
timing leaves the results bitwise unchanged."""
import numpy as np
import pytest

from tests.pairs import Spec, make_gpu, say

pytestmark = pytest.mark.gpu


def H():
    from paper_2606_31707_amd import hlbm
    return hlbm


def spec():
    return Spec(nx=160, ny=41, tau=0.56, u_in=0.05, cyl=(40.0, 20.0, 10.0),
                obj=(1, (2, 0, 0), (150, 40, 0), 0.0))


def test_every_launch_is_timed_once():
    say("timing counts")
    G = make_gpu(spec())
    G.profile_enable(7)
    G.run_primal(30)
    G.run_primal(23, steady_tol=1e-300, check_every=5)  # blocks end at every steady check
    G.window_reset()
    G.run_primal(11, accumulate=True)
    G.solve_adjoint(H().SOURCE_MEAN, tau_adj=0.6, max_iters=40, tol=1e-30, check_every=6)
    p = G.profile()
    assert p["primal"]["sampled"] == 53
    assert p["primal_window"]["sampled"] == 11
    assert p["adjoint"]["sampled"] == 40  # in chunks of 6 between residual checks
    for k in p:
        assert 0.5 < p[k]["mean_us"] < 5e4, (k, p[k])
    G.profile_enable(3)
    assert all(v["sampled"] == 0 for v in G.profile().values())
    G.profile_enable(0)
    G.run_primal(5)
    assert G.profile()["primal"]["sampled"] == 0


def test_timing_leaves_results_unchanged():
    say("timing bitwise")
    out = []
    for every in (0, 1, 5):
        G = make_gpu(spec())
        G.profile_enable(every)
        G.run_primal(40)
        G.window_reset()
        G.run_primal(21, accumulate=True)
        G.solve_adjoint(H().SOURCE_MEAN, tau_adj=0.6, max_iters=30)
        out.append((G.populations(), G.gradient()))
    for f, g in out[1:]:
        assert np.array_equal(f, out[0][0]) and np.array_equal(g, out[0][1])


@pytest.mark.parametrize("stencil,prec", [(0, 0), (0, 2), (1, 1), (1, 2)])
def test_copy_probe_leaves_the_state_unchanged(stencil, prec):
    """The bandwidth probe reads and writes back every population slot (own
    slots, or the odd step's neighbour slots), or pulls them into a second
    array it holds for the call: the lattice is bitwise unchanged, in either
    AA parity, with and without streaming hints, and holds no more memory."""
    say(f"copy probe stencil {stencil} precision {prec}")
    if stencil == 0:
        s = Spec(nx=133, ny=37, tau=0.56, u_in=0.05, cyl=(40.0, 18.0, 10.0))
    else:
        s = Spec(stencil=1, nx=37, ny=18, nz=9, tau=0.6, u_in=0.04, bc_y=0, bc_z=0, inlet_profile=1,
                 cyl=(12.0, 8.5, 6.0))
    G = make_gpu(s, precision=prec)
    for steps in (6, 7):  # even and odd parity afterwards
        G.run_primal(steps)
        f0 = G.populations()
        for pattern in (0, 1):
            for nt in (False, True):
                us = G.copy_probe(pattern, nt, 3)
                assert 0.0 < us < 1e5
        bytes_held = G.device_bytes()
        us = G.copy_probe(2, True, 3)  # into a second array of the call's own
        assert 0.0 < us < 1e5 and G.device_bytes() == bytes_held
        assert np.array_equal(G.populations(), f0)
    with pytest.raises(H().HlbmError):
        G.copy_probe(3, False, 1)
    with pytest.raises(H().HlbmError):
        G.copy_probe(0, False, 0)
