"""Host-side checks of the differentiation wrapper (no GPU): every call that
changes a lattice's porosity, state, window or objective advances its
generation, and a backward pass whose lattice changed after its forward pass
is refused before any adjoint work."""
import ctypes as C

import numpy as np
import pytest


class _FakeLib:
    """Stands in for libhlbm.so: every call succeeds and does nothing."""

    def __getattr__(self, name):
        return lambda *a, **k: 0


def _fake_lattice():
    from paper_2606_31707_amd import hlbm as H
    L = object.__new__(H.Lattice)
    L._lib = _FakeLib()
    L._h = C.c_void_p(None)
    L.desc = H.make_desc(nx=8, ny=4)
    L.q, L.n = 9, 32
    L.generation = 0
    return L


def test_state_changing_calls_advance_the_generation():
    L = _fake_lattice()
    calls = [
        lambda: L.set_porosity(np.ones(32)),
        lambda: L.build_cylinder(3.0, 2.0, 2.0),
        lambda: L.init_equilibrium(),
        lambda: L.set_populations(np.zeros((9, 32))),
        lambda: L.set_objective(0, (1, 0, 0), (1, 3, 0)),
        lambda: L.run_primal(5),
        lambda: L.window_reset(),
        lambda: L.reconfigure(0.7, 0.0, 0.03),
        lambda: L.run_tangent(np.zeros(32), 4, 2),
    ]
    for k, call in enumerate(calls):
        g = L.generation
        call()
        assert L.generation == g + 1, k
    g = L.generation
    L.objective(0)  # reading does not change the state
    L.synchronize()
    assert L.generation == g


def test_backward_after_a_later_change_is_refused():
    from paper_2606_31707_amd import autograd as A

    class Ctx:
        pass

    L = _fake_lattice()
    ctx = Ctx()
    ctx.lat, ctx.plan, ctx.shape, ctx.generation = L, A.Plan(), (32,), L.generation
    L.run_primal(1)  # another forward pass on the same lattice
    import torch
    with pytest.raises(RuntimeError, match="changed"):
        A.HLBMObjective.backward(ctx, torch.tensor(1.0, dtype=torch.float64))
