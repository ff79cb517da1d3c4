"""Pins of the oracle's forward tangent (App. C: the transient sensitivity
dJ(t)/dd . v carried along the primal trajectory).

- central differences of J(t) after a few steps from a common state with the
  porosity moved by +-eps v, for J_FFA, J_DISS (explicit d term), J_MEA and
  the Smagorinsky closure;
- on a converged steady flow the tangent settles to the steady adjoint's
  directional derivative g . v (tangent/adjoint duality of the same linear
  operator).
"""
import math

import numpy as np
import pytest

import oracle as O


def _channel(cs=0.0, tau=0.8):
    p = O.Params(nx=24, ny=12, tau=tau, cs=cs, u_in=0.05)
    L = O.Lattice(p)
    L.build_cylinder(7.0, 5.5, 4.0)
    L.init_equilibrium()
    return L


OBJS = {
    "ffa": (O.OBJ_FFA, (16, 0, 0), (16, 11, 0), 0.05),
    "diss": (O.OBJ_DISS, (2, 0, 0), (20, 11, 0), 0.0),
    "mea": (O.OBJ_MEA, (2, 0, 0), (13, 11, 0), math.pi * 4.0),
}


@pytest.mark.parametrize("obj,cs,tau", [("ffa", 0.0, 0.8), ("diss", 0.0, 0.8), ("mea", 0.0, 0.8),
                                        ("diss", 0.12, 0.52)])
def test_tangent_matches_central_differences(obj, cs, tau):
    kind, lo, hi, u0 = OBJS[obj]
    L = _channel(cs, tau)
    L.set_objective(kind, lo, hi, u0=u0)
    L.step(150)
    f0 = L.populations()
    d0 = L.porosity()
    rng = np.random.default_rng(9)
    v = rng.standard_normal(L.n) * (d0 > 0.01) * (d0 < 0.99)
    v /= np.linalg.norm(v)
    L.tangent_seed()
    L.tangent_step(v, 40)
    tj = L.tangent_objective(v)
    eps = 1e-6
    J = []
    for sgn in (1.0, -1.0):
        L.set_porosity(d0 + sgn * eps * v)
        L.set_populations(f0)
        L.step(40)
        J.append(L.objective())
    fd = (J[0] - J[1]) / (2 * eps)
    assert abs(tj - fd) < 1e-6 * abs(fd), (tj, fd)


def test_tangent_converges_to_steady_adjoint():
    L = _channel()
    kind, lo, hi, u0 = OBJS["ffa"]
    L.set_objective(kind, lo, hi, u0=u0)
    L.run_steady(200000, 1e-14, 100)
    L.adjoint_prepare(0)
    L.adjoint_solve(200000, 1e-14, 100)
    g = L.gradient()
    d0 = L.porosity()
    v = np.zeros(L.n)
    v[5 + 24 * 4] = 1.0
    v[8 + 24 * 6] = -0.5
    L.tangent_seed()
    prev = None
    for _ in range(40):
        L.tangent_step(v, 500)
        tj = L.tangent_objective(v)
        if prev is not None and abs(tj - prev) <= 1e-14 * abs(tj):
            break
        prev = tj
    assert np.allclose(L.porosity(), d0)
    assert abs(tj - g @ v) < 1e-9 * abs(g @ v), (tj, g @ v)
