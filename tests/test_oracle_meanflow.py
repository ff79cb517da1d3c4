"""Pins of the oracle's window and mean-flow path on a flow that changes from
step to step (a channel developing from the equilibrium around a porous
cylinder), beyond the steady-flow reduction in test_oracle_adjoint.py:

* Eq. averageObjective and the mean flow of Sec. 3.3: the window's mean
  populations and mean objective are the plain means of the states and
  objectives read step by step through the oracle's state accessors (R14: a
  mean over the samples; R15: the post-stream state each step reads);
* Eqs. adjoint_unsteady / gradients_unsteady for an objective linear in f
  (J_MEA, Sec. 4 Eq. obj_mea): its mean source equals its source at any
  state, so the mean-flow adjoint and gradient must equal the steady-path
  adjoint and gradient evaluated at the mean state (the BGK-HLBM Jacobian
  depends on the populations only through rho and j, whose means are the
  moments of the mean populations)."""
import numpy as np

import oracle as O


def _developing(kind, lo, hi, u0):
    L = O.Lattice(O.Params(nx=40, ny=15, tau=0.56, u_in=0.05))
    L.build_cylinder(10.0, 7.0, 5.0)
    L.set_objective(kind, lo, hi, u0=u0)
    L.init_equilibrium()
    L.step(30)
    return L


def _window(L, steps):
    L.window_reset()
    states, objectives = [], []
    for _ in range(steps):
        L.step(1)
        states.append(L.populations())
        objectives.append(L.objective())
        L.window_sample()
    return np.array(states), np.array(objectives)


def test_window_means_are_means_of_the_sampled_states():
    for kind, lo, hi in [(O.OBJ_FFA, (30, 0, 0), (30, 14, 0)), (O.OBJ_DISS, (2, 0, 0), (36, 14, 0))]:
        L = _developing(kind, lo, hi, 0.05)
        f, J = _window(L, 25)
        # the flow does change over the window (otherwise the pin is empty)
        assert np.abs(np.diff(f, axis=0)).max() > 1e-4
        assert np.ptp(J) > 1e-3 * np.abs(J).max()
        assert L.window_count() == 25
        fbar = L.window_mean_populations()
        assert np.abs(fbar - f.mean(axis=0)).max() < 1e-15 * np.abs(f).max() * 4
        assert abs(L.window_objective() - J.mean()) < 1e-13 * np.abs(J).max()


def test_linear_objective_mean_flow_equals_steady_path_at_the_mean_state():
    lo, hi, area = (3, 1, 0), (20, 13, 0), np.pi * 5.0
    L = _developing(O.OBJ_MEA, lo, hi, area)
    f, _ = _window(L, 25)
    assert np.abs(np.diff(f, axis=0)).max() > 1e-4
    fbar = L.window_mean_populations()
    L.adjoint_prepare(1)
    L.adjoint_iterate(400)
    phi_mean, g_mean = L.adjoint(), L.gradient()

    R = _developing(O.OBJ_MEA, lo, hi, area)
    R.set_populations(fbar)
    R.adjoint_prepare(0)
    R.adjoint_iterate(400)
    phi_steady, g_steady = R.adjoint(), R.gradient()

    assert np.abs(g_mean).max() > 0
    assert np.abs(phi_mean - phi_steady).max() < 1e-12 * np.abs(phi_steady).max()
    assert np.abs(g_mean - g_steady).max() < 1e-12 * np.abs(g_steady).max()
    # and differs from the steady path at the last state of the window, whose
    # Jacobian is another one (the comparison above is not vacuous)
    S = _developing(O.OBJ_MEA, lo, hi, area)
    S.set_populations(f[-1])
    S.adjoint_prepare(0)
    S.adjoint_iterate(400)
    assert np.abs(S.gradient() - g_steady).max() > 1e-6 * np.abs(g_steady).max()
