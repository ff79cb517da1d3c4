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
  moments of the mean populations);
* the same equations for the objectives nonlinear in f (J_FFA, J_DISS): the
  window-mean source dJ/df and the mean dJ/dd against central differences
  of the per-cell objective at every sampled state."""
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


def test_mean_source_of_nonlinear_objectives_by_finite_differences():
    """Eqs. adjoint_unsteady / gradients_unsteady on a changing flow for the
    objectives nonlinear in f (J_FFA, J_DISS): the mean-flow adjoint's source
    is the window mean of dJ/df and the gradient's explicit term the window
    mean of dJ/dd.  Pinned by central differences of the per-cell objective
    at every sampled state (not by the oracle's derivative code): from
    phi = 0 the gradient is that mean dJ/dd, and one adjoint iteration gives
    phi = S^T(-mean dJ/df) (lambda = A^T 0 - mean dJ/df, Eq. adjoint_unsteady;
    S^T the oracle's explicit streaming transpose)."""
    W = 12
    for kind, lo, hi in [(O.OBJ_FFA, (30, 0, 0), (30, 14, 0)), (O.OBJ_DISS, (2, 0, 0), (36, 14, 0))]:
        L = _developing(kind, lo, hi, 0.05)
        f, _ = _window(L, W)
        assert np.abs(np.diff(f, axis=0)).max() > 1e-4  # a changing flow
        d = L.porosity()
        nx, q, n = 40, 9, 40 * 15
        g = np.zeros((q, n))
        gd = np.zeros(n)
        for t in range(W):
            for y in range(lo[1], hi[1] + 1):
                for x in range(lo[0], hi[0] + 1):
                    c = x + nx * y
                    fc = f[t][:, c].copy()
                    for i in range(q):
                        h = 1e-6
                        fp, fm = fc.copy(), fc.copy()
                        fp[i] += h
                        fm[i] -= h
                        g[i, c] += (O.objective_cell(O.D2Q9, kind, fp, d[c], 0.56, 0.05) -
                                    O.objective_cell(O.D2Q9, kind, fm, d[c], 0.56, 0.05)) / (2 * h)
                    hd = 1e-6
                    gd[c] += (O.objective_cell(O.D2Q9, kind, fc, d[c] + hd, 0.56, 0.05) -
                              O.objective_cell(O.D2Q9, kind, fc, d[c] - hd, 0.56, 0.05)) / (2 * hd)
        g /= W
        gd /= W
        L.adjoint_prepare(1)  # the window means (phi = 0 afterwards)
        grad0 = L.gradient()
        assert np.abs(grad0 - gd).max() <= 1e-8 * max(np.abs(gd).max(), 1e-30) + 1e-14
        if kind == O.OBJ_DISS:
            assert np.abs(gd).max() > 0  # the d-dependence of J_DISS is exercised
        L.adjoint_iterate(1)
        phi, phiv = L.adjoint(), L.adjoint_virtual()
        s_out, s_vout = L.apply_stream_transpose(-g)
        scale = np.abs(g).max()
        assert scale > 0
        assert np.abs(phi - s_out).max() < 1e-8 * scale
        assert np.abs(phiv - s_vout).max() < 1e-8 * scale
        # and the mean source is not the source at any one sampled state
        last = np.zeros((q, n))
        for y in range(lo[1], hi[1] + 1):
            for x in range(lo[0], hi[0] + 1):
                c = x + nx * y
                last[:, c] = O.dJdf_cell(O.D2Q9, kind, f[-1][:, c], d[c], 0.56, 0.05)
        assert np.abs(last - g).max() > 1e-6 * scale
