"""Edge cases: the host-side validation of the C ABI (runs without a GPU:
every rejected descriptor or size fails before any device call), and on the
GPU the degenerate inputs of the method against the oracle — zero steps,
zero adjoint iterations (the gradient is then the explicit dJ/dd alone), an
all-solid and an all-fluid porosity field, and an empty tangent record."""
import numpy as np
import pytest

import oracle as O
from tests.pairs import Spec, make_gpu, make_oracle, rel_err, say, state_mask


def H():
    from paper_2606_31707_amd import hlbm
    return hlbm


@pytest.mark.parametrize("kw,why", [
    (dict(nx=1 << 16, ny=1 << 16, nz=1), "more than 2^31 cells"),
    (dict(stencil=1, nx=2048, ny=2048, nz=1024), "more than 2^31 cells (3D)"),
    (dict(nx=32, ny=16, nz=2), "D2Q9 with nz != 1"),
    (dict(nx=2, ny=16), "inlet/outlet channel with nx < 3"),
    (dict(nx=32, ny=16, tau=0.5), "tau = 1/2"),
    (dict(nx=32, ny=16, cs=-0.1), "negative Smagorinsky constant"),
    (dict(nx=32, ny=16, collision=7), "unknown collision model"),
    (dict(nx=32, ny=16, bc_y=2), "inlet/outlet on y"),
    (dict(nx=32, ny=16, u_in=float("nan")), "non-finite inflow"),
])
def test_descriptor_rejected_without_gpu(kw, why):
    h = H()
    d = h.make_desc(**kw)
    with pytest.raises(h.HlbmError) as e:
        h.footprint_bytes(d)
    assert e.value.status == h.E_INVALID, why
    with pytest.raises(h.HlbmError) as e:
        h.Lattice(d)
    assert e.value.status == h.E_INVALID, why


def test_largest_accepted_lattice_footprint():
    """2^31 cells is the largest lattice (32-bit tile indices); its footprint
    is computed on the host."""
    h = H()
    d = h.make_desc(stencil=h.D3Q19, precision=h.FP16S, nx=2048, ny=1024, nz=1024, bc_y=0, bc_z=0)
    b = h.footprint_bytes(d, False, False)
    assert b >= (1 << 31) * (19 * 2 + 4)


def _channel(**kw):
    base = dict(nx=67, ny=19, tau=0.6, u_in=0.05, cyl=(16.0, 9.0, 6.0),
                obj=(O.OBJ_DISS, (2, 0, 0), (60, 18, 0), 0.05))
    base.update(kw)
    return Spec(**base)


@pytest.mark.gpu
def test_zero_steps_and_zero_adjoint_iterations():
    s = _channel()
    say("edge: zero steps")
    L, G = make_oracle(s), make_gpu(s)
    f0 = G.populations()
    assert G.run_primal(0) == 0
    assert np.array_equal(G.populations(), f0)
    L.step(120)
    G.run_primal(120)
    G.set_populations(L.populations())
    L.adjoint_prepare(0)
    L.adjoint_iterate(0)
    it, res, st = G.solve_adjoint(H().SOURCE_STEADY, max_iters=0)
    assert it == 0
    assert np.abs(G.adjoint()).max() == 0.0
    g, gl = G.gradient(), L.gradient()
    assert np.abs(gl).max() > 0  # the explicit dJ_DISS/dd = -|u|^2/tau0 in the box
    assert rel_err(g, gl) < 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("d", [0.0, 1.0])
def test_uniform_porosity_fields(d):
    """All solid (d = 0: the equilibrium carries no velocity, the inflow is
    damped at the first column) and all fluid (d = 1: a plain channel)."""
    s = _channel(cyl=None, porosity=np.full(67 * 19, d))
    say("edge: uniform porosity", d)
    L, G = make_oracle(s), make_gpu(s)
    L.step(200)
    G.run_primal(200)
    assert rel_err(G.populations(), L.populations(), state_mask(s)) < 1e-12
    G.set_populations(L.populations())
    L.adjoint_prepare(0)
    L.adjoint_iterate(100)
    G.solve_adjoint(H().SOURCE_STEADY, max_iters=100)
    assert rel_err(G.gradient(), L.gradient()) < 1e-12


@pytest.mark.gpu
def test_empty_tangent_record_and_empty_window():
    s = _channel()
    G = make_gpu(s)
    rec = G.run_tangent(np.zeros(s.n), 3, 5)  # fewer steps than one record
    assert rec.shape == (0, 2)
    G.window_reset()
    with pytest.raises(H().HlbmError) as e:
        G.window_objective()
    assert e.value.status == H().E_STATE


@pytest.mark.gpu
def test_adjoint_not_converged_within_max_iters():
    """A tolerance the iteration budget cannot reach: W_NOT_CONVERGED, the
    iterations done and the last residual reported, the outputs valid (equal
    to a plain fixed-count run of the same length)."""
    s = _channel()
    say("edge: adjoint not converged")
    G = make_gpu(s)
    G.run_primal(300)
    it, res, st = G.solve_adjoint(H().SOURCE_STEADY, max_iters=40, tol=1e-14, check_every=10)
    assert st == H().W_NOT_CONVERGED and it == 40 and 1e-14 < res < 1.0
    g1 = G.gradient()
    it2, res2, st2 = G.solve_adjoint(H().SOURCE_STEADY, max_iters=40)
    assert st2 == H().OK and it2 == 40 and res2 == -1.0
    assert np.array_equal(G.gradient(), g1)


@pytest.mark.gpu
def test_non_finite_state_is_reported_as_diverged():
    """A host-supplied state with one non-finite population: the primal's
    steady check and the adjoint's residual check both end the call with
    E_DIVERGED (every kernel runs to completion on the NaN values)."""
    s = _channel()
    say("edge: diverged")
    G = make_gpu(s)
    G.run_primal(50)
    f = G.populations()
    f[3, 20 + 67 * 9] = np.nan
    G.set_populations(f)
    with pytest.raises(H().HlbmError) as e:
        G.run_primal(40, steady_tol=1e-10, check_every=10)
    assert e.value.status == H().E_DIVERGED
    G.set_populations(f)
    with pytest.raises(H().HlbmError) as e:
        G.solve_adjoint(H().SOURCE_STEADY, max_iters=40, tol=1e-10, check_every=10)
    assert e.value.status == H().E_DIVERGED
    # the lattice is still usable: a finite state runs normally again
    f[3, 20 + 67 * 9] = f[3, 21 + 67 * 9]
    G.set_populations(f)
    G.run_primal(10)
    assert np.isfinite(G.populations()).all()
