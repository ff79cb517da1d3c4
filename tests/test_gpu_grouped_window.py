"""Grouped window accumulation (FP32 and FP16 lattices): of every four
consecutive window steps the first three leave their values (drho, j,
tau_eff, f) in FP32 pending slots and the fourth adds them to the FP64 sums,
in step order, before its own; a run that ends inside a group is completed by
a flush.  The sums must be bitwise those of launches that add every step at
once -- the packed group launches, which never defer -- for windows that
start on either step parity and runs that end after 3, 2 and 1 pending
steps, with the Smagorinsky closure (the tau_eff sum) and the mean
populations tracked (the f sums, read by the differentiated-closure and HRR
adjoints)."""
import numpy as np
import pytest

from tests.pairs import say

pytestmark = pytest.mark.gpu


def _lattice(H, prec, coll):
    nx, ny, nz = 48, 24, 16
    G = H.Lattice(stencil=H.D3Q19, precision=prec, nx=nx, ny=ny, nz=nz, tau=0.52, cs=0.1,
                  bc_x=H.BC_INLET_OUTLET, bc_y=H.BC_PERIODIC, bc_z=H.BC_PERIODIC, inlet_profile=1, u_in=0.05,
                  track_mean_populations=True, collision=coll)
    G.build_cylinder(14.0, 11.5, 7.0)
    rng = np.random.default_rng(7)
    G.init_equilibrium(1.0, 0.05 * 0.02 * rng.uniform(-1.0, 1.0, 3 * nx * ny * nz))
    G.set_objective(H.OBJ_FFA, (30, 2, 0), (30, 21, nz - 1), u0=0.05)
    return G


@pytest.mark.parametrize("prec,coll", [(1, 0), (2, 0), (1, 1)])
def test_grouped_sums_equal_ungrouped_launches(prec, coll):
    from paper_2606_31707_amd import hlbm as H
    say("grouped window", prec, coll)
    solo, pack = _lattice(H, prec, coll), _lattice(H, prec, coll)
    # three plain steps: the window starts on an odd step; runs of 7, 10 and
    # 5 window steps end with 3, 2 and 1 steps pending (groups of four)
    solo.run_primal(3)
    for n in (7, 10, 5):
        solo.run_primal(n, accumulate=True)
    g = H.Group()
    g.set([pack], [H.GROUP_PRIMAL])
    g.step(3)
    g.set([pack], [H.GROUP_PRIMAL_WINDOW])
    g.step(22)
    g.synchronize()
    assert np.array_equal(solo.populations(), pack.populations())
    for fld in (H.FIELD_MEAN_RHO, H.FIELD_MEAN_U, H.FIELD_MEAN_TAU):
        assert np.array_equal(solo.field(fld), pack.field(fld)), fld
    assert solo.window_objective() == pack.window_objective()
    # the mean populations enter the adjoint through the differentiated
    # closure (and the HRR collision's frozen data)
    for L in (solo, pack):
        L.solve_adjoint(H.SOURCE_MEAN, tau_adj=0.6, turb=H.TURB_DIFFERENTIATED, max_iters=30)
    assert np.array_equal(solo.gradient(), pack.gradient())
    g.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_window_bytes_per_update(prec):
    """Algorithmic bytes of a window step: 16 B per dense FP64 sum and step
    (read and write); 10 B with the grouping (a read-modify-write per group
    of four steps plus three FP32 values written and read)."""
    from paper_2606_31707_amd import hlbm as H
    G = _lattice(H, prec, 0)
    bpu = G.bytes_per_update()
    m = 1 + 3 + 1 + 19  # rho, j, tau_eff, f
    rfrac = 20 * 16 / G.n
    per_sum = 16.0 if prec == 0 else (16.0 + 8.0 * 3) / 4
    assert bpu["primal_window"] == pytest.approx(bpu["primal"] + per_sum * m + rfrac * 16.0 * 12, rel=1e-12)
    G.close()


@pytest.mark.parametrize("prec", [1, 2, 0])
def test_les_window_means_full_size(prec):
    """The benchmark lattice (768 x 384 x 128 D3Q19 LES; FP32 and FP16S, and
    FP64 where every step adds at once; the streaming sweeps above the
    Infinity Cache): a 7-step window run in one call (one group of four,
    three steps flushed) against the same window run one step per call
    (every step flushed at once) is bitwise the same, and both are the plain
    FP64 means of the per-step densities and momenta (host arithmetic on the
    per-step fields, the rounding of the moments in the arithmetic type
    apart)."""
    from paper_2606_31707_amd import hlbm as H
    from paper_2606_31707_amd import inputs as I
    w = I.les_re3900()
    say("grouped window, full LES lattice", prec)

    def lattice():
        G = H.Lattice(stencil=w.stencil, precision=prec, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs,
                      bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile,
                      u_in=w.u_max)
        G.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode, box_half=w.box_half)
        G.init_equilibrium(1.0, I.initial_velocity(w))
        G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
        return G

    W = 7
    grouped, single = lattice(), lattice()
    grouped.run_primal(101)  # the window starts on an odd step
    grouped.run_primal(W, accumulate=True)
    single.run_primal(101)
    dr_sum = np.zeros(w.n)
    j_sum = np.zeros((3, w.n))
    first = None
    spread = 0.0
    for _ in range(W):
        rho, u = single.field(H.FIELD_RHO), single.field(H.FIELD_U)
        if first is None:
            first = rho.copy()
        spread = max(spread, float(np.abs(rho - first).max()))
        dr_sum += rho - 1.0
        j_sum += u * rho
        single.run_primal(1, accumulate=True)
    for fld in (H.FIELD_MEAN_RHO, H.FIELD_MEAN_U, H.FIELD_MEAN_TAU):
        assert np.array_equal(grouped.field(fld), single.field(fld)), fld
    mean_rho = 1.0 + dr_sum / W
    mean_u = j_sum / W / mean_rho
    cols = (np.arange(w.n) % w.nx) > 0  # the pinned inlet is not in the window
    e_rho = float(np.abs(grouped.field(H.FIELD_MEAN_RHO) - mean_rho)[cols].max())
    e_u = float(np.abs(grouped.field(H.FIELD_MEAN_U) - mean_u)[:, cols].max())
    print(f"full-size window: density spread over the window {spread:.2e}, "
          f"|mean rho - host| {e_rho:.2e}, |mean u - host| {e_u:.2e}", flush=True)
    # a step dropped or added would move the means by ~spread / W
    assert spread > 1e-5
    assert e_rho < 1e-7 and e_u < 1e-7
    grouped.close()
    single.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_grouped_and_packed_steps_mixed_in_one_window(prec):
    """One window advanced in turn by the lattice's own launches (grouped
    sums, runs ending inside a group) and by packed group launches (every
    step added at once) gives bitwise the sums of a window advanced by packed
    launches only: no pending value is lost or added twice across the two
    paths.  A member advanced outside its group since the set is refused."""
    from paper_2606_31707_amd import hlbm as H
    say("grouped and packed steps mixed", prec)
    mixed, pack = _lattice(H, prec, 0), _lattice(H, prec, 0)
    g_mixed, g_pack = H.Group(), H.Group()
    mixed.run_primal(2)
    g_pack.set([pack], [H.GROUP_PRIMAL])
    g_pack.step(2)
    g_pack.set([pack], [H.GROUP_PRIMAL_WINDOW])
    for n_own, n_packed in ((5, 3), (6, 2), (3, 7)):
        mixed.run_primal(n_own, accumulate=True)
        g_mixed.set([mixed], [H.GROUP_PRIMAL_WINDOW])
        g_mixed.step(n_packed)
        g_mixed.synchronize()
        g_pack.step(n_own + n_packed)
        g_pack.synchronize()
    for fld in (H.FIELD_MEAN_RHO, H.FIELD_MEAN_U, H.FIELD_MEAN_TAU):
        assert np.array_equal(mixed.field(fld), pack.field(fld)), fld
    assert mixed.window_objective() == pack.window_objective()
    # the packed tables hold the parity of the set: a member stepped by its
    # own launches in between would be stepped in the wrong AA layout
    mixed.run_primal(1)
    with pytest.raises(H.HlbmError):
        g_mixed.step(1)
    g_mixed.set([mixed], [H.GROUP_PRIMAL])
    g_mixed.step(1)
    g_mixed.synchronize()
    g_mixed.close()
    g_pack.close()
