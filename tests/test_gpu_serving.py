"""Packed launches and the serving loop on the GPU: a lattice stepped in a
packed group gives the same bits as stepped by its own launches, FP64 members
match the oracle, and a query's gradient is the same alone and in a mix."""
import numpy as np
import pytest

import oracle as O
from paper_2606_31707_amd import serving as S
from tests.pairs import Spec, make_oracle, rel_err, say, state_mask

pytestmark = pytest.mark.gpu


def _lat(H, nx, ny, prec, tau=0.6, seed=0, stream=None):
    G = H.Lattice(stencil=H.D2Q9, precision=prec, nx=nx, ny=ny, tau=tau, u_in=0.05, stream=stream)
    rng = np.random.default_rng(seed)
    G.build_cylinder(nx / 4, (ny - 1) / 2, ny / 4, noise=rng.uniform(0, 0.05, nx * ny), noise_mode=H.NOISE_BOX,
                     box_half=ny / 2)
    G.init_equilibrium()
    G.set_objective(H.OBJ_DISS, (2, 0, 0), (nx - 3, ny - 1, 0))
    return G


def _same(a, b, prec):
    """Bitwise in every precision: the packed and the individual kernels run
    the same inlined per-cell code, and multiply-adds are fused per source
    expression only (-ffp-contract=on), so both round identically."""
    return np.array_equal(a, b)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_group_steps_equal_individual_launches(prec):
    from paper_2606_31707_amd import hlbm as H
    say("group vs individual", prec)
    shapes = [(130, 66), (64, 32), (200, 90)]
    solo = [_lat(H, nx, ny, prec, seed=i) for i, (nx, ny) in enumerate(shapes)]
    pack = [_lat(H, nx, ny, prec, seed=i) for i, (nx, ny) in enumerate(shapes)]
    for L in solo:
        L.run_primal(300)
        L.run_primal(101, accumulate=True)
    g = H.Group()
    g.set(pack, [H.GROUP_PRIMAL] * 3)
    g.step(300)
    g.set(pack, [H.GROUP_PRIMAL_WINDOW] * 3)
    g.step(101)
    g.synchronize()
    for a, b in zip(solo, pack):
        assert _same(a.populations(), b.populations(), prec)
        assert _same(np.array(a.window_objective()), np.array(b.window_objective()), prec)
    for L in solo:
        L.solve_adjoint(H.SOURCE_MEAN, max_iters=200)
    for L in pack:
        L.solve_adjoint(H.SOURCE_MEAN, max_iters=0)
    g.set(pack, [H.GROUP_ADJOINT] * 3)
    g.step(200)
    g.synchronize()
    for a, b in zip(solo, pack):
        assert _same(a.adjoint(), b.adjoint(), prec)
        assert _same(a.gradient(), b.gradient(), prec)


def test_group_hrr_and_mea_members_equal_individual_launches():
    """Packed launches of HRRLBM members (the collision is a template
    parameter of the packed kernels too) with a J_MEA and a J_DISS member:
    bitwise equal to the members' own launches."""
    from paper_2606_31707_amd import hlbm as H
    say("group hrr + mea")

    def lat(nx, ny, seed, kind):
        G = H.Lattice(stencil=H.D2Q9, precision=H.FP32, nx=nx, ny=ny, tau=0.58, u_in=0.05, collision=H.COLL_HRR,
                      track_mean_populations=True)
        G.build_cylinder(nx / 4, (ny - 1) / 2, ny / 4)
        G.init_equilibrium()
        if kind == H.OBJ_MEA:
            G.set_objective(kind, (2, 0, 0), (nx // 2, ny - 1, 0), u0=np.pi * ny / 4)
        else:
            G.set_objective(kind, (2, 0, 0), (nx - 3, ny - 1, 0))
        return G

    spec = [(120, 60, 0, H.OBJ_MEA), (96, 44, 1, H.OBJ_DISS)]
    solo = [lat(*a) for a in spec]
    pack = [lat(*a) for a in spec]
    for L in solo:
        L.run_primal(200)
        L.run_primal(61, accumulate=True)
    g = H.Group()
    g.set(pack, [H.GROUP_PRIMAL] * 2)
    g.step(200)
    g.set(pack, [H.GROUP_PRIMAL_WINDOW] * 2)
    g.step(61)
    g.synchronize()
    for a, b in zip(solo, pack):
        assert np.array_equal(a.populations(), b.populations())
        assert a.window_objective() == b.window_objective()
    for L in solo:
        L.solve_adjoint(H.SOURCE_MEAN, tau_adj=0.6, max_iters=150)
    for L in pack:
        L.solve_adjoint(H.SOURCE_MEAN, tau_adj=0.6, max_iters=0)
    g.set(pack, [H.GROUP_ADJOINT] * 2)
    g.step(150)
    g.synchronize()
    for a, b in zip(solo, pack):
        assert np.array_equal(a.adjoint(), b.adjoint())
        assert np.array_equal(a.gradient(), b.gradient())


def test_group_member_matches_oracle_fp64():
    from paper_2606_31707_amd import hlbm as H
    say("group vs oracle")
    s = Spec(nx=150, ny=41, tau=0.6, u_in=0.05, cyl=(37.5, 20.0, 10.25), obj=(O.OBJ_FFA, (100, 0, 0), (100, 40, 0), 0.05))
    L = make_oracle(s)
    G = H.Lattice(nx=150, ny=41, tau=0.6, u_in=0.05)
    G.build_cylinder(37.5, 20.0, 10.25)
    G.init_equilibrium()
    G.set_objective(H.OBJ_FFA, (100, 0, 0), (100, 40, 0), u0=0.05)
    other = _lat(H, 96, 48, 0, seed=5)
    grp = H.Group()
    grp.set([other, G], [H.GROUP_PRIMAL, H.GROUP_PRIMAL])
    grp.step(500)
    grp.synchronize()
    L.step(500)
    assert rel_err(G.populations(), L.populations(), state_mask(s)) < 1e-12
    G.set_populations(L.populations())
    L.adjoint_prepare(0)
    L.adjoint_iterate(300)
    G.solve_adjoint(H.SOURCE_STEADY, max_iters=0)
    grp.set([G, other], [H.GROUP_ADJOINT, H.GROUP_PRIMAL])
    grp.step(300)
    grp.synchronize()
    assert rel_err(G.gradient(), L.gradient()) < 1e-12


def _server():
    return S.Server(S.GPUBackend(pack_max_cells=300_000), mem_cap_bytes=8 << 30, max_slots=16, tick=256)


def test_result_is_the_same_alone_and_in_the_mix():
    say("alone vs mix")
    probe_small = S.Query(0, S.D2Q9, 160, 80, 1, 90.0, S.OBJ_DISS, 777)
    probe_big = S.Query(1, S.D2Q9, 1024, 512, 1, 35.0, S.OBJ_FFA, 778)  # above the packing limit
    mix = S.poisson_mix(10, rate=1e9, seed=5)
    mix = [m for m in mix if m.stencil == S.D2Q9 and m.nx <= 512]
    for i, m in enumerate(mix):
        m.qid = 10 + i
        m.arrival = 0.0
    alone = {}
    for pq in (probe_small, probe_big):
        st = _server().run([pq], realtime=False)
        alone[pq.qid] = st.results[0]
    st = _server().run(mix[:3] + [probe_small] + mix[3:] + [probe_big], realtime=False)
    got = {r.qid: r for r in st.results}
    for qid in (0, 1):
        assert got[qid].J == alone[qid].J
        assert np.array_equal(got[qid].grad, alone[qid].grad), qid
    assert len(st.results) == len(mix) + 2


class _RoundClock:
    """A clock that reads the number of rounds the backend has advanced, so
    that arrivals fall between given rounds whatever the GPU's speed."""

    def __init__(self):
        self.rounds = 0

    def __call__(self):
        return float(self.rounds)


def _counting_server(clock):
    b = S.GPUBackend(pack_max_cells=300_000)
    advance = b.advance

    def counted(work, n):
        advance(work, n)
        clock.rounds += 1

    b.advance = counted
    return S.Server(b, mem_cap_bytes=8 << 30, max_slots=16, tick=256)


def test_query_admitted_mid_run_gives_the_same_result():
    """Probe queries that arrive while the others are several rounds into
    their primal, window or adjoint phases: each result is bitwise the one it
    has alone (FP32, deterministic reductions)."""
    say("alone vs mix, mid-run arrivals")
    probe_small = S.Query(0, S.D2Q9, 176, 88, 1, 120.0, S.OBJ_DISS, 881)   # packed
    probe_big = S.Query(1, S.D2Q9, 1024, 512, 1, 30.0, S.OBJ_FFA, 882)     # own launches
    mix = [m for m in S.poisson_mix(12, rate=1e9, seed=9) if m.stencil == S.D2Q9 and m.nx <= 512][:6]
    for i, m in enumerate(mix):
        m.qid, m.arrival = 10 + i, 0.0
    alone = {}
    for pq in (probe_small, probe_big):
        c = _RoundClock()
        alone[pq.qid] = _counting_server(c).run([S.Query(**{**pq.__dict__, "arrival": 0.0})], clock=c).results[0]
    probe_small.arrival, probe_big.arrival = 5.0, 9.0  # after 5 and 9 rounds of the others
    c = _RoundClock()
    st = _counting_server(c).run(mix + [probe_small, probe_big], clock=c)
    got = {r.qid: r for r in st.results}
    assert len(got) == len(mix) + 2
    assert got[0].admitted >= 5.0 and got[1].admitted >= 9.0
    for qid in (0, 1):
        assert got[qid].J == alone[qid].J
        assert np.array_equal(got[qid].grad, alone[qid].grad), qid


def test_group_graph_replays_match_individual_launches():
    """On a stream of its own a group launches each 256-step run as one HIP
    graph, captured once and replayed while the members repeat.  Every replay
    (with the program's own eager work and synchronisations between them) and
    every recapture (new modes) gives bitwise the results of the members
    advanced one by one with their own launches."""
    import torch
    from paper_2606_31707_amd import hlbm as H
    say("group graph replays")
    stream = torch.cuda.Stream()
    grp = H.Group(stream=stream.cuda_stream)
    shapes = [(96, 48, 1), (128, 64, 2), (144, 72, 3)]
    packed = [_lat(H, nx, ny, 1, seed=sd, stream=stream.cuda_stream) for nx, ny, sd in shapes]
    solo = [_lat(H, nx, ny, 1, seed=sd) for nx, ny, sd in shapes]
    for rnd in range(4):  # the first run captures, the next three replay
        grp.set(packed, [H.GROUP_PRIMAL] * 3)
        grp.step(256)
        grp.synchronize()
        for a in solo:
            a.run_primal(256)
        for a, b in zip(solo, packed):
            assert np.array_equal(a.populations(), b.populations()), rnd
    for rnd in range(2):  # new modes: a new capture, then a replay
        grp.set(packed, [H.GROUP_PRIMAL_WINDOW] * 3)
        grp.step(128)
        grp.synchronize()
        for a in solo:
            a.run_primal(128, accumulate=True)
        for a, b in zip(solo, packed):
            assert np.array_equal(a.field(H.FIELD_MEAN_U), b.field(H.FIELD_MEAN_U)), rnd
    for lat in solo + packed:
        lat.solve_adjoint(H.SOURCE_MEAN, tau_adj=0.6, turb=H.TURB_FROZEN, max_iters=0)
    for rnd in range(3):
        grp.set(packed, [H.GROUP_ADJOINT] * 3)
        grp.step(64)
        grp.synchronize()
        for a in solo:
            a.solve_adjoint(H.SOURCE_MEAN, tau_adj=0.6, turb=H.TURB_FROZEN, max_iters=64, restart=False)
        for a, b in zip(solo, packed):
            assert np.array_equal(a.gradient(), b.gradient()), rnd
    grp.close()
