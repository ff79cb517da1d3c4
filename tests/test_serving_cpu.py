"""Scheduler logic on the CPU with the counting backend: admission by the
memory cap and slot limit in arrival order, every query gets exactly its
phase budgets, rejection of queries larger than the cap, latency records."""
import numpy as np
import pytest

from paper_2606_31707_amd import serving as S


def q(i, nx=128, Re=30.0, arrival=0.0, obj=S.OBJ_FFA):
    return S.Query(i, S.D2Q9, nx, nx // 2, 1, Re, obj, 100 + i, arrival=arrival)


def test_budgets_are_tick_multiples_and_window_only_when_unsteady():
    for nx in (128, 144, 512, 1024):
        for Re, unsteady in ((30.0, False), (120.0, True)):
            pre, win, adj = q(0, nx, Re).budgets(256)
            assert pre % 256 == 0 and win % 256 == 0 and adj % 256 == 0
            assert (win > 0) == unsteady
            assert pre + win >= 60 * nx and adj >= 30 * nx


def test_every_query_gets_its_budgets_and_finishes():
    b = S.FakeBackend()
    srv = S.Server(b, mem_cap_bytes=10**12, max_slots=8, tick=256)
    qs = [q(i, nx=128 + 16 * (i % 5), Re=20.0 + 30 * i) for i in range(12)]
    st = srv.run(qs, realtime=False)
    assert len(st.results) == 12 and not st.rejected
    for x in qs:
        pre, win, adj = x.budgets(256)
        assert b.steps[x.qid] == {S.PRIMAL: pre, S.WINDOW: win, S.ADJOINT: adj}
    assert b.resident == 0
    # at most 8 queries advance together
    assert max(len(e[1]) for e in b.log if e[0] == "advance") <= 8


def test_admission_respects_memory_cap_in_arrival_order():
    b = S.FakeBackend(bytes_per_cell=1)
    cap = 3 * 128 * 64  # room for three 128 x 64 queries
    srv = S.Server(b, mem_cap_bytes=cap, max_slots=100, tick=256)
    qs = [q(i) for i in range(7)]
    st = srv.run(qs, realtime=False)
    assert len(st.results) == 7
    adv = [e[1] for e in b.log if e[0] == "advance"]
    assert max(len(a) for a in adv) == 3
    order = [e[1] for e in b.log if e[0] == "acquire"]
    assert order == sorted(order)


def test_query_above_the_cap_is_rejected_without_blocking():
    b = S.FakeBackend(bytes_per_cell=1)
    srv = S.Server(b, mem_cap_bytes=128 * 64, max_slots=4, tick=256)
    st = srv.run([q(0), q(1, nx=1024), q(2)], realtime=False)
    assert [r.qid for r in st.results] == [0, 2] or sorted(r.qid for r in st.results) == [0, 2]
    assert st.rejected and st.rejected[0][0] == 1


def test_prepare_uses_mean_flow_only_for_unsteady_queries():
    b = S.FakeBackend()
    srv = S.Server(b, mem_cap_bytes=10**12, tick=256)
    srv.run([q(0, Re=30.0), q(1, Re=150.0)], realtime=False)
    prep = {e[1]: e[2] for e in b.log if e[0] == "prepare"}
    assert prep == {0: False, 1: True}


def test_realtime_latency_includes_queueing():
    b = S.FakeBackend(bytes_per_cell=1)
    srv = S.Server(b, mem_cap_bytes=128 * 64, max_slots=1, tick=256)
    qs = [q(i, arrival=0.001 * i) for i in range(3)]
    st = srv.run(qs)
    lat = sorted((r.qid, r.latency) for r in st.results)
    assert all(l >= 0 for _, l in lat)
    s = st.summary()
    assert s["completed"] == 3 and s["p99_latency_s"] >= s["p50_latency_s"]


def test_poisson_mix_matches_the_recipe():
    qs = S.poisson_mix(2000, rate=2.0, seed=2026)
    kinds = np.array([(x.stencil, x.nx) for x in qs])
    small = np.mean((kinds[:, 0] == 0) & (kinds[:, 1] <= 512))
    big = np.mean((kinds[:, 0] == 0) & (kinds[:, 1] == 1024))
    d3 = np.mean(kinds[:, 0] == 1)
    assert abs(small - 0.70) < 0.04 and abs(big - 0.25) < 0.04 and abs(d3 - 0.05) < 0.02
    arr = np.array([x.arrival for x in qs])
    assert np.all(np.diff(arr) > 0)
    assert abs(np.mean(np.diff(arr)) - 0.5) < 0.05
    assert all(20 <= x.Re <= 200 for x in qs)
