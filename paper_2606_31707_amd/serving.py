"""Continuous-batching scheduler for gradient queries.

Each query is one run of the paper's Algorithm 1 (primal, optional window for
unsteady flows, adjoint, gradient) on its own porous-cylinder channel.  The
server keeps lattices resident on the device, admits waiting queries in
arrival order while the device-memory cap and the slot limit allow, and
advances every admitted query by `tick` steps per round: small 2D lattices
all together in one packed launch per step (hlbm_group_*), larger ones with
their own launches on their own streams, so work of different queries
overlaps on the GPU.  A query's arithmetic never depends on its neighbours
(packed members run the same per-cell code, each query always takes the same
route), so a result is the same alone and in the mix.

The scheduler talks to a backend; GPUBackend drives libhlbm.so, FakeBackend
(tests) only counts steps.
"""
from __future__ import annotations

import heapq
import math
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field, replace

import numpy as np

D2Q9, D3Q19 = 0, 1
FP64, FP32, FP16S = 0, 1, 2
OBJ_FFA, OBJ_DISS = 0, 1
PRIMAL, WINDOW, ADJOINT, DONE = "primal", "window", "adjoint", "done"


@dataclass
class Query:
    """A gradient query on a 2D (or 3D extruded) channel past a porous
    cylinder: D = ny/4 at (2D, (ny-1)/2), parabolic inflow u_max = 0.05,
    drag plane at x_c + 4D or dissipation box [x_c - 2D, x_c + 4D]."""
    qid: int
    stencil: int
    nx: int
    ny: int
    nz: int
    Re: float
    objective: int
    seed: int
    arrival: float = 0.0
    precision: int = FP32
    u_max: float = 0.05

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def D(self) -> float:
        return self.ny / 4.0

    @property
    def xc(self) -> float:
        return 2.0 * self.D

    @property
    def yc(self) -> float:
        return (self.ny - 1) / 2.0

    @property
    def tau(self) -> float:
        nu = (2.0 / 3.0) * self.u_max * self.D / self.Re
        return 3.0 * nu + 0.5

    @property
    def cs(self) -> float:
        """Smagorinsky closure (frozen in the adjoint) for the least viscous cases."""
        return 0.1 if self.tau < 0.52 else 0.0

    @property
    def unsteady(self) -> bool:
        return self.Re > 45.0

    def region(self):
        zhi = self.nz - 1
        if self.objective == OBJ_FFA:
            x = min(self.nx - 2, int(self.xc + 4 * self.D))
            return (x, 0, 0), (x, self.ny - 1, zhi)
        return (max(1, int(self.xc - 2 * self.D)), 0, 0), (min(self.nx - 2, int(self.xc + 4 * self.D)),
                                                            self.ny - 1, zhi)

    def budgets(self, tick: int):
        """(primal steps before the window, window steps, adjoint iterations),
        each a multiple of the tick: 60 nx primal steps in total, of which the
        last 30 nx form the window when the flow is unsteady; 30 nx adjoint
        iterations."""
        r = lambda v: int(math.ceil(v / tick)) * tick  # noqa: E731
        total, window, adj = r(60 * self.nx), (r(30 * self.nx) if self.unsteady else 0), r(30 * self.nx)
        return total - window, window, adj

    def lattice_updates(self, tick: int) -> int:
        a, b, c = self.budgets(tick)
        return (a + b + c) * self.cells


def poisson_mix(n: int, rate: float, seed: int = 2026):
    """The serving mix: 70 % D2Q9 with nx uniform in {128, 144, ..., 512} and
    ny = nx/2, 25 % D2Q9 1024 x 512, 5 % D3Q19 192 x 96 x 64; Re uniform in
    [20, 200]; drag or dissipation 50/50; Poisson arrivals at `rate` per s."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        u = rng.uniform()
        if u < 0.70:
            nx = int(rng.choice(np.arange(128, 513, 16)))
            st, ny, nz = D2Q9, nx // 2, 1
        elif u < 0.95:
            st, nx, ny, nz = D2Q9, 1024, 512, 1
        else:
            st, nx, ny, nz = D3Q19, 192, 96, 64
        out.append(Query(i, st, nx, ny, nz, float(rng.uniform(20, 200)), int(rng.integers(0, 2)),
                         10000 + i, arrival=t))
    return out


@dataclass
class _Active:
    q: Query
    lat: object
    phase: str
    left: int
    window: int
    adj: int
    t_admit: float
    t_done: float = 0.0
    J: float = 0.0
    grad: np.ndarray | None = None


@dataclass
class Result:
    qid: int
    arrival: float
    admitted: float
    done: float
    J: float
    grad: np.ndarray
    lattice_updates: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class Stats:
    results: list = field(default_factory=list)
    rejected: list = field(default_factory=list)
    makespan: float = 0.0
    ticks: int = 0

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results]) if self.results else np.zeros(1)
        lu = sum(r.lattice_updates for r in self.results)
        return {"completed": len(self.results), "rejected": len(self.rejected),
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_latency_s": float(lat.mean()), "makespan_s": self.makespan,
                "aggregate_MLUPS": lu / max(self.makespan, 1e-12) / 1e6, "ticks": self.ticks}


class Server:
    """Admission + continuous batching over a backend."""

    def __init__(self, backend, mem_cap_bytes: int, max_slots: int = 64, tick: int = 256, on_done=None):
        if tick % 2:
            raise ValueError("tick must be even (adjoint iterations come in AA pairs)")
        self.b = backend
        self.cap = int(mem_cap_bytes)
        self.max_slots = max_slots
        self.tick = tick
        self.waiting: deque = deque()
        self.active: list[_Active] = []
        self.on_done = on_done

    # -- admission --------------------------------------------------------
    def submit(self, q: Query, stats: Stats, now: float):
        if self.b.footprint(q) > self.cap:
            stats.rejected.append((q.qid, "footprint above the device-memory cap"))
            return
        self.waiting.append(q)

    def _admit(self, now: float):
        while self.waiting and len(self.active) < self.max_slots:
            q = self.waiting[0]
            if not self.b.reserve(q, self.cap):
                break  # head of line waits until memory frees up
            self.waiting.popleft()
            lat = self.b.acquire(q)
            pre, win, adj = q.budgets(self.tick)
            self.active.append(_Active(q, lat, PRIMAL if pre > 0 else WINDOW, pre if pre > 0 else win, win,
                                       adj, now))

    # -- one round ----------------------------------------------------------
    def _round(self, now_fn):
        work = [(a.lat, a.q, a.phase) for a in self.active]
        self.b.advance(work, self.tick)
        t = now_fn()
        still = []
        for a in self.active:
            a.left -= self.tick
            if a.left > 0:
                still.append(a)
                continue
            if a.phase == PRIMAL and a.window > 0:
                a.phase, a.left = WINDOW, a.window
            elif a.phase in (PRIMAL, WINDOW):
                a.J = self.b.prepare_adjoint(a.lat, a.q, mean=a.window > 0)
                a.phase, a.left = ADJOINT, a.adj
            else:
                a.grad = self.b.gradient(a.lat, a.q)
                a.phase, a.t_done = DONE, t
                self.b.release(a.lat, a.q)
                self.finished.append(a)
                if self.on_done:
                    self.on_done(a)
                continue
            still.append(a)
        self.active = still

    def run(self, queries, clock=time.perf_counter, realtime: bool = True) -> Stats:
        """Serves `queries` (arrival times in seconds from the start).  With
        realtime=False arrivals are taken as due whenever the server is idle
        (useful for tests)."""
        stats = Stats()
        self.finished: list[_Active] = []
        pending = [(q.arrival, q.qid, q) for q in queries]
        heapq.heapify(pending)
        t0 = clock()
        now = lambda: clock() - t0  # noqa: E731
        while pending or self.waiting or self.active:
            t = now()
            while pending and (not realtime or pending[0][0] <= t):
                _, _, q = heapq.heappop(pending)
                self.submit(q, stats, t)
            if not (self.waiting or self.active):
                if pending:  # idle until the next arrival
                    time.sleep(min(max(pending[0][0] - now(), 0.0), 0.005))
                continue
            self._admit(now())
            if not self.active:
                raise RuntimeError("no query admitted although the device is idle")
            self._round(now)
            stats.ticks += 1
        stats.makespan = now()
        for a in self.finished:
            stats.results.append(Result(a.q.qid, a.q.arrival if realtime else 0.0, a.t_admit, a.t_done, a.J,
                                        a.grad, a.q.lattice_updates(self.tick)))
        return stats


class GPUBackend:
    """libhlbm.so backend: resident lattices pooled by shape, small 2D
    lattices packed into one launch per step, the others on their own
    streams."""

    def __init__(self, pack_max_cells: int = 300_000, n_streams: int = 4):
        import torch

        from . import hlbm as H
        self.H = H
        self.torch = torch
        self.pack_max_cells = pack_max_cells
        self.group_stream = torch.cuda.Stream()
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self._next_stream = 0
        self.group = H.Group(stream=self.group_stream.cuda_stream)
        self.pool: OrderedDict = OrderedDict()  # key -> list of idle lattices
        self.resident = 0
        self._fp = {}

    def _key(self, q: Query):
        return (q.stencil, q.precision, q.nx, q.ny, q.nz)

    def packed(self, q: Query) -> bool:
        return q.stencil == D2Q9 and q.cells <= self.pack_max_cells

    def _desc(self, q: Query, stream):
        H = self.H
        return H.make_desc(stencil=q.stencil, precision=q.precision, nx=q.nx, ny=q.ny, nz=q.nz, tau=q.tau,
                           cs=q.cs, bc_x=H.BC_INLET_OUTLET, bc_y=H.BC_WALLS, bc_z=H.BC_PERIODIC,
                           inlet_profile=H.INLET_PARABOLIC, u_in=q.u_max, stream=stream)

    def footprint(self, q: Query) -> int:
        """Device bytes of a pooled lattice of the query's shape: its largest
        query (the window, the adjoint and the larger of the two objective
        regions, which a pooled lattice keeps once it has held it)."""
        k = self._key(q)
        if k not in self._fp:
            worst = 0
            for kind in (OBJ_FFA, OBJ_DISS):
                lo, hi = replace(q, objective=kind).region()
                cells = (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1)
                worst = max(worst, self.H.footprint_bytes(self._desc(q, None), True, True, cells, kind))
            self._fp[k] = worst
        return self._fp[k]

    def reserve(self, q: Query, cap: int) -> bool:
        """True if the query fits: a pooled lattice of its shape, or room for a
        new one after evicting idle lattices."""
        k = self._key(q)
        if self.pool.get(k):
            return True
        need = self.footprint(q)
        while self.resident + need > cap and self._evict_one():
            pass
        return self.resident + need <= cap

    def _evict_one(self) -> bool:
        for k, lst in self.pool.items():
            if lst:
                lat = lst.pop()
                self.resident -= self.footprint_key(k)
                lat.close()
                return True
        return False

    def footprint_key(self, k):
        return self._fp[k]

    def acquire(self, q: Query):
        H = self.H
        k = self._key(q)
        lst = self.pool.get(k)
        if lst:
            lat = lst.pop()
            lat.reconfigure(q.tau, q.cs, q.u_max)
        else:
            if self.packed(q):
                stream = self.group_stream.cuda_stream
            else:
                stream = self.streams[self._next_stream % len(self.streams)].cuda_stream
                self._next_stream += 1
            lat = H.Lattice(self._desc(q, stream))
            self.resident += self.footprint(q)
        rng = np.random.default_rng(q.seed)
        noise = rng.uniform(0.0, 0.05, q.cells)
        lat.build_cylinder(q.xc, q.yc, q.D, noise=noise, noise_mode=H.NOISE_BOX, box_half=2 * q.D)
        lat.init_equilibrium()
        lo, hi = q.region()
        lat.set_objective(q.objective, lo, hi, u0=q.u_max)
        return lat

    def advance(self, work, n: int):
        H = self.H
        members, modes = [], []
        for lat, q, phase in work:
            if self.packed(q):
                members.append(lat)
                modes.append({PRIMAL: H.GROUP_PRIMAL, WINDOW: H.GROUP_PRIMAL_WINDOW,
                              ADJOINT: H.GROUP_ADJOINT}[phase])
        # large lattices first, each on its own stream (asynchronous launches)
        for lat, q, phase in work:
            if self.packed(q):
                continue
            if phase == ADJOINT:
                lat.solve_adjoint(self._source(lat), tau_adj=0.0, turb=H.TURB_FROZEN, max_iters=n, restart=False)
            else:
                lat.run_primal(n, accumulate=(phase == WINDOW))
        self.group.set(members, modes)
        self.group.step(n)
        self.group.synchronize()
        for lat, q, phase in work:
            if not self.packed(q):
                lat.synchronize()

    def _source(self, lat):
        return getattr(lat, "_source", self.H.SOURCE_STEADY)

    def prepare_adjoint(self, lat, q: Query, mean: bool) -> float:
        H = self.H
        J = lat.objective(1 if mean else 0)
        lat._source = H.SOURCE_MEAN if mean else H.SOURCE_STEADY
        lat.solve_adjoint(lat._source, tau_adj=0.0, turb=H.TURB_FROZEN, max_iters=0, restart=True)
        lat.synchronize()
        return J

    def gradient(self, lat, q: Query) -> np.ndarray:
        return lat.gradient()

    def release(self, lat, q: Query):
        self.pool.setdefault(self._key(q), []).append(lat)


class FakeBackend:
    """Counts steps per query and phase (CPU tests of the scheduling logic)."""

    def __init__(self, bytes_per_cell: int = 100):
        self.bpc = bytes_per_cell
        self.resident = 0
        self.log = []
        self.steps = {}

    def footprint(self, q):
        return q.cells * self.bpc

    def reserve(self, q, cap):
        if self.resident + self.footprint(q) <= cap:
            return True
        return False

    def acquire(self, q):
        self.resident += self.footprint(q)
        self.steps[q.qid] = {PRIMAL: 0, WINDOW: 0, ADJOINT: 0}
        self.log.append(("acquire", q.qid))
        return q.qid

    def advance(self, work, n):
        for lat, q, phase in work:
            self.steps[q.qid][phase] += n
        self.log.append(("advance", tuple(sorted(q.qid for _, q, _ in work))))

    def prepare_adjoint(self, lat, q, mean):
        self.log.append(("prepare", q.qid, mean))
        return float(q.qid)

    def gradient(self, lat, q):
        return np.full(4, float(q.qid))

    def release(self, lat, q):
        self.resident -= self.footprint(q)
        self.log.append(("release", q.qid))
