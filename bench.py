#!/usr/bin/env python3
"""Benchmark: whole-path throughput of the HLBM mean-flow adjoint on one GPU.

One step = one gradient query of the 3D LES workload (768 x 384 x 128 D3Q19,
spanwise-periodic porous cylinder D = 48, Re = 3900, Smagorinsky C_S = 0.1,
uniform inflow 0.04 with 1 % seeded velocity noise; FP32 populations, FP64
window statistics and reductions): porosity build (a1), equilibrium
initialisation (a2), a fixed block of primal steps (a3, a4) of which the last
ones form the FP64 window of the mean flow and of the drag objective on the
far-field plane (a5, a6), adjoint preparation on the mean flow with the
frozen-turbulence closure at the regularised adjoint relaxation time of the
paper's LES case (a7), a fixed block of adjoint sweeps (a8) and the gradient
assembly (a9).

`value` = (primal + adjoint lattice updates) / wall time of the whole query,
in MLUPS, inputs resident on the device.  Prints one JSON line; progress goes
to stderr.  `--workload vortex_re100` times the 2D vortex-street query
(1100 x 410, FP64, the whole 200 000-step run) instead; the default line also
carries one such query as an extra field.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2606_31707_amd import hlbm as H  # noqa: E402
from paper_2606_31707_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2606_31707_amd", f)
                  for f in ("csrc/hlbm_device.hpp", "csrc/hlbm_kernels.hpp", "build.py")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def shedding_period(uy: np.ndarray):
    """Median spacing of upward zero crossings of u_y - mean over the last
    half of the record (None if fewer than three crossings)."""
    s = uy[len(uy) // 2:]
    if len(s) < 16:
        return None
    s = s - s.mean()
    if np.abs(s).max() < 1e-7:
        return None
    i = np.nonzero((s[:-1] < 0) & (s[1:] >= 0))[0]
    if len(i) < 3:
        return None
    t = i + s[i] / (s[i] - s[i + 1])  # linear interpolation of the crossing
    return float(np.median(np.diff(t)))


class Query:
    """One gradient query on a resident lattice (the lattice is reused)."""

    def __init__(self, w: I.Workload, precision: int, primal_steps: int, adj_max: int, adj_tol: float,
                 adj_check: int, periods: int, tau_adj: float = 0.0):
        self.w = w
        self.G = H.Lattice(stencil=w.stencil, precision=precision, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau,
                           cs=w.cs, bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z,
                           inlet_profile=w.inlet_profile, u_in=w.u_max)
        self.noise = I.porosity_noise(w)
        self.T = primal_steps
        self.W_max = primal_steps // 2
        self.periods = periods
        self.adj_max, self.adj_tol, self.adj_check = adj_max, adj_tol, adj_check
        self.tau_adj = tau_adj
        self.G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)

    def run(self):
        w, G = self.w, self.G
        G.build_cylinder(w.xc, w.yc, w.D, noise=self.noise, noise_mode=w.noise_mode, box_half=w.box_half)
        G.init_equilibrium(1.0, I.initial_velocity(w))
        G.set_probe(*self._probe_xyz(), self.T)
        G.run_primal(self.T - self.W_max)
        P = shedding_period(G.probe())
        if P is not None and self.periods * P <= self.W_max:
            W = int(round(self.periods * P))
        else:  # no developed shedding yet: the last 20 % of the run
            W = self.T // 5
        G.run_primal(self.W_max - W)
        G.run_primal(W, accumulate=True)
        it, res, st = G.solve_adjoint(H.SOURCE_MEAN, tau_adj=self.tau_adj, max_iters=self.adj_max,
                                      tol=self.adj_tol, check_every=self.adj_check)
        self.converged = st == H.OK
        self.grad = G.gradient()
        self.J = G.window_objective()
        self.period, self.window, self.adj_iters, self.adj_res = P, W, it, res
        return self.T * w.n + it * w.n

    def _probe_xyz(self):
        px, py = self.w.extra.get("probe", (int(self.w.xc + 2 * self.w.D), int(self.w.yc)))
        return px, py, 0


def cpu_baseline(w: I.Workload, primal_steps: int, adj_iters: int):
    """The FP64 oracle (test infrastructure) on a bounded sample of the same
    workload, timed on the host cores."""
    import oracle as O
    p = O.Params(stencil=w.stencil, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs, bc_x=O.BC_INLET_OUTLET,
                 bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile, u_in=w.u_max)
    L = O.Lattice(p)
    L.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode, box_half=w.box_half)
    L.init_equilibrium(1.0, I.initial_velocity(w))
    L.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
    t0 = time.perf_counter()
    L.window_reset()
    for _ in range(primal_steps):
        L.window_sample()
        L.step(1)
    L.adjoint_prepare(1)
    L.adjoint_iterate(adj_iters)
    L.gradient()
    dt = time.perf_counter() - t0
    lu = (primal_steps + adj_iters) * w.n
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    return {"value": lu / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{w.name}: {primal_steps} primal steps each with a window sample, adjoint "
                      f"preparation, {adj_iters} adjoint iterations and the gradient ({dt:.1f} s of CPU)"}


# One step of the LES benchmark: a gradient query with a fixed budget in the
# proportions of the LES campaign (spin-up : window = 2 : 3, as 40 000 + 60 000
# steps) at 1/50 of its length, and the adjoint relaxation time the paper's LES
# case uses for stability (tau_adj = 0.6, frozen turbulence).
LES_SPINUP, LES_WINDOW, LES_ADJOINT, LES_TAU_ADJ, LES_CHECK = 800, 1200, 1000, 0.6, 250


class LesQuery:
    """One LES gradient query on a resident lattice (reused by every step);
    its seeded initial velocity is uploaded once and stays on the device."""

    def __init__(self, w: I.Workload, precision: int, spinup: int, window: int, adj_iters: int,
                 tau_adj: float, adj_check: int):
        import torch
        self.w = w
        self.G = H.Lattice(stencil=w.stencil, precision=precision, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau,
                           cs=w.cs, bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z,
                           inlet_profile=w.inlet_profile, u_in=w.u_max)
        self.u_init = torch.tensor(I.initial_velocity(w), device="cuda")
        self.grad = torch.empty(w.n, dtype=torch.float64, device="cuda")
        self.spinup, self.window, self.adj_iters = spinup, window, adj_iters
        self.tau_adj, self.adj_check = tau_adj, adj_check
        self.G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
        torch.cuda.synchronize()

    def run(self):
        w, G = self.w, self.G
        G.build_cylinder(w.xc, w.yc, w.D)
        G.init_equilibrium(1.0, self.u_init)
        G.run_primal(self.spinup)
        G.run_primal(self.window, accumulate=True)
        # a fixed block of adjoint sweeps; the relative change over the last
        # check interval is reported, the tolerance is never reached
        it, res, st = G.solve_adjoint(H.SOURCE_MEAN, tau_adj=self.tau_adj, turb=H.TURB_FROZEN,
                                      max_iters=self.adj_iters, tol=1e-12, check_every=self.adj_check)
        G.gradient(out=self.grad)
        self.J = G.window_objective()
        self.it, self.res, self.status = it, res, st
        return (self.spinup + self.window + it) * w.n


def cpu_baseline_les(w: I.Workload, spinup: int, window: int):
    """The FP64 oracle (test infrastructure) on a bounded sample of the LES
    query: primal steps and window steps (sample + step) on the full lattice,
    timed on the host cores.  The oracle's adjoint stores a dense q x q
    Jacobian per cell (218 GB here) and is not part of the sample."""
    import oracle as O
    p = O.Params(stencil=w.stencil, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs, bc_x=O.BC_INLET_OUTLET,
                 bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile, u_in=w.u_max)
    t0 = time.perf_counter()
    L = O.Lattice(p)
    L.build_cylinder(w.xc, w.yc, w.D)
    L.init_equilibrium(1.0, I.initial_velocity(w))
    L.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
    tset = time.perf_counter() - t0
    t0 = time.perf_counter()
    L.step(spinup)
    L.window_reset()
    for _ in range(window):
        L.window_sample()
        L.step(1)
    dt = time.perf_counter() - t0
    lu = (spinup + window) * w.n
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    return {"value": lu / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{w.name}: {spinup} primal steps and {window} window steps (window sample + step) of the "
                      f"FP64 oracle on the full lattice, {dt:.1f} s timed ({tset:.0f} s set-up untimed); its "
                      f"collide/stream loops use all {threads} threads, its window sample one; the oracle's "
                      f"adjoint keeps a dense q x q Jacobian per cell (218 GB here) and is not sampled"}


ORACLE_CASES = {
    # name: (workload, primal steps, adjoint iterations) for the all-core run;
    # the single-thread run takes 1/10 of them (at least one)
    "channel_re20": (I.channel_re20, 4000, 20000),
    "vortex_re100": (I.vortex_re100, 1000, 200),
    "les_re3900": (I.les_re3900, 20, 0),     # the oracle's dense per-cell adjoint Jacobians need 218 GB here
    "autograd_re40": (I.autograd_re40, 4000, 2000),
}


def oracle_worker(case: str, primal: int, adj: int):
    """One oracle timing in this process (thread count from OMP_NUM_THREADS):
    primal steps, then the steady adjoint's preparation and iterations."""
    import oracle as O
    w = ORACLE_CASES[case][0]()
    p = O.Params(stencil=w.stencil, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs, bc_x=O.BC_INLET_OUTLET,
                 bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile, u_in=w.u_max)
    L = O.Lattice(p)
    L.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode, box_half=w.box_half)
    L.init_equilibrium(1.0, I.initial_velocity(w))
    L.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
    t0 = time.perf_counter()
    L.step(primal)
    tp = time.perf_counter() - t0
    out = {"case": case, "cells": w.n, "primal_steps": primal, "primal_s": tp,
           "primal_MLUPS": primal * w.n / tp / 1e6}
    if adj > 0:
        t0 = time.perf_counter()
        L.adjoint_prepare(0)
        tprep = time.perf_counter() - t0
        t0 = time.perf_counter()
        L.adjoint_iterate(adj)
        ta = time.perf_counter() - t0
        out.update({"adjoint_prepare_s": tprep, "adjoint_iters": adj, "adjoint_s": ta,
                    "adjoint_MLUPS": adj * w.n / ta / 1e6})
    print(json.dumps(out), flush=True)


def gpu_rates(case: str, precision: int, primal: int, adj: int):
    """The library on the same workload: back-to-back primal steps and steady
    adjoint iterations, wall time per launch."""
    w = ORACLE_CASES[case][0]()
    G = H.Lattice(stencil=w.stencil, precision=precision, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs,
                  bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile,
                  u_in=w.u_max)
    G.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode,
                     box_half=w.box_half)
    G.init_equilibrium(1.0, I.initial_velocity(w))
    G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
    G.run_primal(20)
    G.synchronize()
    t0 = time.perf_counter()
    G.run_primal(primal)
    G.synchronize()
    tp = time.perf_counter() - t0
    G.solve_adjoint(H.SOURCE_STEADY, max_iters=20, turb=H.TURB_FROZEN)
    G.synchronize()
    t0 = time.perf_counter()
    G.solve_adjoint(H.SOURCE_STEADY, max_iters=adj, turb=H.TURB_FROZEN, restart=False)
    G.synchronize()
    ta = time.perf_counter() - t0
    G.close()
    return {"primal_MLUPS": primal * w.n / tp / 1e6, "adjoint_MLUPS": adj * w.n / ta / 1e6}


def report_oracle(all_threads: int):
    """The oracle timed beside the GPU: single-thread and all-core FP64
    oracle MLUPS (separate processes, OMP_NUM_THREADS 1 and all), and the
    library's FP64 (and, for the LES lattice, FP32) rates on the same inputs."""
    import subprocess
    rows = []
    for case, (wf, primal, adj) in ORACLE_CASES.items():
        row = {"case": case, "workload": wf().name}
        for threads, scale in ((1, 10), (all_threads, 1)):
            np_, na = max(1, primal // scale), (max(1, adj // scale) if adj else 0)
            env = dict(os.environ, OMP_NUM_THREADS=str(threads))
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-worker", case,
                                str(np_), str(na)], env=env, capture_output=True, text=True, check=True)
            rec = json.loads(r.stdout.strip().splitlines()[-1])
            rec["threads"] = threads
            row["oracle_1_thread" if threads == 1 else "oracle_all_threads"] = rec
            log(f"oracle {case} x{threads}: primal {rec['primal_MLUPS']:.2f} MLUPS"
                + (f", adjoint {rec['adjoint_MLUPS']:.2f} MLUPS" if adj else ""))
        gp = 4000 if wf().n < 10 ** 6 else 100
        row["gpu_fp64"] = gpu_rates(case, H.FP64, gp, gp)
        if wf().stencil == I.D3Q19:
            row["gpu_fp32"] = gpu_rates(case, H.FP32, gp, gp)
        log(f"gpu {case}: {row['gpu_fp64']}")
        rows.append(row)
    import platform
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    print(json.dumps({"report": "oracle beside the GPU", "host_cpu": cpu, "host_threads": all_threads,
                      "machine": platform.machine(), "cases": rows}), flush=True)


def kernel_source_hash() -> str:
    """SHA-256 over the device code and its build flags (the counters are
    tied to them)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def traffic_for(kernel_hash: str, kind: str, case: str = "les_fp32"):
    """HBM bytes per launch of a sweep kind from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_hash:
        return None
    try:
        return rec["cases"][case][kind]["bytes_per_launch"]
    except KeyError:
        return None


# Sweep measurements on lattices that do not fit in any cache: each case runs
# `launches` primal steps, window steps and mean-flow adjoint sweeps, and the
# bandwidth probe (a plain sweep's bytes without arithmetic) in four forms.
# name: (workload, precision, collision, track mean populations, closure in the adjoint)
SWEEP_CASES = {
    "les_fp32": (I.les_re3900, H.FP32, H.COLL_BGK, False, H.TURB_FROZEN),
    "les_fp32_diff": (I.les_re3900, H.FP32, H.COLL_BGK, True, H.TURB_DIFFERENTIATED),
    "les_fp16s": (I.les_re3900, H.FP16S, H.COLL_BGK, False, H.TURB_FROZEN),
    "les_fp64": (I.les_re3900, H.FP64, H.COLL_BGK, False, H.TURB_FROZEN),
    "les_fp32_hrr": (I.les_re3900, H.FP32, H.COLL_HRR, True, H.TURB_FROZEN),
    "les_fp16s_hrr": (I.les_re3900, H.FP16S, H.COLL_HRR, True, H.TURB_FROZEN),
    "grid2d_fp64": (I.grid2d_8192x4096, H.FP64, H.COLL_BGK, False, H.TURB_FROZEN),
    "grid2d_fp32": (I.grid2d_8192x4096, H.FP32, H.COLL_BGK, False, H.TURB_FROZEN),
    "grid2d_fp16s": (I.grid2d_8192x4096, H.FP16S, H.COLL_BGK, False, H.TURB_FROZEN),
}
PRECISION_NAMES = {H.FP64: "fp64", H.FP32: "fp32", H.FP16S: "fp16s"}
PROBES = [("copy_own", 0, False), ("copy_own_nt", 0, True), ("copy_odd", 1, False), ("copy_odd_nt", 1, True),
          ("copy_pull", 2, True)]


def report_sweeps(case: str, launches: int):
    """One sweep case: time per launch of every sweep kind (HIP events around
    back-to-back launches), algorithmic bytes and bandwidth, and the probe."""
    wf, prec, coll, track, turb = SWEEP_CASES[case]
    w = wf()
    G = H.Lattice(stencil=w.stencil, precision=prec, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs,
                  bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile, u_in=w.u_max,
                  track_mean_populations=track, collision=coll)
    G.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode, box_half=w.box_half)
    G.init_equilibrium(1.0, I.initial_velocity(w))
    G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
    G.run_primal(2)
    G.profile_enable(launches)
    G.run_primal(launches)
    G.run_primal(launches, accumulate=True)
    tau_adj = LES_TAU_ADJ if w.cs > 0 else 0.0
    G.solve_adjoint(H.SOURCE_MEAN, tau_adj=tau_adj, turb=turb, max_iters=launches)
    prof = G.profile()
    G.profile_enable(0)
    bpu = G.bytes_per_update()
    rows = {}
    for k in ("primal", "primal_window", "adjoint"):
        us = prof[k]["mean_us"]
        gbs = bpu[k] * w.n / us / 1e3
        rows[k] = {"us_per_launch": us, "bytes_per_update": bpu[k], "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS,
                   "GLUPS": w.n / us / 1e3}
    for name, pattern, nt in PROBES:
        us = G.copy_probe(pattern, nt, launches)
        gbs = bpu["primal"] * w.n / us / 1e3
        rows[name] = {"us_per_launch": us, "bytes_per_update": bpu["primal"], "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS}
    G.close()
    out = {"report": "sweeps", "case": case, "workload": w.name, "cells": w.n,
           "precision": PRECISION_NAMES[prec], "collision": "hrr" if coll == H.COLL_HRR else "bgk",
           "smagorinsky_cs": w.cs, "track_mean_populations": track,
           "adjoint_closure": "differentiated" if turb == H.TURB_DIFFERENTIATED else "frozen",
           "launches": launches, "sweeps": rows}
    log(json.dumps(out))
    print(json.dumps(out), flush=True)


def profile_commands(out: str):
    """The rocprofv3 commands behind the profiles/ summaries ({out}: their
    output directory): the benchmark command's kernel trace, and per sweep case
    a kernel trace and the FETCH_SIZE and WRITE_SIZE counters (one run each),
    plus the copy calibration of the counters."""
    cmds = {"bench_trace": f"rocprofv3 --kernel-trace --stats -d {out}/bench_trace -o bench --output-format csv "
                           f"-- python3 bench.py"}
    for c in SWEEP_CASES:
        run = f"python3 bench.py --report sweeps --sweep-case {c}"
        cmds[f"{c}/trace"] = (f"rocprofv3 --kernel-trace --stats -d {out}/{c}/trace -o sweep --output-format csv "
                              f"-- {run} --sweep-launches 20")
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            cmds[f"{c}/{ctr}"] = (f"rocprofv3 --pmc {ctr} -d {out}/{c}/{ctr} -o sweep --output-format csv "
                                  f"-- {run} --sweep-launches 6")
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        cmds[f"copy_{ctr}"] = (f"rocprofv3 --pmc {ctr} -d {out}/copy_{ctr} -o copy --output-format csv "
                               f"-- python3 bench.py --copy-calibration-mib 512")
    return cmds


def _itanium_kernel(name: str):
    """(base, template arguments) of a mangled hlbm kernel name (the trace
    leaves names with _Float16 arguments mangled), or None."""
    import re
    m = re.match(r"_ZN4hlbm\d+(k_\w+?)I(.*?)EEv", name)
    if not m:
        return None
    base, rest, args = m.group(1), m.group(2), []
    tok = {"d": "double", "f": "float", "DF16_": "_Float16"}
    while rest:
        t = re.match(r"Li(\d+)E|Lb([01])E|(DF16_|d|f)", rest)
        if not t:
            return None
        if t.group(1) is not None:
            args.append(t.group(1))
        elif t.group(2) is not None:
            args.append("true" if t.group(2) == "1" else "false")
        else:
            args.append(tok[t.group(3)])
        rest = rest[t.end():]
    return base, args


def kernel_kind(name: str):
    """(kind, parity) of a sweep kernel's (demangled or mangled) name, or
    (None, None)."""
    import re
    m = re.match(r"(?:void )?hlbm::(k_\w+)<([^>]*)>", name)
    if m:
        base, targs = m.group(1), [a.strip() for a in m.group(2).split(",")]
    else:
        it = _itanium_kernel(name)
        if it is None:
            return None, None
        base, targs = it
    if base in ("k_primal", "k_primal_stream", "k_primal_wstream"):
        return ("primal" if targs[3] == "0" else "primal_window"), targs[2]
    if base in ("k_window_region", "k_window_region_copy"):
        return "region", None
    if base == "k_adjoint":
        return "adjoint", targs[2]
    if base == "k_adjoint_stream":
        return "adjoint", "false"
    if base == "k_adjoint_pstream":
        return "adjoint", "true"
    if base == "k_copy_probe":
        odd, nt = targs[2] == "true", targs[3] == "true"
        return ("copy_odd" if odd else "copy_own") + ("_nt" if nt else ""), None
    if base == "k_copy_probe_pull":
        return "copy_pull", None
    return None, None


def les_dispatches(trace_dir: str, w, short):
    """Total duration, launch count and kernels per sweep kind of the
    dispatches on lattice `w` in a rocprofv3 kernel trace: sweeps with a grid
    of at least half the lattice's cells, region passes with the grid of w's
    objective region (rounded up to whole workgroups).  The reduced record is
    kept beside the trace (les_dispatches.json) so that the summary can be
    redone without the full trace file."""
    import csv
    cache = os.path.join(trace_dir, "les_dispatches.json")
    path = os.path.join(trace_dir, "bench_kernel_trace.csv")
    if not os.path.exists(path):
        return json.load(open(cache))
    region = int(np.prod([h - l + 1 for l, h in zip(w.lo, w.hi)]))
    region_grid = -(-region // 256) * 256
    acc = {}
    per_kernel = {}
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            name = short(r["Kernel_Name"])
            kind, _ = kernel_kind(name)
            if kind is None:
                continue
            if "Grid_Size" in r:
                grid = int(r["Grid_Size"])
            else:
                grid = int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y") or 1) * int(r.get("Grid_Size_Z") or 1)
            if kind == "region" and grid != region_grid:
                continue
            if kind != "region" and grid < w.n // 2:
                continue
            ns = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
            a = acc.setdefault(kind, {"ns": 0.0, "calls": 0, "kernels": []})
            a["ns"] += ns
            a["calls"] += 1
            k = per_kernel.setdefault((kind, name), [0.0, 0])
            k[0] += ns
            k[1] += 1
    for (kind, name), (ns, calls) in sorted(per_kernel.items()):
        acc[kind]["kernels"].append(f"`{name}` {calls} x {ns / calls / 1e3:.1f} us")
    with open(cache, "w") as fh:
        json.dump(acc, fh, indent=1)
    return acc


def summarize_profiles(d: str):
    """Writes the profiles/ summaries from the rocprofv3 CSV output under `d`
    (made by the profile_commands): the benchmark's kernel trace with its
    dominant sweep, one table per sweep case (trace duration, counter traffic
    over algorithmic bytes, the probe ceiling) and the traffic record the
    benchmark reads."""
    import csv

    def rows(path):
        with open(path, newline="") as fh:
            return list(csv.DictReader(fh))

    def short(name):
        name = name.replace("void ", "", 1)
        if name.startswith("hlbm::"):
            return name.split("(")[0]
        it = _itanium_kernel(name)
        if it is not None:  # mangled (_Float16 arguments): written out the same way
            return f"hlbm::{it[0]}<{', '.join(it[1])}>"
        return name.split("(")[0][:60]

    cmds = profile_commands(d)

    def copy_kib(sub, counter):
        v = [float(r["Counter_Value"]) for r in rows(os.path.join(d, sub, "copy_counter_collection.csv"))
             if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter]
        return float(np.mean(v))

    try:
        cf, cw = copy_kib("copy_FETCH_SIZE", "FETCH_SIZE"), copy_kib("copy_WRITE_SIZE", "WRITE_SIZE")
    except OSError as e:  # no calibration runs under d: the benchmark trace only
        log(f"calibration: {e}")
        cf = cw = float("nan")
    ff, wf = 512 * 1024 / cf, 512 * 1024 / cw
    traffic = {"kernel_source_sha256": kernel_source_hash(),
               "calibration": {"kernel": "__amd_rocclr_copyBuffer (torch copy_ of 512 MiB)", "fetch_kib": cf,
                               "write_kib": cw, "fetch_factor": ff, "write_factor": wf,
                               "commands": [cmds["copy_FETCH_SIZE"], cmds["copy_WRITE_SIZE"]]},
               "cases": {}}

    def per_kind(stats_rows):
        """total ns and launch counts per kind from a kernel-trace stats file."""
        acc = {}
        for r in stats_rows:
            k, _ = kernel_kind(short(r["Name"]))
            if k is None:
                continue
            a = acc.setdefault(k, {"ns": 0.0, "calls": 0, "kernels": []})
            a["ns"] += float(r["TotalDurationNs"])
            a["calls"] += int(r["Calls"])
            a["kernels"].append(f"`{short(r['Name'])}` {int(r['Calls'])} x {float(r['AverageNs']) / 1e3:.1f} us")
        return acc

    def launch_us(acc, kind):
        if kind not in acc or acc[kind]["calls"] == 0:
            return None
        t = acc[kind]["ns"]
        if kind == "primal_window" and "region" in acc:
            t += acc["region"]["ns"]  # the region pass belongs to the window step
        return t / acc[kind]["calls"] / 1e3

    def counters(sub, counter):
        acc = {}
        for r in rows(os.path.join(d, sub, "sweep_counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            k, _ = kernel_kind(short(r["Kernel_Name"]))
            if k is None:
                continue
            a = acc.setdefault(k, [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
        return acc

    for case in SWEEP_CASES if np.isfinite(cf) else ():
        rep = None
        try:
            for line in open(os.path.join(d, case, "report.json")):
                if line.startswith("{"):
                    rep = json.loads(line)
        except OSError:
            pass
        try:
            acc = per_kind(rows(os.path.join(d, case, "trace", "sweep_kernel_stats.csv")))
            fe, wr = counters(f"{case}/FETCH_SIZE", "FETCH_SIZE"), counters(f"{case}/WRITE_SIZE", "WRITE_SIZE")
        except OSError as e:
            log(f"{case}: {e}")
            continue
        wf_, prec, coll, track, turb = SWEEP_CASES[case]
        w = wf_()
        rec = {}
        lines = [f"# Sweeps: {w.name}, {PRECISION_NAMES[prec]}, "
                 f"{'HRRLBM' if coll == H.COLL_HRR else 'BGK-HLBM'}"
                 + (", Smagorinsky C_S 0.1" if w.cs > 0 else "")
                 + (", full mean populations tracked" if track else "")
                 + (", differentiated closure in the adjoint" if turb == H.TURB_DIFFERENTIATED else ""), "",
                 f"{w.n} cells; every sweep kind launched back to back (even and odd AA steps alternating). "
                 "Commands (run from the repository root on the MI355X box, `export TMPDIR=/tmp`):", "", "```",
                 cmds[f"{case}/trace"], cmds[f"{case}/FETCH_SIZE"], cmds[f"{case}/WRITE_SIZE"], "```", "",
                 f"Counter values are scaled by what the same counter reads for a plain 512 MiB device copy "
                 f"(FETCH_SIZE x{ff:.3f}, WRITE_SIZE x{wf:.3f}).", "",
                 "| sweep | B/LU (algorithmic) | trace us / launch | GB/s (algorithmic / trace) | % of 8 TB/s "
                 "| counter read MB | counter write MB | traffic / algorithmic | library event us |",
                 "|---|---|---|---|---|---|---|---|---|"]
        bpu = {k: v["bytes_per_update"] for k, v in rep["sweeps"].items()} if rep else {}
        for kind in ("primal", "primal_window", "adjoint", "copy_own", "copy_own_nt", "copy_odd", "copy_odd_nt",
                     "copy_pull"):
            us = launch_us(acc, kind)
            if us is None or kind not in bpu:
                continue
            alg = bpu[kind] * w.n
            nl = fe.get(kind, [0, 0])[1]
            rd = wt = None
            if nl:
                rd = fe[kind][0] / nl * ff * 1024
                wt = wr[kind][0] / wr[kind][1] * wf * 1024
                if kind == "primal_window" and "region" in fe:
                    rd += fe["region"][0] / nl * ff * 1024
                    wt += wr["region"][0] / nl * wf * 1024
            gbs = alg / us / 1e3
            ev = rep["sweeps"][kind]["us_per_launch"] if rep else float("nan")
            rec[kind] = {"us_per_launch": us, "algorithmic_bytes_per_launch": alg, "GB_s": gbs,
                         "frac": gbs / HBM_PEAK_GBS, "read_bytes_per_launch": rd, "write_bytes_per_launch": wt,
                         "bytes_per_launch": (rd + wt) if rd is not None else None,
                         "traffic_over_algorithmic": (rd + wt) / alg if rd is not None else None,
                         "library_event_us": ev, "kernels": acc[kind]["kernels"]
                         + (acc["region"]["kernels"] if kind == "primal_window" and "region" in acc else [])}
            tr = f"{(rd + wt) / alg:.3f}" if rd is not None else "—"
            lines.append(f"| {kind} | {bpu[kind]:.1f} | {us:.1f} | {gbs:.0f} | {gbs / HBM_PEAK_GBS * 100:.1f} | "
                         + (f"{rd / 1e6:.0f} | {wt / 1e6:.0f} | " if rd is not None else "— | — | ")
                         + f"{tr} | {ev:.1f} |")
        lines += ["", "`copy_*` rows: the bandwidth probe (`hlbm_copy_probe`), a plain sweep's bytes (populations "
                      "read and written in place, porosity read) with no arithmetic; `_nt` with nontemporal hints; "
                      "`own` the even step's own slots, `odd` the odd step's upstream slots; `pull` the two-array "
                      "pattern (upstream slots read, own slots of a second array written with nontemporal hints). "
                      "The window row includes the region pass of the drag plane.", "", "Kernels (trace):", ""]
        for kind, r in rec.items():
            lines.append(f"- {kind}: " + "; ".join(r["kernels"]))
        traffic["cases"][case] = rec
        fname = f"sweeps_{w.name}_{PRECISION_NAMES[prec]}" + ("_hrr" if coll == H.COLL_HRR else "") \
                + ("_diff" if turb == H.TURB_DIFFERENTIATED else "") + ".md"
        with open(os.path.join(ROOT, "profiles", fname), "w") as fh:
            fh.write("\n".join(lines) + "\n")
        log(f"wrote profiles/{fname}")

    # the benchmark command's own kernel trace
    try:
        stats = rows(os.path.join(d, "bench_trace", "bench_kernel_stats.csv"))
        live = None
        try:
            live = json.load(open(os.path.join(d, "bench.json")))
        except (OSError, ValueError):
            pass
        # per-launch figures from the LES lattice's own dispatches (the serving
        # stream's small D3Q19 lattices run some of the same kernels)
        acc = les_dispatches(os.path.join(d, "bench_trace"), I.les_re3900(), short)
        lines = ["# Kernel trace of the benchmark command (les_re3900_768x384x128, D3Q19 FP32)", "",
                 "Command (run from the repository root on the MI355X box, `export TMPDIR=/tmp`):", "", "```",
                 cmds["bench_trace"], "```", "",
                 "The default benchmark: one warm-up and three timed LES gradient queries, the extra 2D vortex-street "
                 "queries and the CPU-oracle sample.", "",
                 "| kernel | calls | mean us | min us | max us | share % |", "|---|---|---|---|---|---|"]
        for r in stats[:40]:
            lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                         f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                         f"{float(r['Percentage']):.2f} |")
        lines += ["", "Per launch of each LES sweep kind (trace durations of the dispatches on the LES lattice, "
                      "selected by grid size; a window step = its sweep + the region pass):", ""]
        w = I.les_re3900()
        for kind in ("primal", "primal_window", "adjoint"):
            us = launch_us(acc, kind)
            if us is None:
                continue
            ev = live["sweeps"][kind]["us_per_launch"] if live else None
            lines.append(f"- {kind}: {us:.1f} us per launch (trace)" +
                         (f"; the benchmark's own HIP-event figure in an unprofiled run of the same command: "
                          f"{ev:.1f} us" if ev else ""))
        for kind in ("primal", "primal_window", "adjoint", "region"):
            if kind in acc:
                lines.append(f"  - {kind}: " + "; ".join(acc[kind]["kernels"]))
        if live:
            lines += ["", f"Dominant sweep of the benchmark line: {live['roofline']['kind']} "
                          f"({live['roofline']['achieved']:.0f} GB/s algorithmic, frac {live['roofline']['frac']:.3f})."]
        with open(os.path.join(ROOT, "profiles", "bench_trace_les_re3900_768x384x128.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    except OSError as e:
        log(f"bench trace: {e}")
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(traffic, fh, indent=1)
        fh.write("\n")
    print(json.dumps({"cases": list(traffic["cases"])}))


def report_differentiation(n_fields: int, fd_fields: int, fd_dirs: int):
    """The differentiation batch: seeded porosity fields on the 400 x 160
    Re = 40 channel (drag), gradients through the torch.autograd.Function in
    FP64 and FP32 at converged steady states, and central differences of the
    converged FP64 objective along seeded unit directions (eps = 1e-4)."""
    import torch
    from paper_2606_31707_amd import autograd as A
    p64 = A.Plan(primal_steps=400000, steady_tol=1e-13, check_every=500, adjoint_iters=400000,
                 adjoint_tol=1e-13)
    p32 = A.Plan(primal_steps=400000, steady_tol=1e-6, check_every=500, adjoint_iters=400000,
                 adjoint_tol=1e-6)
    rows, fd = [], []
    lat = {}
    for k in range(n_fields):
        seed = 400 + k
        w = I.autograd_re40(seed)
        for prec in (H.FP64, H.FP32):
            if prec not in lat:
                lat[prec] = A.make_lattice(precision=prec, nx=w.nx, ny=w.ny, tau=w.tau, u_in=w.u_max)
                lat[prec].set_objective(H.OBJ_FFA, w.lo, w.hi, u0=w.u0)
        G = lat[H.FP64]
        G.build_cylinder(w.xc, w.yc, w.D, noise=I.porosity_noise(w), noise_mode=w.noise_mode,
                         box_half=w.box_half)
        d0 = torch.tensor(G.porosity(), device="cuda")
        grads, Js, secs = {}, {}, {}
        for prec, plan in ((H.FP64, p64), (H.FP32, p32)):
            d = d0.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            J = A.objective(d, lat[prec], plan)
            J.backward()
            torch.cuda.synchronize()
            secs[prec] = time.perf_counter() - t
            grads[prec], Js[prec] = d.grad.detach().cpu().numpy(), J.item()
        g64, g32 = grads[H.FP64], grads[H.FP32]
        rows.append({"seed": seed, "J_fp64": Js[H.FP64], "J_fp32_rel": abs(Js[H.FP32] - Js[H.FP64]) / abs(Js[H.FP64]),
                     "grad_fp32_rel_l2": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64)),
                     "grad_fp32_cosine": float(g32 @ g64 / np.linalg.norm(g32) / np.linalg.norm(g64)),
                     "seconds_fp64": secs[H.FP64], "seconds_fp32": secs[H.FP32]})
        log(rows[-1])
        if k < fd_fields:
            dn = d0.cpu().numpy()
            inside = (dn > 1e-3) & (dn < 1 - 1e-3)
            for ds in range(500, 500 + fd_dirs):
                v = np.random.default_rng(ds).standard_normal(w.n) * inside
                v /= np.linalg.norm(v)
                vt = torch.tensor(v, device="cuda")
                Jp = A.objective(d0 + 1e-4 * vt, G, p64).item()
                Jm = A.objective(d0 - 1e-4 * vt, G, p64).item()
                fdv = (Jp - Jm) / 2e-4
                ad = float(g64 @ v)
                fd.append({"seed": seed, "direction_seed": ds, "adjoint": ad, "fd": fdv,
                           "rel_err": abs(ad - fdv) / abs(fdv)})
                log(fd[-1])
    rel = [r["grad_fp32_rel_l2"] for r in rows]
    out = {"report": "differentiation batch (400x160, Re 40, drag)", "fields": len(rows),
           "fd_checks": len(fd), "fd_max_rel_err": max(f["rel_err"] for f in fd) if fd else None,
           "fp32_grad_rel_l2_median": float(np.median(rel)), "fp32_grad_rel_l2_max": float(np.max(rel)),
           "fp32_grad_cosine_min": float(min(r["grad_fp32_cosine"] for r in rows)),
           "rows": rows, "fd": fd}
    print(json.dumps(out), flush=True)


def report_serving(n: int, rate: float, cap_gib: float, tick: int, slots: int):
    """Continuous-batching serving of a Poisson stream of gradient queries
    (mixed D2Q9 / D3Q19 sizes, FP32): p50/p99 latency and aggregate MLUPS."""
    from paper_2606_31707_amd import serving as S
    qs = S.poisson_mix(n, rate)
    t0 = time.perf_counter()

    def done(a):
        log(f"[{time.perf_counter() - t0:7.2f} s] query {a.q.qid} ({a.q.nx}x{a.q.ny}x{a.q.nz}, Re {a.q.Re:.0f}) "
            f"latency {a.t_done - a.q.arrival:.2f} s")

    srv = S.Server(S.GPUBackend(), mem_cap_bytes=int(cap_gib * (1 << 30)), max_slots=slots, tick=tick,
                   on_done=done)
    st = srv.run(qs)
    out = {"report": "serving", "queries": n, "rate_qps": rate, "mem_cap_GiB": cap_gib, "tick": tick,
           "max_slots": slots, "precision": "fp32", **st.summary()}
    print(json.dumps(out), flush=True)


def report_les(spinup: int, window: int, adj_iters: int, forms, collision: int = 0, tau_adjs=(0.0, 0.6),
               adj_tol: float = 1e-8):
    """The 3D LES case (768 x 384 x 128 D3Q19, Smagorinsky C_S = 0.1, Re 3900,
    drag plane): FP32, FP16-shifted and FP64 population storage with FP64
    window accumulation; the mean flow of each form against the FP64 form
    beside its own statistical error (difference of the two window halves);
    mean-flow drag adjoints with the frozen (FTA) and the differentiated
    closure, tau_adj in {tau0, 0.6}; sweep rates."""
    w = I.les_re3900()
    names = {H.FP64: "fp64", H.FP32: "fp32", H.FP16S: "fp16s"}
    res, means, grads = {}, {}, {}
    chunk = 2000

    def l2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def cos(a, b):
        return float(a @ b / np.linalg.norm(a) / np.linalg.norm(b))

    for prec in forms:
        name = names[prec]
        # the differentiated closure (and every HRR mean-flow adjoint) needs the full mean populations
        diff = prec == H.FP32
        track = diff or collision == H.COLL_HRR
        t0 = time.perf_counter()
        G = H.Lattice(stencil=w.stencil, precision=prec, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs,
                      bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile,
                      u_in=w.u_max, track_mean_populations=track, collision=collision)
        G.build_cylinder(w.xc, w.yc, w.D)
        G.init_equilibrium(1.0, I.initial_velocity(w))
        G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
        G.profile_enable(97)
        r = {"track_mean_populations": track}
        ok = True
        for done in range(0, spinup, chunk):
            G.run_primal(min(chunk, spinup - done))
            umax = float(np.abs(G.field(H.FIELD_U)[0]).max())
            log(f"les {name}: step {done + chunk}, max u_x {umax:.4f} ({time.perf_counter() - t0:.0f} s)")
            if not np.isfinite(umax) or umax > 0.4:
                ok = False
                break
        r["stable"] = ok
        if not ok:
            res[name] = r
            G.close()
            continue
        G.window_reset()
        half = window // 2
        for k in range(2):
            for done in range(0, half, chunk):
                G.run_primal(min(chunk, half - done), accumulate=True)
                log(f"les {name}: window half {k}, step {done + chunk} ({time.perf_counter() - t0:.0f} s)")
            if k == 0:
                u_h1, J_h1 = G.field(H.FIELD_MEAN_U), G.window_objective()
        u_all, J_all = G.field(H.FIELD_MEAN_U), G.window_objective()
        u_h2, J_h2 = 2.0 * u_all - u_h1, 2.0 * J_all - J_h1
        means[name] = u_all
        r.update({"J_mean": J_all, "J_halves": [J_h1, J_h2], "mean_u_halves_rel_l2": l2(u_h1, u_h2),
                  "J_halves_rel": abs(J_h1 - J_h2) / abs(J_all)})
        def vname(kind, ta):
            return kind if ta <= 0.0 else f"{kind}_tau{ta:g}"
        variants = [(vname("fta", ta), H.TURB_FROZEN, ta) for ta in tau_adjs]
        if diff:
            variants += [(vname("diff", ta), H.TURB_DIFFERENTIATED, ta) for ta in tau_adjs]
        r["adjoint"] = {}
        p = G.profile()
        bpu = G.bytes_per_update()
        r["sweeps"] = {k: {"us_per_launch": p[k]["mean_us"], "GLUPS": w.n / p[k]["mean_us"] / 1e3,
                           "GB_s": bpu[k] * w.n / p[k]["mean_us"] / 1e3} for k in p if p[k]["sampled"]}
        for vn, turb, tau_adj in variants:
            ta = time.perf_counter()
            G.profile_enable(97)
            it, st, rr = 0, H.W_NOT_CONVERGED, -1.0
            while it < adj_iters and st != H.OK:  # in blocks, each ending with a progress line
                k, rr, st = G.solve_adjoint(H.SOURCE_MEAN, tau_adj=tau_adj, turb=turb,
                                            max_iters=min(10000, adj_iters - it), tol=adj_tol, check_every=1000,
                                            restart=(it == 0))
                it += k
                log(f"les {name} adjoint {vn}: {it} it, residual {rr:.2e}")
            g = G.gradient()
            grads[(name, vn)] = g
            pa, ba = G.profile()["adjoint"]["mean_us"], G.bytes_per_update()["adjoint"]
            r["adjoint"][vn] = {"iters": it, "residual": rr, "tol": adj_tol, "converged": st == H.OK,
                                   "seconds": time.perf_counter() - ta,
                                   "max_abs_grad": float(np.abs(g).max()), "us_per_launch": pa,
                                   "GB_s": ba * w.n / pa / 1e3 if pa > 0 else None}
            log(f"les {name} adjoint {vn}: {it} it, residual {rr:.2e}")
        r["seconds"] = time.perf_counter() - t0
        res[name] = r
        G.close()

    ref = "fp64" if "fp64" in means else "fp32"
    cmp = {}
    def vname(kind, ta):
        return kind if ta <= 0.0 else f"{kind}_tau{ta:g}"
    f0 = vname("fta", tau_adjs[0])
    for name in means:
        if name == ref:
            continue
        c = {"mean_u_rel_l2_vs_" + ref: l2(means[name], means[ref]),
             "J_mean_rel_vs_" + ref: abs(res[name]["J_mean"] - res[ref]["J_mean"]) / abs(res[ref]["J_mean"])}
        if (ref, f0) in grads and (name, f0) in grads:
            c["grad_fta_rel_l2_vs_" + ref] = l2(grads[(name, f0)], grads[(ref, f0)])
            c["grad_fta_cosine_vs_" + ref] = cos(grads[(name, f0)], grads[(ref, f0)])
        cmp[name] = c
    c2 = {}
    for ta in tau_adjs:
        a, b = ("fp32", vname("fta", ta)), ("fp32", vname("diff", ta))
        if a in grads and b in grads:
            c2[f"tau_adj {ta:g}" if ta > 0 else "tau_adj tau0"] = {"cosine": cos(grads[a], grads[b]),
                                                                   "rel_l2": l2(grads[a], grads[b])}
    if c2:
        cmp["fp32_fta_vs_diff"] = c2
    out = {"report": "les", "workload": w.name, "collision": "hrr" if collision == H.COLL_HRR else "bgk",
           "spinup_steps": spinup, "window_steps": window, "adjoint_max_iters": adj_iters,
           "adjoint_tol": adj_tol, "tau_adj": list(tau_adjs), "forms": res, "comparison": cmp}
    print(json.dumps(out), flush=True)


def report_validation3d(steps: int, adj_iters: int, fd_scale: float, fd_points: int):
    """The steady 3D validation case (permeable cylinder, Re 40, D3Q19): FP64
    and FP32 primal over T = 32 s, steady adjoints for the drag (FFA) and
    dissipation objectives, FP32 against FP64 (objective, whole gradient field
    and the cylinder-surface samples at mid-span), and central differences of
    the converged FP64 objective on a scaled copy of the case."""
    w = I.porous3d_re40()
    box = w.extra["dissipation_box"]
    objs = {"ffa": (H.OBJ_FFA, w.lo, w.hi), "diss": (H.OBJ_DISS, box[0], box[1])}
    names = {H.FP64: "fp64", H.FP32: "fp32"}
    R = 0.5 * w.D
    x, y, z = np.arange(w.n) % w.nx, (np.arange(w.n) // w.nx) % w.ny, np.arange(w.n) // (w.nx * w.ny)
    r = np.hypot(x - w.xc, y - w.yc)
    ring = np.nonzero((np.abs(r - R) <= 0.5) & (z == w.nz // 2))[0]
    ring = ring[np.argsort(np.arctan2(y[ring] - w.yc, x[ring] - w.xc))]
    res, grads = {}, {}

    def make(wl, prec):
        G = H.Lattice(stencil=wl.stencil, precision=prec, nx=wl.nx, ny=wl.ny, nz=wl.nz, tau=wl.tau,
                      bc_x=H.BC_INLET_OUTLET, bc_y=wl.bc_y, bc_z=wl.bc_z, inlet_profile=wl.inlet_profile,
                      u_in=wl.u_max)
        G.build_cylinder(wl.xc, wl.yc, wl.D, d_solid=wl.d_solid)
        G.init_equilibrium()
        return G

    for prec in (H.FP64, H.FP32):
        name = names[prec]
        t0 = time.perf_counter()
        G = make(w, prec)
        G.set_objective(H.OBJ_FFA, w.lo, w.hi, u0=w.u0)
        for done in range(0, steps - 1000, 5000):
            G.run_primal(min(5000, steps - 1000 - done))
            log(f"validation3d {name}: step {min(done + 5000, steps - 1000)} ({time.perf_counter() - t0:.0f} s)")
        u1 = G.field(H.FIELD_U)
        G.run_primal(1000)
        u2 = G.field(H.FIELD_U)
        r_ = {"steady_residual_per_1000": float(np.abs(u2 - u1).max() / np.abs(u2).max()),
              "primal_seconds": time.perf_counter() - t0}
        for oname, (kind, lo, hi) in objs.items():
            G.set_objective(kind, lo, hi, u0=w.u0)
            J = G.objective(0)
            ta = time.perf_counter()
            it, rr, _ = G.solve_adjoint(H.SOURCE_STEADY, max_iters=adj_iters, tol=1e-10, check_every=1000)
            g = G.gradient()
            grads[(name, oname)] = g
            r_[oname] = {"J": J, "adjoint_iters": it, "adjoint_residual": rr,
                         "adjoint_seconds": time.perf_counter() - ta,
                         "surface_gradient": [float(v) for v in g[ring]]}
            log(f"validation3d {name} {oname}: J {J:.9e}, adjoint {it} it, residual {rr:.2e}")
        res[name] = r_
        G.close()
    cmp = {}
    for oname in objs:
        a, b = grads[("fp32", oname)], grads[("fp64", oname)]
        cmp[oname] = {"J_rel": abs(res["fp32"][oname]["J"] - res["fp64"][oname]["J"]) / abs(res["fp64"][oname]["J"]),
                      "grad_rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                      "grad_cosine": float(a @ b / np.linalg.norm(a) / np.linalg.norm(b)),
                      "surface_rel_max": float(np.abs(a[ring] - b[ring]).max() / np.abs(b[ring]).max())}

    # central differences of the converged FP64 drag on a scaled copy at
    # Re 20 (the 2D validation Reynolds number: a steady wake at this
    # resolution; the coarser Re 40 copy does not settle)
    from dataclasses import replace as _replace
    ws = _replace(I.scaled(w, fd_scale), Re=20.0)
    G = make(ws, H.FP64)
    G.set_objective(H.OBJ_FFA, ws.lo, ws.hi, u0=ws.u0)
    base_steps = G.run_primal(400000, steady_tol=1e-13, check_every=500)
    log(f"validation3d FD base: {base_steps} steps to steady (tau {ws.tau:.4f})")
    d0 = G.porosity()
    f0 = G.populations()
    J0 = G.objective(0)
    G.solve_adjoint(H.SOURCE_STEADY, max_iters=400000, tol=1e-13, check_every=500)
    g = G.gradient()
    xs, ys, zs = np.arange(ws.n) % ws.nx, (np.arange(ws.n) // ws.nx) % ws.ny, np.arange(ws.n) // (ws.nx * ws.ny)
    rs = np.hypot(xs - ws.xc, ys - ws.yc)
    cand = np.nonzero((np.abs(rs - 0.5 * ws.D) <= 0.5) & (zs == ws.nz // 2) & (d0 > 2e-4) & (d0 < 1 - 2e-4))[0]
    cand = cand[np.argsort(np.arctan2(ys[cand] - ws.yc, xs[cand] - ws.xc))]
    pick = cand[np.linspace(0, len(cand) - 1, fd_points).astype(int)]
    fd = []
    eps = 1e-4
    for c in pick:
        vals = []
        for sgn in (1.0, -1.0):
            d = d0.copy()
            d[c] += sgn * eps
            G.set_porosity(d)
            G.set_populations(f0)
            ns = G.run_primal(400000, steady_tol=1e-13, check_every=500)
            vals.append(G.objective(0))
            log(f"validation3d FD cell {c} ({sgn:+.0f}): {ns} steps")
        fdv = (vals[0] - vals[1]) / (2 * eps)
        fd.append({"cell": int(c), "angle_deg": float(np.degrees(np.arctan2(ys[c] - ws.yc, xs[c] - ws.xc))),
                   "adjoint": float(g[c]), "fd": fdv, "rel_err": abs(g[c] - fdv) / abs(fdv)})
        log(f"validation3d FD cell {c}: adjoint {g[c]:.9e}, FD {fdv:.9e}")
    G.close()
    out = {"report": "validation3d", "workload": w.name, "steps": steps, "d_solid": w.d_solid,
           "surface_samples": len(ring), "forms": res, "fp32_vs_fp64": cmp,
           "fd": {"workload": ws.name, "Re": ws.Re, "tau": ws.tau, "cells": ws.n, "base_steps": base_steps,
                  "J": J0, "eps": eps, "points": fd,
                  "max_rel_err": max(p_["rel_err"] for p_ in fd)}}
    print(json.dumps(out), flush=True)


def report_tangent(steps: int, late: int, record: int, blocks: int):
    """App. C on the Re = 100 vortex street (1100 x 410, FP64, dissipation
    box): the forward tangent dJ(t)/dd . v for a unit porosity change of one
    cylinder-rim cell, seeded at t = 0 and again once shedding is developed;
    its growth over time, its time average over the last ten periods against
    the mean-flow adjoint's derivative of the time average."""
    w = I.vortex_re100()
    noise = I.porosity_noise(w)

    def fresh():
        G = H.Lattice(stencil=w.stencil, precision=H.FP64, nx=w.nx, ny=w.ny, tau=w.tau, bc_x=H.BC_INLET_OUTLET,
                      bc_y=w.bc_y, inlet_profile=w.inlet_profile, u_in=w.u_max)
        G.build_cylinder(w.xc, w.yc, w.D, noise=noise, noise_mode=w.noise_mode)
        G.init_equilibrium()
        G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
        return G

    G = fresh()
    d = G.porosity()
    x, y = np.arange(w.n) % w.nx, np.arange(w.n) // w.nx
    rim = np.nonzero((d > 0.05) & (d < 0.95) & (x == int(w.xc)) & (y > w.yc))[0]
    cell = int(rim[0])
    v = np.zeros(w.n)
    v[cell] = 1.0

    def growth(rec):
        b = np.array_split(np.abs(rec[:, 1]), blocks)
        return [float(np.max(a)) for a in b]

    t0 = time.perf_counter()
    recA = G.run_tangent(v, steps, record)
    log(f"tangent seeded at 0: {steps} steps ({time.perf_counter() - t0:.1f} s)")
    G.close()
    G = fresh()
    G.set_probe(*w.extra["probe"], 0, late)
    G.run_primal(late)
    P = shedding_period(G.probe())
    recB = G.run_tangent(v, steps - late, record)
    log(f"tangent seeded at {late}: period {P}")
    # mean-flow adjoint over the last ten periods of the same trajectory
    G.close()
    G = fresh()
    W = int(round(10 * P)) if P else steps // 5
    G.run_primal(steps - W)
    G.run_primal(W, accumulate=True)
    it, rr, _ = G.solve_adjoint(H.SOURCE_MEAN, max_iters=60000, tol=1e-6, check_every=1000)
    gv = float(G.gradient()[cell])
    nwin = max(1, W // record)
    out = {"report": "tangent", "workload": w.name, "steps": steps, "record_every": record,
           "cell": cell, "cell_xy": [int(x[cell]), int(y[cell])], "d_cell": float(d[cell]),
           "shedding_period": P, "window_steps": W,
           "seeded_at_0": {"max_abs_dJdd_per_block": growth(recA),
                           "mean_over_window": float(recA[-nwin:, 1].mean()),
                           "J_mean_over_window": float(recA[-nwin:, 0].mean())},
           "seeded_at_%d" % late: {"max_abs_dJdd_per_block": growth(recB),
                                   "mean_over_window": float(recB[-nwin:, 1].mean())},
           "mean_flow_adjoint": {"dJmean_dd": gv, "iters": it, "residual": rr, "J_mean": G.window_objective()}}
    G.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--primal-steps", type=int, default=None)
    ap.add_argument("--periods", type=int, default=10)
    ap.add_argument("--workload", choices=["les_re3900", "vortex_re100"], default="les_re3900")
    ap.add_argument("--les-spinup-steps", type=int, default=LES_SPINUP)
    ap.add_argument("--les-window-steps", type=int, default=LES_WINDOW)
    ap.add_argument("--les-adjoint-iters", type=int, default=LES_ADJOINT)
    ap.add_argument("--les-tau-adj", type=float, default=LES_TAU_ADJ)
    ap.add_argument("--cpu-les-spinup", type=int, default=2)
    ap.add_argument("--cpu-les-window", type=int, default=2)
    ap.add_argument("--no-vortex", action="store_true", help="leave out the extra 2D vortex-street query")
    ap.add_argument("--vortex-tau-adj", type=float, default=0.6)
    ap.add_argument("--adjoint-max", type=int, default=120000)
    ap.add_argument("--adjoint-tol", type=float, default=1e-4)
    ap.add_argument("--profile-every", type=int, default=49)  # block length of the sweep timing
    ap.add_argument("--cpu-primal", type=int, default=40)
    ap.add_argument("--cpu-adjoint", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="leave out the short serving stream")
    ap.add_argument("--serving-queries", type=int, default=64,
                    help="queries of the serving stream the benchmark line reports beside the headline")
    ap.add_argument("--report", choices=["differentiation", "serving", "les", "validation3d", "tangent", "oracle",
                                         "sweeps"],
                    default=None,
                    help="print a secondary measurement report instead of the benchmark line")
    ap.add_argument("--sweep-case", choices=list(SWEEP_CASES), default="les_fp32")
    ap.add_argument("--sweep-launches", type=int, default=20)
    ap.add_argument("--fields", type=int, default=32)
    ap.add_argument("--fd-fields", type=int, default=2)
    ap.add_argument("--fd-directions", type=int, default=8)
    ap.add_argument("--les-spinup", type=int, default=30000)
    ap.add_argument("--les-window", type=int, default=30000)
    ap.add_argument("--les-adjoint", type=int, default=8000)
    ap.add_argument("--les-forms", default="fp32,fp16s,fp64")
    ap.add_argument("--les-collision", choices=["bgk", "hrr"], default="bgk")
    ap.add_argument("--les-tau-adjs", default="0,0.6", help="adjoint relaxation times (0: tau0)")
    ap.add_argument("--les-adjoint-tol", type=float, default=1e-8)
    ap.add_argument("--v3d-steps", type=int, default=42336)
    ap.add_argument("--v3d-adjoint", type=int, default=60000)
    ap.add_argument("--v3d-fd-scale", type=float, default=1.0 / 3.0)
    ap.add_argument("--v3d-fd-points", type=int, default=4)
    ap.add_argument("--tan-steps", type=int, default=200000)
    ap.add_argument("--tan-late", type=int, default=150000)
    ap.add_argument("--tan-record", type=int, default=50)
    ap.add_argument("--queries", type=int, default=200)
    ap.add_argument("--rate", type=float, default=2.0)
    ap.add_argument("--mem-cap-gib", type=float, default=1.0)
    ap.add_argument("--tick", type=int, default=256)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--oracle-threads", type=int, default=0, help="all-core thread count (0: the host's)")
    ap.add_argument("--oracle-worker", nargs=3, default=None, metavar=("CASE", "PRIMAL", "ADJ"),
                    help=argparse.SUPPRESS)
    ap.add_argument("--profile-summary", default=None, metavar="DIR",
                    help="write the profiles/ summaries from the rocprofv3 output under DIR and exit")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.oracle_worker:
        oracle_worker(args.oracle_worker[0], int(args.oracle_worker[1]), int(args.oracle_worker[2]))
        return
    if args.profile_summary:
        summarize_profiles(args.profile_summary)
        return
    if args.report == "oracle":
        threads = args.oracle_threads or int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
        report_oracle(threads)
        return
    if args.report == "sweeps":
        report_sweeps(args.sweep_case, args.sweep_launches)
        return
    if args.report == "differentiation":
        report_differentiation(args.fields, args.fd_fields, args.fd_directions)
        return
    if args.report == "les":
        forms = {"fp64": H.FP64, "fp32": H.FP32, "fp16s": H.FP16S}
        report_les(args.les_spinup, args.les_window, args.les_adjoint,
                   [forms[f] for f in args.les_forms.split(",")],
                   H.COLL_HRR if args.les_collision == "hrr" else H.COLL_BGK,
                   tuple(float(v) for v in args.les_tau_adjs.split(",")), args.les_adjoint_tol)
        return
    if args.report == "validation3d":
        report_validation3d(args.v3d_steps, args.v3d_adjoint, args.v3d_fd_scale, args.v3d_fd_points)
        return
    if args.report == "tangent":
        report_tangent(args.tan_steps, args.tan_late, args.tan_record, 20)
        return
    if args.report == "serving":
        report_serving(args.queries, args.rate, args.mem_cap_gib, args.tick, args.slots)
        return

    if args.copy_calibration_mib:
        import torch
        nbytes = args.copy_calibration_mib << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "vortex_re100":
        out = bench_vortex(args)
    else:
        out = bench_les(args)
    print(json.dumps(out), flush=True)


def timed_queries(q, steps: int, warmup: int, every: int, describe):
    """Runs `warmup` untimed and `steps` timed queries; returns lattice
    updates, wall seconds, per-query wall times and the sweep timing."""
    for i in range(warmup):
        t = time.perf_counter()
        q.run()
        log(f"warmup {i}: {time.perf_counter() - t:.2f} s; {describe(q)}")
    q.G.profile_enable(every)
    q.G.synchronize()
    t0 = time.perf_counter()
    lu = 0
    each = []  # wall time of every timed query (each ends on its host-side results)
    for i in range(steps):
        tq = time.perf_counter()
        lu += q.run()
        each.append(time.perf_counter() - tq)
        log(f"step {i}: {each[-1]:.3f} s; {describe(q)}")
    q.G.synchronize()
    dt = time.perf_counter() - t0
    prof = q.G.profile()
    q.G.profile_enable(0)
    return lu, dt, each, prof


def bench_les(args):
    """The LES gradient query (768 x 384 x 128 D3Q19, FP32) as the benchmark
    step; the roofline of its dominant sweep; the oracle sample; one 2D
    vortex-street query as an extra field."""
    w = I.les_re3900()
    q = LesQuery(w, H.FP32, args.les_spinup_steps, args.les_window_steps, args.les_adjoint_iters,
                 args.les_tau_adj, LES_CHECK)

    def describe(qq):
        return f"J {qq.J:.6e}, adjoint {qq.it} it, residual {qq.res:.3e}"

    lu, dt, each, prof = timed_queries(q, args.steps, args.warmup, args.profile_every, describe)
    bpu = q.G.bytes_per_update()
    n = w.n
    launches = {"primal": q.spinup, "primal_window": q.window, "adjoint": q.it}
    sweeps = {}
    for k in ("primal", "primal_window", "adjoint"):
        us = prof[k]["mean_us"]
        gbs = bpu[k] * n / (us * 1e-6) / 1e9 if us > 0 else 0.0
        sweeps[k] = {"us_per_launch": us, "launches_per_step": launches[k],
                     "ms_per_step": us * launches[k] / 1e3, "bytes_per_update": bpu[k],
                     "GB_s": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "launches_timed": prof[k]["sampled"]}
    dom = max(sweeps, key=lambda k: sweeps[k]["ms_per_step"])
    names = {"primal": "k_primal<19, float, *, 0, false> (AA step, Smagorinsky, no window)",
             "primal_window": "k_primal(_stream|_wstream)<19, float, *, 3, false> + k_window_region_copy<19, float> "
                              "(AA step with the FP64 window: rho, j, tau_eff sums updated once per group of four "
                              "steps; drag-plane terms by the region pass from the sweep's record of the plane)",
             "adjoint": "k_adjoint<19, float, *, false, false> (mean-flow adjoint sweep, frozen turbulence)"}
    d = sweeps[dom]
    khash = kernel_source_hash()
    log(f"sweeps: " + ", ".join(f"{k} {v['us_per_launch']:.1f} us ({v['GB_s']:.0f} GB/s)" for k, v in sweeps.items())
        + f"; dominant {dom}")
    out = {
        "metric": "primal+adjoint MLUPS (whole mean-flow gradient query)",
        "value": lu / dt / 1e6,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 1 % velocity noise on the uniform inflow)",
        "query_latency_s": {"p50": float(np.median(each)), "max": float(np.max(each)),
                            "each": [round(v, 4) for v in each],
                            "note": "one query at a time; latency under a Poisson query stream: --report serving"},
        "config": {"workload": w.name, "cells": n, "stencil": "D3Q19", "collision": "BGK-HLBM + Smagorinsky C_S 0.1",
                   "precision": "FP32 populations and arithmetic; FP64 window sums, objective, gradient, residual",
                   "step": f"one gradient query: porosity build, equilibrium initialisation, {q.spinup} spin-up "
                           f"steps, {q.window} window steps, mean-flow adjoint ({q.adj_iters} sweeps, frozen "
                           f"turbulence, tau_adj {q.tau_adj}), gradient",
                   "objective": "drag (far-field plane x = 432, y 48..335)",
                   "primal_steps": q.spinup + q.window, "window_steps": q.window,
                   "adjoint_iters": q.it, "adjoint_tau": q.tau_adj,
                   "adjoint_residual": q.res,
                   "adjoint_note": f"a fixed block of sweeps: the residual is the relative change of phi over "
                                   f"the last {LES_CHECK} sweeps, reported, not a convergence claim",
                   "J_mean": q.J},
        "roofline": {"bound": "hbm", "achieved": d["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": d["GB_s"] / HBM_PEAK_GBS, "traffic": traffic_for(khash, dom),
                     "kernel": names[dom], "kind": dom,
                     "bytes_per_update": d["bytes_per_update"], "updates_per_launch": n,
                     "us_per_launch": d["us_per_launch"],
                     "timing": "HIP events on the sweep stream around blocks of back-to-back launches",
                     "note": "2.9 GB of FP32 populations, 1.5 GB of FP64 window sums and 2.3 GB of FP32 pending "
                             "window values: HBM-resident"},
        "sweeps": sweeps,
    }
    if not args.no_vortex:
        out["vortex_re100_1100x410"] = vortex_extra(args)
    q.G.close()
    if not args.no_serving:
        out["serving"] = serving_extra(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_les(w, args.cpu_les_spinup, args.cpu_les_window)
    return out


def serving_extra(args):
    """Latency under load beside the headline: a short Poisson stream of the
    serving mix (continuous batching, packed small lattices), p50/p99."""
    from paper_2606_31707_amd import serving as S
    n, rate = args.serving_queries, args.rate
    srv = S.Server(S.GPUBackend(), mem_cap_bytes=int(args.mem_cap_gib * (1 << 30)), max_slots=args.slots,
                   tick=args.tick)
    st = srv.run(S.poisson_mix(n, rate)).summary()
    log(f"serving: {st['completed']}/{n} queries, p50 {st['p50_latency_s']:.2f} s, "
        f"p99 {st['p99_latency_s']:.2f} s, {st['aggregate_MLUPS']:.0f} MLUPS")
    return {"queries": n, "rate_qps": rate, "precision": "fp32", "mem_cap_GiB": args.mem_cap_gib,
            "mix": "70 % D2Q9 128x64..512x256, 25 % D2Q9 1024x512, 5 % D3Q19 192x96x64; Re 20..200; "
                   "drag or dissipation; Poisson arrivals (seed 2026)",
            **st,
            "note": "wall-clock latency from arrival to gradient; a longer stream: --report serving"}


def vortex_extra(args):
    """One 2D vortex-street query (FP64, the whole 200 000-step run, ten
    shedding periods of window) with the adjoint regularised as the paper does
    for its unsteady cases (tau_adj 0.6) and converged to a stated
    tolerance, and the same query in FP32 against it."""
    w = I.vortex_re100()
    T = w.primal_steps
    res = {}
    grads = {}
    for name, prec in (("fp64", H.FP64), ("fp32", H.FP32)):
        q = Query(w, prec, T, 120000, 1e-4, 1000, args.periods, tau_adj=0.6)
        t = time.perf_counter()
        lu = q.run()
        q.G.synchronize()
        dt = time.perf_counter() - t
        grads[name] = q.grad
        res[name] = {"MLUPS": lu / dt / 1e6, "seconds": dt, "window_steps": q.window, "J_mean": q.J,
                     "adjoint_iters": q.adj_iters, "adjoint_residual": q.adj_res, "adjoint_converged": q.converged}
        log(f"vortex {name}: {dt:.2f} s, window {q.window}, adjoint {q.adj_iters} it, residual {q.adj_res:.2e}")
        q.G.close()
    g64, g32 = grads["fp64"], grads["fp32"]
    return {"primal_steps": T, "adjoint": "mean-flow, tau_adj 0.6, tol 1e-4 (relative change over 1000 sweeps)",
            **res,
            "fp32_vs_fp64": {"grad_rel_l2": float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64)),
                             "grad_cosine": float(g32 @ g64 / np.linalg.norm(g32) / np.linalg.norm(g64)),
                             "J_mean_rel": abs(res["fp32"]["J_mean"] - res["fp64"]["J_mean"]) / abs(res["fp64"]["J_mean"])}}


def bench_vortex(args):
    """The 2D vortex-street gradient query (1100 x 410, FP64) as the step."""
    w = I.vortex_re100()
    T = args.primal_steps or w.primal_steps
    q = Query(w, H.FP64, T, args.adjoint_max, args.adjoint_tol, 1000, args.periods, tau_adj=args.vortex_tau_adj)

    def describe(qq):
        return (f"period {qq.period}, window {qq.window}, J {qq.J:.6e}, adjoint {qq.adj_iters} it, "
                f"residual {qq.adj_res:.2e}")

    lu, dt, each, prof = timed_queries(q, args.steps, args.warmup, args.profile_every, describe)
    bpu = q.G.bytes_per_update()
    n = w.n
    kus = prof["primal"]["mean_us"]
    achieved = bpu["primal"] * n / (kus * 1e-6) / 1e9 if kus > 0 else 0.0
    out = {
        "metric": "primal+adjoint MLUPS (whole mean-flow gradient query)",
        "value": lu / dt / 1e6,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded porosity noise on the cylinder rim)",
        "query_latency_s": {"p50": float(np.median(each)), "max": float(np.max(each)),
                            "each": [round(v, 4) for v in each]},
        "config": {"workload": w.name, "cells": n, "primal_steps": T, "window_steps": q.window,
                   "shedding_period_steps": q.period, "objective": "dissipation",
                   "adjoint": f"mean-flow, tau_adj {args.vortex_tau_adj or w.tau}, tol {args.adjoint_tol:g}",
                   "adjoint_iters": q.adj_iters, "adjoint_residual": q.adj_res,
                   "adjoint_converged": q.converged, "J_mean": q.J},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_primal<9, double> (AA step, no window)",
                     "bytes_per_update": bpu["primal"], "updates_per_launch": n, "us_per_launch": kus,
                     "timing": "HIP events on the sweep stream around blocks of back-to-back launches",
                     "note": "effective bandwidth: the 36 MB of FP64 populations stay resident in the 256 MB "
                             "Infinity Cache, so this is not an HBM fraction"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_primal, args.cpu_adjoint)
    return out


if __name__ == "__main__":
    main()
