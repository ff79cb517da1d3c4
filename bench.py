#!/usr/bin/env python3
"""Benchmark: whole-path throughput of the HLBM mean-flow adjoint on one GPU.

One step = one gradient query of the workload: porosity field build (a1),
equilibrium initialisation (a2), the primal sweep with its FP64 window over
the last shedding periods (a3-a6), adjoint preparation (a7), the adjoint
sweep to a steady state (a8) and the gradient assembly (a9).  `value` is
primal plus adjoint lattice updates per second of the whole query (MLUPS),
inputs resident on the device.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_lattice(w: I.Workload, precision: int) -> H.Lattice:
    return H.Lattice(stencil=w.stencil, precision=precision, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs,
                     bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile,
                     u_in=w.u_max, track_mean_populations=False)


class Query:
    """One gradient query on a resident lattice."""

    def __init__(self, w: I.Workload, precision: int, primal_steps: int, window_steps: int,
                 adj_max: int, adj_tol: float, adj_check: int):
        self.w = w
        self.G = make_lattice(w, precision)
        self.noise = I.porosity_noise(w)
        self.primal_steps = primal_steps
        self.window_steps = window_steps
        self.adj_max, self.adj_tol, self.adj_check = adj_max, adj_tol, adj_check
        self.G.set_objective(w.objective, w.lo, w.hi, u0=w.u0)
        self.grad = None

    def run(self):
        w, G = self.w, self.G
        G.build_cylinder(w.xc, w.yc, w.D, noise=self.noise, noise_mode=w.noise_mode, box_half=w.box_half)
        G.init_equilibrium(1.0, I.initial_velocity(w))
        G.run_primal(self.primal_steps - self.window_steps)
        G.run_primal(self.window_steps, accumulate=True)
        it, res, _ = G.solve_adjoint(H.SOURCE_MEAN, max_iters=self.adj_max, tol=self.adj_tol,
                                     check_every=self.adj_check)
        self.grad = G.gradient()
        self.adj_iters, self.adj_res = it, res
        return self.primal_steps * w.n + it * w.n


def roofline(G: H.Lattice, n: int, launches: int, accumulate: bool = False):
    G.profile_enable(True)
    G.run_primal(launches, accumulate=accumulate)
    prof = G.profile()
    G.profile_enable(False)
    avg_ms = prof["primal_ms"] / prof["primal_launches"]
    bpu = G.bytes_per_update()["primal_window" if accumulate else "primal"]
    achieved = bpu * n / (avg_ms * 1e-3) / 1e9
    return avg_ms, bpu, achieved


def cpu_baseline(w: I.Workload, primal_steps: int, adj_iters: int):
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
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": lu / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{w.name}: {primal_steps} primal steps with window sampling + adjoint preparation + "
                      f"{adj_iters} adjoint iterations + gradient, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32", "fp16s"], default="fp64")
    ap.add_argument("--primal-steps", type=int, default=None)
    ap.add_argument("--window-steps", type=int, default=None)
    ap.add_argument("--adjoint-max", type=int, default=100000)
    ap.add_argument("--adjoint-tol", type=float, default=1e-6)
    ap.add_argument("--roofline-launches", type=int, default=2000)
    ap.add_argument("--cpu-primal", type=int, default=60)
    ap.add_argument("--cpu-adjoint", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    prec = {"fp64": H.FP64, "fp32": H.FP32, "fp16s": H.FP16S}[args.precision]
    w = I.vortex_re100()
    primal = args.primal_steps or w.primal_steps
    window = args.window_steps or primal // 5
    q = Query(w, prec, primal, window, args.adjoint_max, args.adjoint_tol, 1000)

    for i in range(args.warmup):
        t = time.perf_counter()
        q.run()
        log(f"warmup {i}: {time.perf_counter() - t:.2f} s, adjoint iters {q.adj_iters}, residual {q.adj_res:.2e}")
    q.G.synchronize()
    t0 = time.perf_counter()
    lu = 0
    for i in range(args.steps):
        lu += q.run()
        log(f"step {i}: adjoint iters {q.adj_iters}, residual {q.adj_res:.2e}")
    q.G.synchronize()
    dt = time.perf_counter() - t0

    n = w.n
    avg_ms, bpu, achieved = roofline(q.G, n, args.roofline_launches)
    log(f"primal sweep: {avg_ms * 1e3:.2f} us/launch, {bpu:.0f} B/LU, {achieved:.0f} GB/s, "
        f"{n / (avg_ms * 1e-3) / 1e9:.2f} GLUPS")
    out = {
        "metric": "primal+adjoint MLUPS (whole gradient query)",
        "value": lu / dt / 1e6,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16s": "f16-storage/f32"}[args.precision],
        "data": "synthetic (seeded porosity noise on the cylinder rim)",
        "config": {"workload": w.name, "cells": n, "primal_steps": primal, "window_steps": window,
                   "objective": "dissipation", "adjoint": "mean-flow, tol %.0e" % args.adjoint_tol,
                   "adjoint_iters_last": q.adj_iters},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_primal (no window)", "bytes_per_update": bpu,
                     "us_per_launch": avg_ms * 1e3},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_primal, args.cpu_adjoint)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
