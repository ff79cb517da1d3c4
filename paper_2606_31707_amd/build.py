"""Builds libhlbm.so (gfx950 HIP kernels + C ABI) in-tree with hipcc, and
libhlbm_canary.so, the same sources with 64 x 4 tiles and every sweep's
workgroup order flipped (XCD-renumbered where the default keeps the dispatch
order and the other way round): the race canary, under which every per-cell
result must be bitwise the same."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libhlbm.so")
CANARY_PATH = os.path.join(HERE, "libhlbm_canary.so")
SOURCES = ["hlbm_launch.hip", "hlbm_api.hip"]
ARCH = os.environ.get("HLBM_OFFLOAD_ARCH", "gfx950")
CANARY_DEFINES = ["-DHLBM_TILE_BX=64", "-DHLBM_XCD_REMAP=0"]


def _command(out: str, defines) -> list:
    return [
        "hipcc", "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-shared",
        "-Wall", "-Wno-unused-function",
        # multiply-adds fused per source expression only, so the same inlined
        # per-cell code rounds identically in every kernel that contains it
        "-ffp-contract=on",
        # no packed FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        *defines, "-o", out + ".tmp",
    ] + [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, canary: bool = True) -> str:
    jobs = [(LIB_PATH, [])] + ([(CANARY_PATH, CANARY_DEFINES)] if canary else [])
    procs = []
    for out, defines in jobs:
        cmd = _command(out, defines)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = False
    for out, p in procs:
        _, stderr = p.communicate()
        # the host pass warns about the device-only target feature; keep other diagnostics
        err = "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if p.returncode != 0:
            sys.stderr.write(err + "\n")
            failed = True
            continue
        if err and verbose:
            sys.stderr.write(err + "\n")
        os.replace(out + ".tmp", out)
    if failed:
        raise RuntimeError("hipcc failed building the HLBM library")
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
