"""Builds the oracle's shared library with gcc (plain C, FP64, no FMA contraction).

Test infrastructure: compiled by ``__graft_entry__.build()`` and on first use
by the oracle binding.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hlbm_oracle.c")
LIB_PATH = os.path.join(HERE, "libhlbm_oracle.so")


def build(verbose: bool = False, out: str = LIB_PATH, sanitize: bool = False) -> str:
    """sanitize: AddressSanitizer and UndefinedBehaviorSanitizer build (host
    code only; any undefined behaviour aborts)."""
    san = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    cmd = [
        "gcc", *san, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-Wextra", "-o", out + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
