"""The adjoint's stop rule (host logic of hlbm_solve_adjoint), compiled from
its header with the host compiler and driven with residual sequences: the
tolerance ends the solve, a non-finite value or a residual grown past 1e3
times its minimum is a divergence, anything else continues."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_2606_31707_amd", "csrc")

DRIVER = r'''
#include <cmath>
#include <cstdio>
#include "hlbm_stop.hpp"
// each line: tol, then pairs (dmax pmax) until a decision other than continue
int main() {
  double tol;
  while (std::scanf("%lf", &tol) == 1) {
    int n;
    std::scanf("%d", &n);
    double min_res = HUGE_VAL, res = -1.0;
    int k = 0, dec = 0;
    for (; k < n; ++k) {
      double a, b;
      std::scanf("%lf %lf", &a, &b);
      if (dec == 0) {
        dec = hlbm::adjoint_stop(a, b, tol, &min_res, &res);
        if (dec != 0) std::printf("%d %d %.3g\n", dec, k, res);
      }
    }
    if (dec == 0) std::printf("0 %d %.3g\n", n, res);
  }
  return 0;
}
'''


def run(cases):
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "stop.cpp")
        exe = os.path.join(td, "stop")
        open(src, "w").write(DRIVER)
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", HEADER_DIR, src, "-o", exe], check=True)
        text = ""
        for tol, seq in cases:
            text += f"{tol!r} {len(seq)} " + " ".join(f"{a!r} {b!r}" for a, b in seq) + "\n"
        out = subprocess.run([exe], input=text.replace("inf", "inf").replace("nan", "nan"),
                             capture_output=True, text=True, check=True).stdout.split("\n")
    return [tuple(float(v) for v in line.split()) for line in out if line.strip()]


def test_stop_rule_decisions():
    res = run([
        (1e-6, [(1.0, 1.0), (1e-3, 1.0), (1e-7, 1.0)]),              # converges at the third check
        (1e-6, [(1.0, 1.0), (1e-2, 1.0), (5e-3, 1.0)]),              # keeps going
        (1e-6, [(1.0, 1.0), (float("nan"), 1.0)]),                   # non-finite difference
        (1e-6, [(1.0, 1.0), (1e-3, float("inf"))]),                  # non-finite adjoint
        (1e-9, [(1e-2, 1.0), (1e-6, 1.0), (2e-3, 1.0)]),             # 2000x its minimum: diverged
        (1e-9, [(1e-2, 1.0), (1e-6, 1.0), (9e-4, 1.0)]),             # 900x: still continuing
        (1e-6, [(0.0, 0.0)]),                                        # phi still zero and unchanged
        (1e-6, [(2e-3, 0.0)]),                                       # phi zero: absolute change
    ])
    assert res[0][:2] == (1.0, 2.0)
    assert res[1][0] == 0.0 and abs(res[1][2] - 5e-3) < 1e-12
    assert res[2][:2] == (2.0, 1.0)
    assert res[3][:2] == (2.0, 1.0)
    assert res[4][:2] == (2.0, 2.0) and abs(res[4][2] - 2e-3) < 1e-12
    assert res[5][0] == 0.0
    assert res[6][:2] == (1.0, 0.0)
    assert res[7][0] == 0.0 and abs(res[7][2] - 2e-3) < 1e-12
