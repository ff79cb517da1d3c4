"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the test oracle driven through every entry point on tiny lattices
(tests/sanitize_driver.c), the library's host-only argument arithmetic
(tests/sanitize_host_driver.cpp) and the adjoint's stop rule, each compiled with
-fsanitize=address,undefined; any report fails the test."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "driver")
        rc, out = _run(["gcc", "-std=c11", "-ffp-contract=off", "-fopenmp", *SAN, "-I", os.path.join(ROOT, "oracle"),
                        os.path.join(ROOT, "tests", "sanitize_driver.c"), os.path.join(ROOT, "oracle", "hlbm_oracle.c"),
                        "-o", exe, "-lm"])
        assert rc == 0, out
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
        rc, out = _run([exe], env=env)
        assert rc == 0 and "ok" in out, out
        assert "runtime error" not in out and "AddressSanitizer" not in out, out


def test_stop_rule_under_sanitizers():
    drv = r'''
#include <cmath>
#include <cstdio>
#include "hlbm_stop.hpp"
int main() {
  double m = HUGE_VAL, r = -1.0;
  const double seq[][2] = {{1.0, 1.0}, {1e-3, 1.0}, {2e-3, 0.0}, {5.0, 1.0}, {NAN, 1.0}};
  int d[5];
  for (int i = 0; i < 5; ++i) d[i] = hlbm::adjoint_stop(seq[i][0], seq[i][1], 1e-9, &m, &r);
  std::printf("%d %d %d %d %d\n", d[0], d[1], d[2], d[3], d[4]);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as td:
        src, exe = os.path.join(td, "s.cpp"), os.path.join(td, "s")
        open(src, "w").write(drv)
        rc, out = _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2606_31707_amd", "csrc"), src,
                        "-o", exe])
        assert rc == 0, out
        rc, out = _run([exe])
        assert rc == 0 and out.split()[:5] == ["0", "0", "0", "2", "2"], out


def test_library_host_arithmetic_under_sanitizers():
    """Descriptor checks, plane strides and footprints (csrc/hlbm_host.hpp,
    the host-only part of the C ABI's argument handling)."""
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "host")
        rc, out = _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2606_31707_amd", "csrc"),
                        os.path.join(ROOT, "tests", "sanitize_host_driver.cpp"), "-o", exe])
        assert rc == 0, out
        rc, out = _run([exe])
        assert rc == 0 and "ok 0" in out, out
        assert "runtime error" not in out and "AddressSanitizer" not in out, out
