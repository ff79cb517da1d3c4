// Drives the library's host-only arithmetic (descriptor checks, plane
// strides, footprint of a query; csrc/hlbm_host.hpp) over valid and invalid
// descriptors, for the AddressSanitizer / UndefinedBehaviorSanitizer build of
// tests/test_sanitizers.py.  Prints "ok 0" when every answer is as expected.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "hlbm_host.hpp"

static hlbm_desc base() {
  hlbm_desc d;
  std::memset(&d, 0, sizeof d);
  d.struct_size = sizeof d;
  d.stencil = HLBM_D2Q9;
  d.precision = HLBM_FP64;
  d.nx = 220;
  d.ny = 41;
  d.nz = 1;
  d.tau = 0.53;
  d.bc_x = HLBM_BC_INLET_OUTLET;
  d.bc_y = HLBM_BC_WALLS;
  d.inlet_profile = HLBM_INLET_PARABOLIC;
  d.u_in = 0.03;
  return d;
}

int main() {
  using namespace hlbm;
  int fails = 0;
  uint64_t b = 0;
  for (int st = 0; st < 2; ++st)
    for (int pr = 0; pr < 3; ++pr)
      for (int w = 0; w < 2; ++w)
        for (int kind = 0; kind < 4; ++kind) {
          hlbm_desc e = base();
          e.stencil = st;
          e.precision = pr;
          if (st == HLBM_D3Q19) {  // the largest accepted lattice
            e.nx = 2048;
            e.ny = 1024;
            e.nz = 1024;
            e.bc_y = HLBM_BC_PERIODIC;
            e.smagorinsky_cs = 0.1;
            e.track_mean_populations = 1;
          }
          const int64_t n = (int64_t)e.nx * e.ny * e.nz;
          if (desc_problem(&e) != nullptr) ++fails;
          if (footprint_of(&e, w, w, n / 3, kind, 128, 2, &b) != nullptr || b == 0) ++fails;
          if (plane_stride(n, ssize_of(pr)) < n) ++fails;
        }
  hlbm_desc bad[11];
  for (auto& d : bad) d = base();
  bad[0].struct_size = 3;
  bad[1].stencil = 7;
  bad[2].nx = 1 << 16, bad[2].ny = 1 << 16;
  bad[3].tau = 0.5;
  bad[4].smagorinsky_cs = -1.0;
  bad[5].bc_y = HLBM_BC_INLET_OUTLET;
  bad[6].u_in = NAN;
  bad[7].nz = 2;
  bad[8].collision = 9;
  bad[9].cache_policy = -4;
  bad[10].force[2] = INFINITY;
  for (auto& d : bad)
    if (desc_problem(&d) == nullptr) ++fails;
  if (desc_problem(nullptr) == nullptr) ++fails;
  hlbm_desc d = base();
  if (footprint_of(&d, 1, 1, -1, 0, 128, 2, &b) == nullptr) ++fails;
  if (footprint_of(&d, 1, 1, 220 * 41 + 1, 0, 128, 2, &b) == nullptr) ++fails;
  if (footprint_of(&d, 1, 1, 10, 8, 128, 2, &b) == nullptr) ++fails;
  if (plane_stride(100, 0) != -1 || plane_stride(100, 512) != -1) ++fails;
  std::printf("%s %d\n", fails ? "FAILED" : "ok", fails);
  return fails != 0;
}
