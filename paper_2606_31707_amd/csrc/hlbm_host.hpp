// hlbm_host.hpp -- host-only arithmetic of the C ABI: descriptor checks,
// plane strides and the device-memory footprint of a query.  Plain C++ (no
// HIP types), so that it can be checked on its own.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "../../include/hlbm.h"

namespace hlbm {

// Window steps per FP64 read-modify-write of the dense window sums on FP32
// and FP16 lattices (the first PEND_GROUP - 1 steps of a group leave their
// values in FP32 pending slots for the last one).
constexpr int PEND_GROUP = 4;

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Window steps accumulate the objective terms of a region of at most 1/8 of
// the lattice in a separate region pass; for the moment-form objectives
// (not J_MEA, which reads neighbours) the sweep hands that pass each region
// cell's pre-collision state through a compact copy.
inline bool region_copy_used(int64_t region_cells, int64_t n, int objective) {
  return objective != HLBM_OBJ_MEA && region_cells > 0 && region_cells * 8 <= n;
}
// Values per region cell in that copy: the q populations and the porosity,
// padded to whole 128-byte lines (each cell's record fills its own lines, so
// no line is written by two wavefronts of the sweep).
constexpr int region_copy_stride(int q, int value_bytes) {
  return (q + 1 + 128 / value_bytes - 1) / (128 / value_bytes) * (128 / value_bytes);
}

// Plane stride in elements: a multiple of 256 B, and an odd number of 256 B
// blocks so that the q planes do not start on the same memory channel (power-
// of-two strides measured up to 8% slower on the D3Q19 sweeps).
inline int64_t plane_stride(int64_t n, size_t ssize) {
  if (ssize == 0 || ssize > 256) return -1;
  const int64_t unit = 256 / (int64_t)ssize;
  int64_t m = (n + unit - 1) / unit;
  if (m % 2 == 0) m += 1;
  return m * unit < round_up(n, 128) ? round_up(n, 128) : m * unit;
}

inline int q_of(int stencil) { return stencil == HLBM_D2Q9 ? 9 : 19; }
inline int dim_of(int stencil) { return stencil == HLBM_D2Q9 ? 2 : 3; }
inline size_t ssize_of(int prec) { return prec == HLBM_FP64 ? 8 : (prec == HLBM_FP32 ? 4 : 2); }
inline size_t dsize_of(int prec) { return prec == HLBM_FP64 ? 8 : 4; }
inline size_t asize_of(int prec) { return prec == HLBM_FP64 ? 8 : 4; }
inline int nsym_of(int stencil) { return stencil == HLBM_D2Q9 ? 3 : 6; }
inline int ncoef_of(int stencil) { return 3 + dim_of(stencil) + nsym_of(stencil); }
inline int nb_of(int stencil) { return 1 + dim_of(stencil) + nsym_of(stencil); }

// What is wrong with a descriptor, or nullptr if it is valid.
inline const char* desc_problem(const hlbm_desc* d) {
  if (!d) return "null descriptor";
  if (d->struct_size != sizeof(hlbm_desc)) return "hlbm_desc.struct_size does not match this library";
  if (d->stencil != HLBM_D2Q9 && d->stencil != HLBM_D3Q19) return "bad stencil";
  if (d->precision < HLBM_FP64 || d->precision > HLBM_FP16S) return "bad precision";
  if (d->nx < 2 || d->ny < 1 || d->nz < 1) return "bad lattice size";
  if (d->stencil == HLBM_D2Q9 && d->nz != 1) return "D2Q9 needs nz = 1";
  if ((int64_t)d->nx * d->ny * d->nz > (int64_t)1 << 31) return "lattice too large";
  if (!(d->tau > 0.5) || !std::isfinite(d->tau)) return "tau must exceed 1/2";
  if (!(d->smagorinsky_cs >= 0.0) || !std::isfinite(d->smagorinsky_cs)) return "Smagorinsky constant must be >= 0";
  if (d->bc_x < 0 || d->bc_x > 2 || d->bc_y < 0 || d->bc_y > 1 || d->bc_z < 0 || d->bc_z > 1)
    return "bad boundary kinds (only x may be INLET_OUTLET)";
  if (d->bc_x == HLBM_BC_INLET_OUTLET) {
    if (d->inlet_profile != HLBM_INLET_UNIFORM && d->inlet_profile != HLBM_INLET_PARABOLIC)
      return "bad inlet profile";
    if (d->nx < 3) return "inlet/outlet channel needs nx >= 3";
  }
  if (!std::isfinite(d->u_in)) return "u_in not finite";
  if (d->collision != HLBM_COLL_BGK && d->collision != HLBM_COLL_HRR) return "bad collision";
  if (d->cache_policy < HLBM_CACHE_AUTO || d->cache_policy > HLBM_CACHE_STREAMING) return "bad cache policy";
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->force[a])) return "force not finite";
  return nullptr;
}

// Device bytes of one query (see hlbm_footprint_bytes) for a descriptor that
// desc_problem accepted; bx, by: the tile shape of the set-up and reduction
// kernels (their block partials).  Returns what is wrong with the region
// arguments, or nullptr.
inline const char* footprint_of(const hlbm_desc* desc, int with_window, int with_adjoint, int64_t region_cells,
                                int32_t objective, int bx, int by, uint64_t* bytes) {
  const int64_t n = (int64_t)desc->nx * desc->ny * desc->nz;
  if (region_cells < 0 || region_cells > n) return "region_cells outside [0, n]";
  if (objective < HLBM_OBJ_FFA || objective > HLBM_OBJ_MEA) return "bad objective kind";
  const int q = q_of(desc->stencil), dim = dim_of(desc->stencil), ncoef = ncoef_of(desc->stencil);
  const uint64_t P = (uint64_t)plane_stride(n, ssize_of(desc->precision));
  const uint64_t G = (uint64_t)round_up((int64_t)desc->ny * desc->nz, 128);
  const uint64_t ss = ssize_of(desc->precision), ds = dsize_of(desc->precision), as = asize_of(desc->precision);
  const uint64_t blocks = (uint64_t)((desc->nx + bx - 1) / bx) * (uint64_t)((desc->ny + by - 1) / by) *
                          (uint64_t)desc->nz;
  // populations, porosity, outlet values, reduction partials, steady-check snapshot
  uint64_t b = P * (q * ss + ds) + G * q * ss + 8 * (2 * blocks + 8) + 8 * P * dim;
  if (region_cells > 0) {  // objective terms and adjoint source over the region
    const uint64_t rp = (uint64_t)round_up(region_cells, 128);
    b += 2 * 8 * rp * ncoef;
    if (objective == HLBM_OBJ_MEA) b += rp + 8 * q * rp;  // surface flags and source
    if (region_copy_used(region_cells, n, objective))  // region cells' state
      b += rp * (uint64_t)region_copy_stride(q, (int)as) * as;
  }
  if (with_window) {
    b += P * 8 * (1 + dim);
    if (desc->track_mean_populations) b += P * 8 * q;
    if (desc->smagorinsky_cs > 0) b += P * 8;
    // FP32 pending slots of the grouped accumulation
    if (desc->precision != HLBM_FP64)
      b += (uint64_t)(PEND_GROUP - 1) * P * 4 * (2 + dim + (desc->track_mean_populations ? q : 0));
  }
  if (with_adjoint) {
    b += P * as * q;                                    // phi
    b += P * as * (dim + 2 + q + nb_of(desc->stencil)); // frozen coefficients
    b += P * 8 * (dim + 2);                             // gradient data
    b += G * (8 * (1 + dim) + 2 * as * q);              // outlet data, outlet adjoint values
    b += P * as * q;                                    // residual snapshot
  }
  *bytes = b;
  return nullptr;
}

}  // namespace hlbm
