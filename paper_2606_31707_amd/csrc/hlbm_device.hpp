// hlbm_device.hpp -- device-side building blocks of the gfx950 HLBM sweeps.
//
// Populations are stored SoA (one plane per direction, planes padded to
// 256 B), shifted by the lattice weights: the stored value of direction i is
// s_i = f_i - w_i.  With sum w = 1 and sum w xi = 0 the moments become
// rho = 1 + sum s, j = sum xi s, which keeps FP32/FP16 storage accurate for
// the near-equilibrium states of these flows (f_i ~ w_i).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlbm {

enum { BC_PERIODIC = 0, BC_WALLS = 1, BC_INOUT = 2 };
enum { OBJ_FFA = 0, OBJ_DISS = 1, OBJ_MOMENTUM = 2, OBJ_MEA = 3 };
enum { NB_CELL = 0, NB_BOUNCE = 1, NB_OUTLET = 2, NB_DROP = 3 };

#ifndef HLBM_TILE_BX
#define HLBM_TILE_BX 128
#endif
// 1: the tuned workgroup orders (sweep_tile); 0: every order flipped
// (renumbered where the tuned build keeps the dispatch order and the other
// way round) -- the race-canary build.
#ifndef HLBM_XCD_REMAP
#define HLBM_XCD_REMAP 1
#endif
// BX x BY tiles: the cell grid of the set-up, gather and reduction kernels
// and the per-member tiles of the packed launches; the sweeps proper take
// runs of SWEEP_BLOCK consecutive cells (see sweep_cell).
constexpr int BX = HLBM_TILE_BX;   // wavefronts along x: BX consecutive cells per row
constexpr int BY = 256 / BX;       // rows per 256-thread workgroup
constexpr int SWEEP_BLOCK = 256;   // consecutive cells per workgroup of the sweeps
constexpr int NXCD = 8;            // MI355X: 8 accelerator complex dies, one L2 each

// ---- velocity sets (Sec. 2.1: D2Q9 and D3Q19) ------------------------------
template <int Q>
struct Lat;

template <>
struct Lat<9> {
  static constexpr int D = 2;
  static constexpr int NSYM = 3;  // xx, yy, xy
  static constexpr int cx[9] = {0, 1, 0, 1, -1, -1, 0, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36,
                                  1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36};
};

template <>
struct Lat<19> {
  static constexpr int D = 3;
  static constexpr int NSYM = 6;  // xx, yy, zz, xy, xz, yz
  static constexpr int cx[19] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
  static constexpr int cy[19] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
  static constexpr int cz[19] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
  static constexpr int opp[19] = {0, 10, 11, 12, 13, 14, 15, 16, 17, 18,
                                  1, 2, 3, 4, 5, 6, 7, 8, 9};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

// Number of per-region-cell objective coefficients: J, dJ/dd, then the
// quadratic form dJ/df_i = a0 + a1.xi_i + a2:xi_i xi_i (a2 symmetric).
template <int Q>
struct Coef {
  static constexpr int J = 0, DJDD = 1, A0 = 2, A1 = 3;
  static constexpr int A2 = A1 + Lat<Q>::D;
  static constexpr int N = A2 + Lat<Q>::NSYM;
  static constexpr int NB = 1 + Lat<Q>::D + Lat<Q>::NSYM;  // b0, b1, b2 of dtau/df
};

// Third-order Hermite components H_aab = xi_b (xi_a^2 - 1/3), a != b, that
// D2Q9 and D3Q19 support (the third order of the HRRLBM collision).
template <int Q>
struct H3Types;
template <>
struct H3Types<9> {
  static constexpr int N = 2;
  static constexpr int a[2] = {0, 1}, b[2] = {1, 0};
};
template <>
struct H3Types<19> {
  static constexpr int N = 6;
  static constexpr int a[6] = {0, 0, 1, 1, 2, 2}, b[6] = {1, 2, 0, 2, 0, 1};
};

template <int Q>
__device__ __forceinline__ constexpr int lat_c(int k, int a) {
  return a == 0 ? Lat<Q>::cx[k] : (a == 1 ? Lat<Q>::cy[k] : Lat<Q>::cz[k]);
}

// H_aab of direction k for third-order type t.
template <int Q>
__device__ __forceinline__ constexpr double h3(int k, int t) {
  const int ca = lat_c<Q>(k, H3Types<Q>::a[t]), cb = lat_c<Q>(k, H3Types<Q>::b[t]);
  return cb * (ca * ca - 1.0 / 3.0);
}

// ---- storage / compute types ----------------------------------------------
template <typename S>
struct Prec;
template <>
struct Prec<double> {
  using T = double;   // arithmetic
  using Dd = double;  // porosity storage
};
template <>
struct Prec<float> {
  using T = float;
  using Dd = float;
};
template <>
struct Prec<_Float16> {
  using T = float;
  using Dd = float;
};

// ---- geometry and boundary classification ---------------------------------
struct Geo {
  int nx, ny, nz;
  int tiles_x, tiles_y;  // BX x BY tiles per row / per plane of the sweep grid
  int bcx, bcy, bcz;
  int64_t plane;   // population plane stride (elements)
  int64_t gplane;  // outlet (y, z) plane stride (elements)
  int inlet_profile;
  double u_in;
  // Whether the odd step's 32-bit lane offsets hold every slot offset of a
  // tile, (3 nx + 256) * 8 < 2^32 bytes (the fast-lane slot addressing).
  int slot32;
};

__device__ __forceinline__ int64_t cell_of(const Geo& g, int x, int y, int z) {
  return (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
}

// Classifies the lattice position (x, y, z) reached from a cell: wraps the
// periodic axes in place; a wall crossing (halfway bounce-back) takes
// precedence over the inlet/outlet ends of the x axis.
__device__ __forceinline__ int classify(const Geo& g, int& x, int& y, int& z) {
  int bounce = 0;
  if (y < 0 || y >= g.ny) {
    if (g.bcy == BC_PERIODIC)
      y = (y < 0) ? y + g.ny : y - g.ny;
    else
      bounce = 1;
  }
  if (z < 0 || z >= g.nz) {
    if (g.bcz == BC_PERIODIC)
      z = (z < 0) ? z + g.nz : z - g.nz;
    else
      bounce = 1;
  }
  if (x < 0 || x >= g.nx) {
    if (g.bcx == BC_PERIODIC)
      x = (x < 0) ? x + g.nx : x - g.nx;
    else if (g.bcx == BC_WALLS)
      bounce = 1;
    else if (!bounce)
      return (x >= g.nx) ? NB_OUTLET : NB_DROP;
  }
  return bounce ? NB_BOUNCE : NB_CELL;
}

// Inlet velocity u_in(y): uniform, or the parabola vanishing at the halfway
// walls y = -1/2 and y = ny - 1/2.
template <typename T>
__device__ __forceinline__ T inlet_velocity(const Geo& g, int y) {
  if (g.inlet_profile == 2) {
    const double H = (double)g.ny;
    return (T)(4.0 * g.u_in * (y + 0.5) * (H - 0.5 - y) / (H * H));
  }
  return (T)g.u_in;
}

// ---- block reductions (deterministic: fixed lane / wave order) -------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over a 256-thread block; result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* lds) {
  const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  v = wave_sum(v);
  if ((t & 63) == 0) lds[t >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (t == 0) r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_max256(double v, double* lds) {
  const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  v = wave_max(v);
  if ((t & 63) == 0) lds[t >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (t == 0) r = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
  __syncthreads();
  return r;
}

// The sweeps run on a 1D grid of BX x BY tiles.  Workgroups are dispatched
// round-robin over the XCDs, each with its own L2; renumbering them so that
// XCD k takes one contiguous range of tiles (row-major) keeps x-neighbouring
// tiles, whose odd-step pulls and pushes share the cache lines at the tile
// edges, in the same L2.  When the whole grid is resident at once (at most
// 2048 workgroups: 256 CUs x 8 workgroups of 256 threads), the dispatch order
// decides which tiles finish last; there the last XCD walks its range from
// the end, so that the tiles of the last rows (a wall row takes the longer
// boundary path) start first rather than last (2 % per step on the
// 1100 x 410 channel; on larger grids the reversed walk measured 2-4 %
// slower).  b -> tile is a bijection of [0, nt): the last XCD's range has q
// tiles (r < NXCD) and k < q there.  remap = false keeps the dispatch order
// (see runs_remap); the canary build flips the choice.
__device__ __forceinline__ int sweep_tile(int b, int nt, bool remap = true) {
  if (HLBM_XCD_REMAP ? !remap : remap) return b;
  const int q = nt / NXCD, r = nt % NXCD;
  const int xcd = b % NXCD, k = b / NXCD;
  const int start = xcd * q + (xcd < r ? xcd : r);
  return (xcd == NXCD - 1 && nt <= 2048) ? start + (q - 1 - k) : start + k;
}

__device__ __forceinline__ int linear_block() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

}  // namespace hlbm
