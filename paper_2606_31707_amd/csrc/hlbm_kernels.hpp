// hlbm_kernels.hpp -- gfx950 kernels of the HLBM mean-flow adjoint path.
//
// Propagation is the in-place AA pattern: the even step reads a cell's own
// slots and writes its post-collision values back swapped (slot opp(i)); the
// odd step pulls the neighbours' swapped values, collides, and pushes to the
// neighbours' slots.  Each cell reads and writes the same slot set in both
// steps, so one population array suffices and every slot is read and written
// exactly once per step.  All boundary conditions are resolved inside the
// odd step's pull/push; the pressure outlet additionally uses a small ghost
// buffer (even step -> odd step) for the values of its virtual column.
//
// The adjoint sweep (Eqs. adjoint_steady/adjoint_unsteady) runs on relabelled
// adjoint populations phihat_k = phi_opp(k), which turns "collide at x, then
// move against xi_i" into the same forward AA propagation; halfway bounce-back
// is self-adjoint, the pinned inlet contributes zeros, and the outlet's
// virtual column becomes a double-buffered array of adjoint values.
//
// All reductions are deterministic: wavefront shuffles, four waves through
// LDS, per-block partials, one final single-block pass in a fixed order.
#pragma once

#include <cmath>

#include "hlbm_internal.hpp"

namespace hlbm {

// =========================================================================
// small helpers
// =========================================================================

// Accesses of the population planes.  Every slot is read and written once
// per step.  NT: nontemporal (streaming) hints on both the load and the
// store, taken by the sweeps when the lattice exceeds the 256 MB
// Infinity Cache: both D2Q9 primal steps (5-20 % faster there), the D3Q19
// primal even step (1-2 %; its odd step, whose z neighbours reuse lines one
// xy layer later, is 7 % slower with them) and the adjoint's even step
// (D2Q9 4-5 %, D3Q19 1 %; both adjoint steps together measured up to 9 %
// slower).  A lattice that stays in that cache between steps is 5-20 %
// slower with them.  Either way the values are the same.
template <bool NT = false, typename P>
__device__ __forceinline__ auto ld_stream(P p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT = false, typename P, typename S>
__device__ __forceinline__ void st_stream(P p, S v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Conversion of an arithmetic value to the storage type S.  FP16 storage of
// an FP32 result always rounds that FP32 value: the opaque copy keeps the
// compiler from fusing the last multiply-add into the conversion (a
// mixed-precision FMA rounds the exact result to FP16 once), which it would
// do or not depending on the shape of the surrounding code, changing rare
// values by one FP16 unit from one build of the same arithmetic to the next.
// FP64 values (initialisation, user input) are converted directly.
template <typename S, typename T>
__device__ __forceinline__ S to_store(T v) {
  if constexpr (sizeof(S) == 2 && sizeof(T) == 4) {
    float t = (float)v;
    asm("" : "+v"(t));
    return (S)t;
  } else {
    return (S)v;
  }
}

// Values that are the same in every lane of a wavefront (tile indices, tile
// base cells), moved to scalar registers: the integer divisions of the tile
// decode run on the vector unit, and without this their results, and all
// address arithmetic built on them, would stay there.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t wave_uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Plane addressing of the sweeps.  A workgroup's tile starts at cell c0 (the
// same for all its lanes) and a lane sits lo = tx + nx ty cells further on.
// The per-plane base address (array + plane offset + c0, plus a fixed
// neighbour offset in the odd step) is formed once in scalar registers, so
// each access adds only the lane's 32-bit offset: no 64-bit vector address
// arithmetic per population.  The base is a global-memory (address space 1)
// pointer, so the accesses are global loads/stores with a scalar base.
template <typename S>
struct Glob {
  typedef __attribute__((address_space(1))) S type;
};
template <typename S>
__device__ __forceinline__ typename Glob<S>::type* plane_base(S* A, int64_t elem) {
  const uint64_t a = (uint64_t)A + (uint64_t)(elem * (int64_t)sizeof(S));
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return (typename Glob<S>::type*)(((uint64_t)hi << 32) | lo);
}
// Element at plane offset elem (uniform) for lane offset lo (cells).  The
// byte offset is formed in 32 bits, matching the scalar-base address form.
template <typename S>
__device__ __forceinline__ typename Glob<S>::type& at(S* A, int64_t elem, uint32_t lo) {
  typedef typename Glob<char>::type gchar;
  uint32_t off = lo * (uint32_t)sizeof(S);
  asm volatile("" : "+v"(off));  // a 32-bit offset local to this access
  return *(typename Glob<S>::type*)((gchar*)plane_base(A, elem) + off);
}

// A lane's 32-bit offset from its tile base, kept opaque to the optimizer so
// that it stays a 32-bit register offset (the address form with a scalar
// base) instead of being folded into 64-bit vector address arithmetic.
__device__ __forceinline__ uint32_t lane_offset(uint32_t v) {
  asm("" : "+v"(v));
  return v;
}

// Slot addressing of the odd AA step on its fast lanes (cells whose
// neighbours are lattice cells, or the inlet/outlet ends).  The odd step
// reads direction opp(p) from, and writes direction p to, the same slot:
// plane p at cell c + xi_p.  Its byte address is split three ways:
//  * a scalar base per plane, A + p plane + c0 - nx + cz_p nx ny, reached by
//    stepping one plane stride at a time (plus the z shift), so that no
//    64-bit multiplication is spent on it (with the offsets formed from
//    plane, nx and ny at each access, the D3Q19 FP16S odd step issued about
//    600 scalar instructions per wavefront, 3.5 times the even step);
//  * a 32-bit lane offset per y shift, lo + (cy_p + 1) nx, three per cell;
//  * the x shift cx_p as the instruction's immediate offset.
// The lane offsets stay below 2^32 bytes where Geo::slot32 holds (checked on
// the host); elsewhere the odd step takes its generic path.
template <int Q, typename S>
struct OddSlots {
  typedef typename Glob<char>::type gchar;
  uint64_t plane0;  // scalar base of plane 0, bytes
  uint64_t pstep;   // plane stride, bytes
  uint64_t zstep;   // xy-layer stride, bytes
  uint32_t v[3];    // lane offsets for cy = -1, 0, +1, bytes
  __device__ __forceinline__ OddSlots(const Geo& g, const void* A, int64_t c0, uint32_t lo) {
    // (wave_uniform64 combines the two halves as unsigned words: the builtin
    // returns int, which a plain | would sign-extend into the high word)
    plane0 = (uint64_t)wave_uniform64((int64_t)((uint64_t)A + (uint64_t)((c0 - g.nx) * (int64_t)sizeof(S))));
    pstep = (uint64_t)wave_uniform64(g.plane * (int64_t)sizeof(S));
    zstep = (uint64_t)wave_uniform64((int64_t)g.nx * g.ny * (int64_t)sizeof(S));
    const uint32_t nxb = (uint32_t)g.nx * (uint32_t)sizeof(S);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      v[j] = lo * (uint32_t)sizeof(S) + (uint32_t)j * nxb;
      asm("" : "+v"(v[j]));  // kept as a 32-bit lane offset
    }
  }
  // The next plane's base from this one's (kept in scalar registers).
  __device__ __forceinline__ uint64_t next(uint64_t pb) const {
    pb += pstep;
    asm("" : "+s"(pb));
    return pb;
  }
  // Slot of plane p, given plane p's base.
  __device__ __forceinline__ typename Glob<S>::type* slot(uint64_t pb, int p) const {
    using L = Lat<Q>;
    if (L::cz[p] > 0) pb += zstep;
    if (L::cz[p] < 0) pb -= zstep;
    return (typename Glob<S>::type*)((gchar*)pb + v[L::cy[p] + 1] + L::cx[p] * (int)sizeof(S));
  }
};

// Reach of the fast lanes (OddSlots): an outlet lane's slots of planes
// with cx = +1 lie at cell indices up to n (one past the plane's cells, for
// cy = +1 and, in 3D, cz = +1), an inlet lane's slots of planes with cx = -1
// down to -1.  Both stay inside the population array when no plane of the
// first kind is the last one and no plane of the second kind is the first
// (the rest direction).
template <int Q>
constexpr bool odd_reach_in_bounds() {
  using L = Lat<Q>;
  for (int p = 0; p < Q; ++p) {
    if (L::cx[p] == 1 && L::cy[p] == 1 && (L::D == 2 || L::cz[p] == 1) && p == Q - 1) return false;
    if (L::cx[p] == -1 && p == 0) return false;
  }
  return true;
}
static_assert(odd_reach_in_bounds<9>() && odd_reach_in_bounds<19>(), "odd-step fast lanes would leave the array");

// Signed sum of the components selected by the (compile-time) lattice
// coefficients a, b, c in {-1, 0, 1}; zero terms are never formed, so no
// floating-point operation is spent on them.
template <typename T>
__device__ __forceinline__ T csum(int a, int b, int c, T x, T y, T z) {
  if (a != 0) {
    T r = a > 0 ? x : -x;
    if (b != 0) r = b > 0 ? r + y : r - y;
    if (c != 0) r = c > 0 ? r + z : r - z;
    return r;
  }
  if (b != 0) {
    T r = b > 0 ? y : -y;
    if (c != 0) r = c > 0 ? r + z : r - z;
    return r;
  }
  if (c != 0) return c > 0 ? z : -z;
  return (T)0;
}

// 1/x for the densities of the sweeps (x near 1): hardware reciprocal
// refined by Newton steps to within an ulp of the rounded quotient.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// Cells whose every neighbour is an ordinary lattice cell: no wall, inlet,
// outlet or periodic wrap (a whole wavefront usually qualifies).
template <int Q>
__device__ __forceinline__ bool interior_cell(const Geo& g, int x, int y, int z) {
  bool in = x > 0 && x < g.nx - 1 && y > 0 && y < g.ny - 1;
  if (Lat<Q>::D == 3) in = in && z > 0 && z < g.nz - 1;
  return in;
}

template <int Q>
__device__ __forceinline__ int64_t nb_offset(const Geo& g, int k) {
  return (int64_t)Lat<Q>::cx[k] + (int64_t)g.nx * ((int64_t)Lat<Q>::cy[k] + (int64_t)g.ny * Lat<Q>::cz[k]);
}

template <int Q, typename T>
__device__ __forceinline__ void cell_moments(const T (&s)[Q], T& drho, T& jx, T& jy, T& jz) {
  using L = Lat<Q>;
  // Sums start from their first term (no 0 + v), in direction order.
  bool hx = false, hy = false, hz = false;
  drho = s[0];
  jx = jy = jz = (T)0;
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    drho += s[k];
    if (L::cx[k] != 0) {
      jx = hx ? (L::cx[k] > 0 ? jx + s[k] : jx - s[k]) : (L::cx[k] > 0 ? s[k] : -s[k]);
      hx = true;
    }
    if (L::cy[k] != 0) {
      jy = hy ? (L::cy[k] > 0 ? jy + s[k] : jy - s[k]) : (L::cy[k] > 0 ? s[k] : -s[k]);
      hy = true;
    }
    if (L::cz[k] != 0) {
      jz = hz ? (L::cz[k] > 0 ? jz + s[k] : jz - s[k]) : (L::cz[k] > 0 ? s[k] : -s[k]);
      hz = true;
    }
  }
}

// Second moments p_ab = sum xi_a xi_b s of the shifted populations, in the
// order xx, yy, zz, xy, xz, yz (zz, xz, yz zero in 2D).
template <int Q, typename T>
__device__ __forceinline__ void second_moments(const T (&s)[Q], T (&p)[6]) {
  using L = Lat<Q>;
  // Signed sums over the directions with a nonzero coefficient, each started
  // from its first term (no 0 + v), in direction order.
#pragma unroll
  for (int m = 0; m < 6; ++m) p[m] = (T)0;
  bool h[6] = {false, false, false, false, false, false};
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int cf[6] = {L::cx[k] * L::cx[k], L::cy[k] * L::cy[k], L::cz[k] * L::cz[k],
                       L::cx[k] * L::cy[k], L::cx[k] * L::cz[k], L::cy[k] * L::cz[k]};
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      if (cf[m] == 0) continue;
      p[m] = h[m] ? (cf[m] > 0 ? p[m] + s[k] : p[m] - s[k]) : (cf[m] > 0 ? s[k] : -s[k]);
      h[m] = true;
    }
  }
}

// Non-equilibrium momentum flux with respect to f^eq(rho, u) from the second
// moments: Pi_ab = p_ab - (drho/3) delta_ab - j_a j_b / rho (same order).
// drho/3 as a product with the rounded 1/3 (within an ulp of the quotient;
// an IEEE division is a sequence of about ten instructions per lane).
template <int Q, typename T>
__device__ __forceinline__ void neq_from_moments(const T (&p)[6], T drho, T jx, T jy, T jz, T ir, T (&P)[6]) {
  const T pxx = p[0], pyy = p[1], pzz = p[2], pxy = p[3], pxz = p[4], pyz = p[5];
  const T d3 = drho * (T)(1.0 / 3.0);
  P[0] = pxx - d3 - jx * jx * ir;
  P[1] = pyy - d3 - jy * jy * ir;
  P[3] = pxy - jx * jy * ir;
  if (Lat<Q>::D == 3) {
    P[2] = pzz - d3 - jz * jz * ir;
    P[4] = pxz - jx * jz * ir;
    P[5] = pyz - jy * jz * ir;
  } else {
    P[2] = 0;
    P[4] = 0;
    P[5] = 0;
  }
}

// The same from the shifted populations.
template <int Q, typename T>
__device__ __forceinline__ void neq_flux(const T (&s)[Q], T drho, T jx, T jy, T jz, T ir, T (&P)[6]) {
  T p[6];
  second_moments<Q, T>(s, p);
  neq_from_moments<Q, T>(p, drho, jx, jy, jz, ir, P);
}

template <typename T>
__device__ __forceinline__ T frob2(const T (&P)[6]) {
  return P[0] * P[0] + P[1] * P[1] + P[2] * P[2] + (T)2 * (P[3] * P[3] + P[4] * P[4] + P[5] * P[5]);
}

// Symmetric-tensor storage used by the quadratic forms: 2D (xx, yy, xy),
// 3D (xx, yy, zz, xy, xz, yz).
template <int Q>
__device__ __forceinline__ int sym_index(int m6) {
  // maps 6-vector index to the compact storage index (or -1 if absent in 2D)
  if (Lat<Q>::D == 3) return m6;
  return m6 == 0 ? 0 : (m6 == 1 ? 1 : (m6 == 3 ? 2 : -1));
}

// a0 + a1.xi_i + a2:xi_i xi_i for a compact coefficient vector a.
// Only the terms with nonzero lattice coefficients are formed.
template <int Q, typename T>
__device__ __forceinline__ T quad_eval(const T* a, int i) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  const int c[3] = {L::cx[i], L::cy[i], D == 3 ? L::cz[i] : 0};
  if (c[0] == 0 && c[1] == 0 && c[2] == 0) return a[0];
  const T odd = csum<T>(c[0], c[1], c[2], a[1], a[2], D == 3 ? a[3] : (T)0);
  // a2 : xi xi over the symmetric storage (diagonal, then off-diagonal x2)
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  constexpr int NS = L::NSYM;
  const int sidx3[6] = {0, 1, 2, 3, 4, 5}, sidx2[6] = {0, 1, -1, 2, -1, -1};
  T even = (T)0;
  bool he = false;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int si = (NS == 6) ? sidx3[m] : sidx2[m];
    if (si < 0) continue;
    const int cf = c[ia[m]] * c[ib[m]] * (m < 3 ? 1 : 2);
    if (cf == 0) continue;
    const T v = a[1 + D + si];
    const T t = cf == 1 ? v : (cf == -1 ? -v : (T)cf * v);
    even = he ? even + t : t;
    he = true;
  }
  return he ? (a[0] + odd) + even : a[0] + odd;
}

// Objective terms of one region cell (Sec. 4, Eqs. obj_ffa and obj_diss),
// FP64: J, dJ/dd and the coefficients of dJ/df_i = a0 + a1.xi + a2:xi xi.
template <int Q>
__device__ void objective_terms(const ObjBox& ob, double d, double drho, double jx, double jy,
                                double jz, const double (&P)[6], double* out) {
  using C = Coef<Q>;
  constexpr int D = Lat<Q>::D;
#pragma unroll
  for (int m = 0; m < C::N; ++m) out[m] = 0.0;
  const double rho = 1.0 + drho, ir = 1.0 / rho;
  const double u[3] = {jx * ir, jy * ir, jz * ir};
  if (ob.kind == OBJ_FFA) {
    // J = rho (u_x u0 - u_x^2) + p0 - rho/3 ; dJ/df_i = u0 xi_x - 2 u_x xi_x + u_x^2 - 1/3
    out[C::J] = jx * ob.u0 - jx * jx * ir + ob.p0 - rho / 3.0;
    out[C::A0] = u[0] * u[0] - 1.0 / 3.0;
    out[C::A1] = ob.u0 - 2.0 * u[0];
  } else if (ob.kind == OBJ_DISS) {
    // J = cS Pi:Pi + cD |u|^2, cS = 9 nu/(2 tau0^2), cD = (1 - d)/tau0;
    // dJ/df_i = 2 cS Pi:[(xi-u)(xi-u) - I/3] + 2 cD u.(xi - u)/rho
    const double nu = (ob.tau0 - 0.5) / 3.0;
    const double cS = 9.0 * nu / (2.0 * ob.tau0 * ob.tau0);
    const double cD = (1.0 - d) / ob.tau0;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double Pm[3][3] = {{P[0], P[3], P[4]}, {P[3], P[1], P[5]}, {P[4], P[5], P[2]}};
    double Pu[3], uPu = 0.0;
    for (int a = 0; a < 3; ++a) {
      Pu[a] = Pm[a][0] * u[0] + Pm[a][1] * u[1] + Pm[a][2] * u[2];
      uPu += u[a] * Pu[a];
    }
    const double tr = P[0] + P[1] + P[2];
    out[C::J] = cS * frob2(P) + cD * uu;
    out[C::DJDD] = -uu / ob.tau0;
    out[C::A0] = 2.0 * cS * (uPu - tr / 3.0) - 2.0 * cD * uu * ir;
    for (int a = 0; a < D; ++a) out[C::A1 + a] = -4.0 * cS * Pu[a] + 2.0 * cD * u[a] * ir;
    for (int m6 = 0; m6 < 6; ++m6) {
      const int m = sym_index<Q>(m6);
      if (m >= 0) out[C::A2 + m] = 2.0 * cS * P[m6];
    }
  } else {
    out[C::J] = jx;
    out[C::A1] = 1.0;
  }
}

template <int Q>
__device__ __forceinline__ bool region_index(const ObjBox& ob, int x, int y, int z, int64_t& r) {
  const int rx = x - ob.lo[0], ry = y - ob.lo[1], rz = z - ob.lo[2];
  if (!ob.active || rx < 0 || ry < 0 || rz < 0 || rx >= ob.rn[0] || ry >= ob.rn[1] || rz >= ob.rn[2])
    return false;
  r = (int64_t)rx + (int64_t)ob.rn[0] * ((int64_t)ry + (int64_t)ob.rn[1] * rz);
  return true;
}

// acc[m * stride + r] += v[m], m < N.  Every old value is read before any is
// written back: the compiler has to assume that the slots may alias, so
// updates written one after the other would each wait for a memory round
// trip.
template <int N>
__device__ __forceinline__ void accumulate_terms(double* acc, int64_t stride, int64_t r, const double (&v)[N]) {
  double o[N];
#pragma unroll
  for (int m = 0; m < N; ++m) o[m] = acc[m * stride + r];
#pragma unroll
  for (int m = 0; m < N; ++m) acc[m * stride + r] = o[m] + v[m];
}

// ---- J_MEA, the momentum-exchange drag (Sec. 4, Eq. obj_mea) -------------
// J = (1/A) sum_{x in surface} sum_i xi_i,x (f_i(x + xi_i) - f_opp(i)(x)) is
// linear in f.  Collected by the slot each term reads it is
// J = sum_y sum_k g_k(y) f_k(y),  g_k(y) = (xi_k,x / A)(s(y) + s(y - xi_k)),
// with s the surface flag (0 unless y - xi_k is a lattice cell of the
// region).  g is the constant adjoint source; dJ/dd = 0.
// g is tabulated per region cell when the flags change (k_mea_source).
template <int Q>
__device__ __forceinline__ double mea_g(const Geo& g, const ObjBox& ob, int x, int y, int z, int64_t r,
                                        int k) {
  (void)g;
  (void)x;
  (void)y;
  (void)z;
  if (Lat<Q>::cx[k] == 0) return 0.0;
  return ob.mea[k * ob.rplane + r];
}

// Region-cell terms of J_MEA from the shifted state sd (only J is nonzero).
template <int Q>
__device__ __forceinline__ double mea_value(const Geo& g, const ObjBox& ob, int x, int y, int z, int64_t r,
                                            const double (&sd)[Q]) {
  using L = Lat<Q>;
  double J = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (L::cx[k] != 0) J += mea_g<Q>(g, ob, x, y, z, r, k) * (sd[k] + L::w[k]);
  return J;
}

template <int Q>
__device__ void mea_terms(const Geo& g, const ObjBox& ob, int x, int y, int z, int64_t r,
                          const double (&sd)[Q], double* out) {
#pragma unroll
  for (int m = 0; m < Coef<Q>::N; ++m) out[m] = 0.0;
  out[Coef<Q>::J] = mea_value<Q>(g, ob, x, y, z, r, sd);
}

// Neighbour (x + dx, y + dy, z + dz) of a lattice cell, dx, dy, dz in
// {-1, 0, 1} (compile-time after unrolling): wraps the periodic axes, flags a
// wall crossing (halfway bounce-back, which takes precedence) and an exit
// through the inlet/outlet ends of the x axis.  The same classification as
// classify(), written with selects and skipping the unchanged axes, so that
// the nine pulls and pushes of a boundary cell stay short and their loads
// issue back to back.
__device__ __forceinline__ void neighbour(const Geo& g, int dx, int dy, int dz, int& x, int& y, int& z,
                                          bool& bounce, bool& leaves) {
  bounce = false;
  leaves = false;
  if (dy != 0) {
    y += dy;
    const bool o = (y < 0) | (y >= g.ny), per = g.bcy == BC_PERIODIC;
    y += (o & per) ? (y < 0 ? g.ny : -g.ny) : 0;
    bounce = o & !per;
  }
  if (dz != 0) {
    z += dz;
    const bool o = (z < 0) | (z >= g.nz), per = g.bcz == BC_PERIODIC;
    z += (o & per) ? (z < 0 ? g.nz : -g.nz) : 0;
    bounce = bounce | (o & !per);
  }
  if (dx != 0) {
    x += dx;
    const bool o = (x < 0) | (x >= g.nx), per = g.bcx == BC_PERIODIC, walls = g.bcx == BC_WALLS;
    x += (o & per) ? (x < 0 ? g.nx : -g.nx) : 0;
    leaves = o & !per & !walls & !bounce;
    bounce = bounce | (o & walls);
  }
}

// AA odd-step pull of direction k into cell (x, y, z): post-collision value of
// the upstream cell (stored swapped), bounce-back from the own cell, or the
// outlet's virtual column.  The source address is selected, then loaded.
template <int Q, typename S, typename T>
__device__ __forceinline__ T pull(const Geo& g, const S* __restrict__ A, const S* __restrict__ ghost,
                                  int x, int y, int z, int64_t cell, int k) {
  using L = Lat<Q>;
  int sx = x, sy = y, sz = z;
  bool bounce, leaves;
  neighbour(g, -L::cx[k], -L::cy[k], -L::cz[k], sx, sy, sz, bounce, leaves);
  // leaves: the outlet's virtual column (an upstream position beyond x = nx-1)
  const int64_t ia = bounce ? k * g.plane + cell : L::opp[k] * g.plane + cell_of(g, sx, sy, sz);
  const S* pa = A + ia;
  const S* pg = ghost + (k * g.gplane + sy + (int64_t)g.ny * sz);
  return (T)*(leaves ? pg : pa);
}

// AA odd-step push of direction k from cell (x, y, z); a population that
// leaves through the inlet or outlet end is dropped.
template <int Q, typename S>
__device__ __forceinline__ void push(const Geo& g, S* __restrict__ A, int x, int y, int z,
                                     int64_t cell, int k, S v) {
  using L = Lat<Q>;
  int tx = x, ty = y, tz = z;
  bool bounce, leaves;
  neighbour(g, L::cx[k], L::cy[k], L::cz[k], tx, ty, tz, bounce, leaves);
  const int64_t ia = bounce ? L::opp[k] * g.plane + cell : k * g.plane + cell_of(g, tx, ty, tz);
  if (!leaves) A[ia] = v;
}

// Canonical (post-stream) state of a cell for either step parity.
template <int Q, typename S, typename T>
__device__ __forceinline__ void load_state(const Geo& g, const S* __restrict__ A,
                                           const S* __restrict__ ghost, int parity, int x, int y,
                                           int z, int64_t cell, T (&s)[Q]) {
  if (parity == 0) {
#pragma unroll
    for (int k = 0; k < Q; ++k) s[k] = (T)A[k * g.plane + cell];
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) s[k] = pull<Q, S, T>(g, A, ghost, x, y, z, cell, k);
  }
}

template <int Q, typename T>
__device__ __forceinline__ void inlet_state(const Geo& g, int y, T (&s)[Q]) {
  using L = Lat<Q>;
  const T ui = inlet_velocity<T>(g, y);
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const T cu = (T)L::cx[k] * ui;
    s[k] = (T)L::w[k] * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * ui * ui);
  }
}

// HRRLBM collision (Sec. 2.2, Eq. HRRLBM) on shifted populations s = f - w:
// s* = (f^eq - w) + (1 - omega) f^(1), f^eq the third-order Hermite
// equilibrium at (rho, u~ = d u), f^(1) the regularized non-equilibrium part
// with Hermite coefficients a1 = (1 - d) j, a2 = sum xi xi s - drho/3 I -
// rho u~u~ (projection) and a3 recursive (a3_aab = 2 u~_a a2_ab + u~_b a2_aa)
// on the supported third-order components.  The caller passes ir = 1/rho and
// the second moments p = sum xi xi s (second_moments), which the closure
// shares.
template <int Q, typename T>
__device__ __forceinline__ void hrr_collide(T (&s)[Q], T drho, T jx, T jy, T jz, T ir, T d, T omega,
                                            const double* force, const T (&p)[6]) {
  using L = Lat<Q>;
  using H = H3Types<Q>;
  constexpr int D = L::D;
  const T rho = (T)1 + drho;
  const T ut[3] = {d * jx * ir, d * jy * ir, d * jz * ir};
  // S = sum xi xi s from the caller's second moments p (xx, yy, zz, xy, xz, yz)
  const int pm[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  T a2[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      a2[a][b] = (a < D && b < D) ? p[pm[a][b]] - (a == b ? drho * (T)(1.0 / 3.0) : (T)0) - rho * ut[a] * ut[b]
                                  : (T)0;
  const T tt = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  const T tr = a2[0][0] + a2[1][1] + a2[2][2];
  T e3c[H::N], a3[H::N];
#pragma unroll
  for (int t = 0; t < H::N; ++t) {
    const int a = H::a[t], b = H::b[t];
    e3c[t] = rho * ut[a] * ut[a] * ut[b];
    a3[t] = (T)2 * ut[a] * a2[a][b] + ut[b] * a2[a][a];
  }
  // Per opposite pair (k, opp k): xi.u~, xi.j and the third-order terms
  // change sign, the second-order terms do not, so each pair is one
  // symmetric part plus or minus one antisymmetric part; only the nonzero
  // lattice coefficients enter the sums.  With xi.u~ = (d / rho) xi.j, the
  // per-cell factors are combined once, so that a pair costs one projection
  // xi.j, the second-order sum xi xi : a2 and one third-order sum:
  //   sym = w (base2 + kb (xi.j)^2 + kn xi xi : a2),
  //   asy = w (ka xi.j + sum_t H3_t(xi) c3_t),
  // base2 = base - kn tr(a2) / 3, kb = 4.5 rho (d/rho)^2, kn = 4.5 (1 - omega),
  // ka = 3 rho (d/rho) + 3 (1 - omega)(1 - d), c3_t = 13.5 (e3_t + (1 - omega) a3_t):
  // the equilibrium (base, 3 rho xi.u~, 4.5 rho (xi.u~)^2, 13.5 e3) plus
  // (1 - omega) times the regularised non-equilibrium part (4.5 xi xi : a2
  // minus its trace part, 3 (1 - d) xi.j, 13.5 a3).
  const T omd = (T)1 - d, om1 = (T)1 - omega;
  const T dir = d * ir;
  const T base = drho - (T)1.5 * rho * tt;  // the equilibrium's isotropic part
  const T kn = (T)4.5 * om1;
  const T base2 = base - kn * (tr * (T)(1.0 / 3.0));  // plus the isotropic part of xi xi : a2
  const T ka = (T)3 * rho * dir + om1 * ((T)3 * omd);
  const T kb = (T)4.5 * rho * dir * dir;
  T c3[H::N];
#pragma unroll
  for (int t = 0; t < H::N; ++t) c3[t] = (T)13.5 * (e3c[t] + om1 * a3[t]);
  s[0] = (T)L::w[0] * base2;
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    if (L::opp[k] < k) continue;
    const int o = L::opp[k];
    const T cj = csum<T>(L::cx[k], L::cy[k], L::cz[k], jx, jy, jz);
    T m2 = 0, g3 = 0;
    bool f2 = true, f3 = true;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (lat_c<Q>(k, a) * lat_c<Q>(k, b) != 0) {
          const T v = (T)(lat_c<Q>(k, a) * lat_c<Q>(k, b)) * a2[a][b];
          m2 = f2 ? v : m2 + v;
          f2 = false;
        }
#pragma unroll
    for (int t = 0; t < H::N; ++t) {
      const T h = (T)h3<Q>(k, t);
      if (h != (T)0) {
        g3 = f3 ? h * c3[t] : g3 + h * c3[t];
        f3 = false;
      }
    }
    const T w = (T)L::w[k];
    const T sym = w * (base2 + kb * cj * cj + kn * m2);
    const T asy = w * (ka * cj + g3);
    s[k] = sym + asy;
    s[o] = sym - asy;
  }
  if (force[0] != 0.0 || force[1] != 0.0 || force[2] != 0.0) {  // body force 3 w xi.F
#pragma unroll
    for (int k = 1; k < Q; ++k)
      s[k] += (T)(3.0 * L::w[k]) * csum<T>(L::cx[k], L::cy[k], L::cz[k], (T)force[0], (T)force[1], (T)force[2]);
  }
}

// Sweep kernels, two lane-to-cell maps over a 1D grid (workgroup order after
// the XCD renumbering of sweep_tile):
//  * runs (SWEEP_PROLOGUE_RUNS): workgroup b takes the 256 consecutive cells
//    [256 b, 256 b + 256) of the x-fastest order, one per lane; a wavefront's
//    64 cells run along a row and continue on the next row where one ends.
//    The block's first cell is uniform; its coordinates come from two uniform
//    divisions and each lane steps on from there.  No lanes are lost to
//    ragged row ends.  Used by the plain primal step and the tangent
//    (measured -9 % on the even, +1.5 % on the odd step, -2 % per pair on the
//    1100 x 410 lattice) and by the D3Q19 FP32/FP16 window steps and adjoint
//    (sweep_runs, adjoint_runs);
//  * tiles (SWEEP_PROLOGUE_TILES): 128 x 2 tiles of two half-rows.  Used by
//    the other window steps and adjoints (D2Q9: 3-4 % slower with runs).
__device__ __forceinline__ bool sweep_cell(const Geo& g, uint32_t c0, uint32_t lane, int& x, int& y, int& z) {
  const uint32_t nxy = (uint32_t)g.nx * (uint32_t)g.ny;
  const uint32_t z0 = (uint32_t)wave_uniform((int)(c0 / nxy));
  const uint32_t r0 = c0 - z0 * nxy;
  const uint32_t y0 = (uint32_t)wave_uniform((int)(r0 / (uint32_t)g.nx));
  x = (int)(r0 - y0 * (uint32_t)g.nx + lane);
  y = (int)y0;
  z = (int)z0;
  while (x >= g.nx) {  // at most 1 + 255 / nx times
    x -= g.nx;
    if (++y == g.ny) {
      y = 0;
      ++z;
    }
  }
  return z < g.nz;
}

// Lane map and tile order of the sweeps, chosen per stencil and precision by
// measurement on 768 x 384 x 128 (D3Q19) and 8192 x 4096 (D2Q9):
//  * sweep_runs: runs for every plain step, and for the window steps of D3Q19
//    with FP32/FP16 populations (window sweep 1717 -> 1695 us FP32,
//    1174 -> 1121 FP16S against 128 x 2 tiles; FP64 +1 %: tiles stay);
//  * runs_remap: the XCD renumbering of sweep_tile for D2Q9 runs (its odd
//    step's x-neighbouring runs share cache lines) and for the D3Q19 FP64 odd
//    plain step; every other D3Q19 run keeps the dispatch order, in which the
//    XCDs sweep neighbouring runs at the same time (per plain step: FP16S
//    even 596 -> 544 us, odd 667 -> 635; FP32 1121 -> 1094, 1150 -> 1127;
//    FP64 even 2285 -> 2223, but odd 2323 -> 2557, so that one keeps it; in
//    D2Q9 the dispatch order measured -2 % to +6 %);
//  * adjoint_runs: the D3Q19 adjoint with an FP32 adjoint state takes runs in
//    dispatch order (FP32 1244 -> 1194 us, FP16S lattices 1245 -> 1185;
//    FP64 +0.5 %: tiles stay).
// Tiles always take the renumbering (the dispatch order measured 2-13 %
// slower for them).
template <int Q, typename S, int ACC>
__host__ __device__ constexpr bool sweep_runs() {
  return ACC == 0 || (Lat<Q>::D == 3 && sizeof(S) <= 4);
}
template <int Q, typename S, bool ODD, int ACC>
__host__ __device__ constexpr bool runs_remap() {
  return Lat<Q>::D == 2 || (ACC == 0 && ODD && sizeof(S) == 8);
}
template <int Q, typename SA>
__host__ __device__ constexpr bool adjoint_runs() {
  return Lat<Q>::D == 3 && sizeof(SA) == 4;
}

#define SWEEP_PROLOGUE_RUNS(REMAP)                                            \
  const int t_ = sweep_tile((int)blockIdx.x, (int)gridDim.x, (REMAP));        \
  const int64_t tile_c0 = (int64_t)t_ * SWEEP_BLOCK;                          \
  const uint32_t tile_lo = lane_offset(threadIdx.x);                          \
  int x, y, z;                                                                \
  const bool valid = sweep_cell(g, (uint32_t)tile_c0, threadIdx.x, x, y, z);  \
  const int64_t cell = tile_c0 + threadIdx.x;                                 \
  const bool inout = (g.bcx == BC_INOUT);                                     \
  (void)inout;                                                                \
  (void)tile_lo;                                                              \
  (void)cell;

#define SWEEP_PROLOGUE_TILES                                                 \
  const int t_ = sweep_tile((int)blockIdx.x, (int)gridDim.x);                \
  const int z = wave_uniform(t_ / (g.tiles_x * g.tiles_y));                  \
  const int r_ = t_ - z * g.tiles_x * g.tiles_y;                             \
  const int x0_ = wave_uniform((r_ % g.tiles_x) * BX);                       \
  const int y0_ = wave_uniform((r_ / g.tiles_x) * BY);                       \
  const int x = x0_ + threadIdx.x;                                           \
  const int y = y0_ + threadIdx.y;                                           \
  const bool valid = (x < g.nx) && (y < g.ny);                               \
  const int64_t cell = valid ? cell_of(g, x, y, z) : 0;                      \
  const int64_t tile_c0 = wave_uniform64(cell_of(g, x0_, y0_, z));          \
  const uint32_t tile_lo = lane_offset(threadIdx.x + (uint32_t)g.nx * threadIdx.y); \
  const bool inout = (g.bcx == BC_INOUT);                                    \
  (void)inout;                                                               \
  (void)cell;

#define CELL_PROLOGUE                                   \
  const int x = blockIdx.x * BX + threadIdx.x;          \
  const int y = blockIdx.y * BY + threadIdx.y;          \
  const int z = blockIdx.z;                             \
  const bool valid = (x < g.nx) && (y < g.ny);          \
  const int64_t cell = valid ? cell_of(g, x, y, z) : 0; \
  const bool inout = (g.bcx == BC_INOUT);               \
  (void)inout;                                          \
  (void)cell;

// =========================================================================
// primal sweep (rows a3, a4, a5): HLBM-BGK collision (Eq. hlbm) toward
// f^eq(rho, d u), optional Smagorinsky tau_eff (Eqs. turbVisc, tauEff),
// AA propagation with boundaries, fused FP64 window accumulation.
// =========================================================================

// One lattice update of cell (x, y, z) (inside the lattice), at lane offset
// lo from its tile's first cell c0 (see plane_base).
// ACC: 0 no window; 1 window with the moment-form objective terms; 2 window
// with J_MEA (its own terms; a separate instantiation keeps the register
// budget of the common case); 3 window statistics only, the objective terms
// of a small region being accumulated by k_window_region before the step.
template <int Q, typename S, bool ODD, int ACC, bool HRR, bool NT = false, bool NTW = NT>
__device__ __forceinline__ void primal_cell(const Geo& g, const Coll& c, const ObjBox& ob, S* __restrict__ A,
                                            const typename Prec<S>::Dd* __restrict__ dpor,
                                            S* __restrict__ ghost, const Acc& acc, const int x, const int y,
                                            const int z, const int64_t c0, const uint32_t lo) {
  using L = Lat<Q>;
  using T = typename Prec<S>::T;
  const int64_t cell = c0 + lo;
  const bool inout = (g.bcx == BC_INOUT);
  // The pinned inlet (x = 0: equilibrium inflow, not collided, a source only)
  // and the outlet (x = nx-1) of an inlet/outlet channel.
  const bool inlet = inout && x == 0, outlet = inout && (x == g.nx - 1);
  // Fast lanes: every lane of the even step; in the odd step the cells whose
  // neighbours are ordinary cells except across the inlet and outlet ends,
  // i.e. the interior cells plus the inlet and outlet cells of rows away from
  // walls and periodic seams.  They run one instruction stream (the inlet and
  // outlet only switch a few loads and stores), so a wavefront that holds a
  // row end does not run a second, generic path for it.
  bool fast = true;
  if constexpr (ODD) {
    const bool rows = y > 0 && y < g.ny - 1 && (L::D == 2 || (z > 0 && z < g.nz - 1));
    fast = g.slot32 && rows && ((x > 0 && x < g.nx - 1) || inlet || outlet);
  }
  T s[Q];
  if (inlet && !fast) {  // odd step, inlet cell of a wall row: pinned, pushed
    inlet_state<Q, T>(g, y, s);
#pragma unroll
    for (int k = 0; k < Q; ++k) push<Q, S>(g, A, x, y, z, cell, k, to_store<S>(s[k]));
    return;
  }
  // Porosity and populations are requested together.
  const T d = (T)at(dpor, c0, lo);
  // Grouped window accumulation (FP32 arithmetic, acc.pend set): of every
  // PEND_GROUP consecutive window steps the first PEND_GROUP - 1 store their
  // values (drho, j, tau_eff, f) as FP32 in a pending slot instead of adding
  // them to the FP64 sums, and the last adds the pending values in step
  // order before its own (acc.pend_in): the sums receive
  // sum + v_1 + ... + v_K, the same FP64 additions in the same order as when
  // each step adds its value at once (bitwise the same sums), with one FP64
  // read-modify-write per group instead of one per step.  The values are
  // FP32 already, so storing them loses nothing.
  constexpr bool GROUPED = sizeof(T) == 4;
  constexpr int KP = PEND_GROUP - 1;  // pending slots
  const bool pend_out = GROUPED && ACC != 0 && acc.pend_out >= 0;
  const bool pend_add = GROUPED && ACC != 0 && acc.pend_in != 0;
  // Window sums of rho and j: their old values are requested with the
  // populations (and all of them before any is written back, see
  // accumulate_terms).  The inlet's slots are read but not updated.  The
  // dense window sums take their own cache hints (NTW: the populations' in
  // the streaming kernels, and streaming in the D3Q19 odd window step too).
  double wold[L::D + 1];
  float pold[KP][L::D + 1];
  if constexpr (ACC != 0) {
    if (!pend_out) {
      wold[0] = ld_stream<NTW>(&at(acc.rho, c0, lo));
#pragma unroll
      for (int a = 0; a < L::D; ++a) wold[1 + a] = ld_stream<NTW>(&at(acc.j, a * g.plane + c0, lo));
    }
    if (pend_add) {
#pragma unroll
      for (int i = 0; i < KP; ++i)
#pragma unroll
        for (int a = 0; a <= L::D; ++a)
          pold[i][a] = ld_stream<NTW>(&at(acc.pend, i * acc.pslot + a * g.plane + c0, lo));
    }
  }
  // All population loads are issued before any arithmetic on them (the
  // scheduler otherwise interleaves early sums, which forces a wait for the
  // first loads before the remaining ones are even issued).
  if (!ODD) {
#pragma unroll
    for (int k = 0; k < Q; ++k) s[k] = (T)ld_stream<NT>(&at(A, k * g.plane + c0, lo));
    __builtin_amdgcn_sched_barrier(0);
  } else if (fast && ACC == 0) {
    // Every fast lane requests all its slots, the inlet and outlet lanes
    // included: their requests across the row end (x - xi_k = -1 or nx) land
    // on in-bounds slots of other cells (OddSlots, odd_reach_in_bounds), and
    // those values are replaced below.
    const OddSlots<Q, S> sl(g, A, c0, lo);
    uint64_t pb = sl.plane0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      s[L::opp[p]] = (T)ld_stream<NT>(sl.slot(pb, p));
      pb = sl.next(pb);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (outlet) {  // upstream (nx, y - cy, z - cz): the virtual column
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (L::cx[k] == -1) s[k] = (T)ghost[k * g.gplane + (y - L::cy[k]) + (int64_t)g.ny * (z - L::cz[k])];
    }
  } else if (fast) {
    // The window steps address each slot from its own scalar base (plane and
    // neighbour offset formed per access): with the plane-stepped bases of
    // OddSlots the D2Q9 window steps measured 3-7 % slower (same addresses;
    // the plain steps, which are not bound by memory alone in FP16, 7-15 %
    // faster with them).
    if (!inlet) {  // the inlet's upstream lies outside the lattice
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (L::cx[k] == -1 && outlet)  // upstream (nx, y - cy, z - cz): the virtual column
          s[k] = (T)ghost[k * g.gplane + (y - L::cy[k]) + (int64_t)g.ny * (z - L::cz[k])];
        else
          s[k] = (T)ld_stream<NT>(&at(A, L::opp[k] * g.plane + c0 - nb_offset<Q>(g, k), lo));
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) s[k] = pull<Q, S, T>(g, A, ghost, x, y, z, cell, k);
  }
  if (ODD && inlet) {  // loaded nothing; its update is replaced by the pinned values below
#pragma unroll
    for (int k = 0; k < Q; ++k) s[k] = (T)0;
  }
  if constexpr (ACC == 3) {  // a small region's cells hand their state to the region pass
    int64_t rr;
    if (acc.rcopy && region_index<Q>(ob, x, y, z, rr)) {
      // one record of whole 128-byte lines per cell, written as 16-byte vectors
      constexpr int RC = region_copy_stride(Q, (int)sizeof(T));
      constexpr int V = 16 / (int)sizeof(T);
      typedef T TV __attribute__((ext_vector_type(V)));
      TV* rc = (TV*)((T*)acc.rcopy + rr * RC);
#pragma unroll
      for (int v = 0; v < RC / V; ++v) {
        TV t;
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const int k = v * V + i;
          t[i] = k < Q ? s[k < Q ? k : 0] : (k == Q ? d : (T)0);
        }
        rc[v] = t;
      }
    }
  }

  T drho, jx, jy, jz;
  cell_moments<Q, T>(s, drho, jx, jy, jz);
  const T rho = (T)1 + drho;
  const T ir = recip(rho);

  if (cell == c.probe_cell && !inlet) *c.probe_out = (double)(jy * ir);
  T omega = (T)c.omega0;
  T taue = (T)c.tau0;
  T p2[6];  // second moments, shared by the closure and the HRR collision
  if constexpr (HRR) second_moments<Q, T>(s, p2);
  if (c.smag) {
    T P[6];
    if constexpr (HRR)
      neq_from_moments<Q, T>(p2, drho, jx, jy, jz, ir, P);
    else
      neq_flux<Q, T>(s, drho, jx, jy, jz, ir, P);
    const T tau0 = (T)c.tau0;
    taue = (T)0.5 * (tau0 + sqrt(tau0 * tau0 + (T)c.kS * sqrt(frob2(P))));
    omega = recip(taue);  // refined hardware reciprocal, as for 1/rho
  }

  // Objective terms of a region cell (moment form): from the pre-collision
  // moments, evaluated after the stores so that their temporaries do not
  // add to the collision's register budget.
  bool in_region = false;
  int64_t r = 0;
  double odr = 0.0, oax = 0.0, oay = 0.0, oaz = 0.0, oP[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double omea = 0.0;  // J_MEA of the cell
  (void)omea;
  (void)odr;
  (void)oax;
  (void)oay;
  (void)oaz;
  if (ACC != 0 && !inlet) {  // the pinned inlet is not part of the window
    // pending slot planes: drho, j (D), tau_eff, then f (Q)
    constexpr int PT = L::D + 1, PF = L::D + 2;
    const int64_t sb = pend_out ? (int64_t)acc.pend_out * acc.pslot : 0;
    if (pend_out) {
      st_stream<NTW>(&at(acc.pend, sb + c0, lo), (float)drho);
      st_stream<NTW>(&at(acc.pend, sb + g.plane + c0, lo), (float)jx);
      st_stream<NTW>(&at(acc.pend, sb + 2 * g.plane + c0, lo), (float)jy);
      if constexpr (L::D == 3) st_stream<NTW>(&at(acc.pend, sb + 3 * g.plane + c0, lo), (float)jz);
    } else {
      if (pend_add) {
#pragma unroll
        for (int i = 0; i < KP; ++i)
#pragma unroll
          for (int a = 0; a <= L::D; ++a) wold[a] = wold[a] + (double)pold[i][a];
      }
      st_stream<NTW>(&at(acc.rho, c0, lo), wold[0] + (double)drho);
      st_stream<NTW>(&at(acc.j, c0, lo), wold[1] + (double)jx);
      st_stream<NTW>(&at(acc.j, g.plane + c0, lo), wold[2] + (double)jy);
      if constexpr (L::D == 3) st_stream<NTW>(&at(acc.j, 2 * g.plane + c0, lo), wold[3] + (double)jz);
    }
    if (acc.f) {  // in groups of 4 (read, then write back)
      if (pend_out) {
#pragma unroll
        for (int k = 0; k < Q; ++k) st_stream<NTW>(&at(acc.pend, sb + (PF + k) * g.plane + c0, lo), (float)s[k]);
      } else {
#pragma unroll
        for (int k0 = 0; k0 < Q; k0 += 4) {
          double o[4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (k0 + i < Q) o[i] = ld_stream<NTW>(&at(acc.f, (k0 + i) * g.plane + c0, lo));
          if (pend_add) {
            float po[KP][4];
#pragma unroll
            for (int j = 0; j < KP; ++j)
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (k0 + i < Q)
                  po[j][i] = ld_stream<NTW>(&at(acc.pend, j * acc.pslot + (PF + k0 + i) * g.plane + c0, lo));
#pragma unroll
            for (int j = 0; j < KP; ++j)
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (k0 + i < Q) o[i] = o[i] + (double)po[j][i];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (k0 + i < Q) st_stream<NTW>(&at(acc.f, (k0 + i) * g.plane + c0, lo), o[i] + (double)s[k0 + i]);
        }
      }
    }
    if (acc.tau) {
      if (pend_out) {
        st_stream<NTW>(&at(acc.pend, sb + PT * g.plane + c0, lo), (float)taue);
      } else {
        double ot = ld_stream<NTW>(&at(acc.tau, c0, lo));
        if (pend_add) {
          float pt[KP];
#pragma unroll
          for (int j = 0; j < KP; ++j) pt[j] = ld_stream<NTW>(&at(acc.pend, j * acc.pslot + PT * g.plane + c0, lo));
#pragma unroll
          for (int j = 0; j < KP; ++j) ot = ot + (double)pt[j];
        }
        st_stream<NTW>(&at(acc.tau, c0, lo), ot + (double)taue);
      }
    }
    if constexpr (ACC == 1 || ACC == 2) in_region = region_index<Q>(ob, x, y, z, r);
    if (in_region) {
      double sd[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) sd[k] = (double)s[k];
      if constexpr (ACC == 2) {  // J_MEA (linear in f): only its J term is nonzero
        omea = mea_value<Q>(g, ob, x, y, z, r, sd);
      } else {  // moments of the pre-collision state; the terms follow the stores
        cell_moments<Q, double>(sd, odr, oax, oay, oaz);
        neq_flux<Q, double>(sd, odr, oax, oay, oaz, 1.0 / (1.0 + odr), oP);
      }
    }
  }

  if constexpr (HRR) {
    hrr_collide<Q, T>(s, drho, jx, jy, jz, ir, d, omega, c.force, p2);
  } else {
    // s <- (1 - omega) s + omega (f^eq(rho, u~) - w), u~ = d j / rho, written
    // per opposite pair (k, opp k): with cu = xi_k . u~ the equilibrium is
    // w (A0 + C cu^2) +- w B cu, A0 = drho - 1.5 rho u~^2, B = 3 rho,
    // C = 4.5 rho; omega is folded into A0, B and C.
    const T dir = d * ir;
    const T tx = jx * dir, ty = jy * dir, tz = (L::D == 3) ? jz * dir : (T)0;
    const T tt = (L::D == 3) ? tx * tx + ty * ty + tz * tz : tx * tx + ty * ty;
    const T orho = omega * rho;
    const T a0 = omega * drho - (T)1.5 * orho * tt;
    const T b1 = (T)3 * orho, c2 = (T)4.5 * orho;
    const T omc = (T)1 - omega;
    s[0] = omc * s[0] + (T)L::w[0] * a0;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      if (L::opp[k] < k) continue;
      const int o = L::opp[k];
      const T w = (T)L::w[k];
      const T cu = csum<T>(L::cx[k], L::cy[k], L::cz[k], tx, ty, tz);
      const T sym = (w * a0) + ((w * c2) * cu) * cu;
      const T asy = (w * b1) * cu;
      s[k] = omc * s[k] + (sym + asy);
      s[o] = omc * s[o] + (sym - asy);
    }
    if (c.force[0] != 0.0 || c.force[1] != 0.0 || c.force[2] != 0.0) {  // body force 3 w xi.F
#pragma unroll
      for (int k = 1; k < Q; ++k)
        s[k] += (T)(3.0 * L::w[k]) *
                csum<T>(L::cx[k], L::cy[k], L::cz[k], (T)c.force[0], (T)c.force[1], (T)c.force[2]);
    }
  }

  if (inlet) inlet_state<Q, T>(g, y, s);  // pinned: not collided

  if (!ODD) {
#pragma unroll
    for (int k = 0; k < Q; ++k) st_stream<NT>(&at(A, L::opp[k] * g.plane + c0, lo), to_store<S>(s[k]));
    if (outlet) {
      const T ux = jx * ir, uy = jy * ir, uz = jz * ir;
      const T uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (L::cx[k] != -1) continue;
        const T cu = (T)L::cx[k] * ux + (T)L::cy[k] * uy + (T)L::cz[k] * uz;
        const T vs = (T)L::w[k] * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);
        ghost[k * g.gplane + y + (int64_t)g.ny * z] = to_store<S>(vs);
      }
    }
  } else {
    if (fast && ACC == 0) {
      const OddSlots<Q, S> sl(g, A, c0, lo);
      uint64_t pb = sl.plane0;
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        // populations leaving through the inlet or outlet end are dropped
        if (!((L::cx[p] == -1 && inlet) || (L::cx[p] == 1 && outlet)))
          st_stream<NT>(sl.slot(pb, p), to_store<S>(s[p]));
        pb = sl.next(pb);
      }
    } else if (fast) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if ((L::cx[k] == -1 && inlet) || (L::cx[k] == 1 && outlet)) continue;
        st_stream<NT>(&at(A, k * g.plane + c0 + nb_offset<Q>(g, k), lo), to_store<S>(s[k]));
      }
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) push<Q, S>(g, A, x, y, z, cell, k, to_store<S>(s[k]));
    }
    if (outlet) {
      const T ux = jx * ir, uy = jy * ir, uz = jz * ir;
      const T uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (L::cx[k] != -1) continue;
        const T cu = (T)L::cx[k] * ux + (T)L::cy[k] * uy + (T)L::cz[k] * uz;
        const T vs = (T)L::w[k] * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);
        if (fast) {  // away from walls and seams (nx-1, y+cy, z+cz) is a lattice cell
          at(A, k * g.plane + c0 + (int64_t)L::cy[k] * g.nx + (int64_t)L::cz[k] * g.nx * g.ny, lo) = to_store<S>(vs);
        } else {
          int vx = x, vy = y + L::cy[k], vz = z + L::cz[k];
          if (classify(g, vx, vy, vz) != NB_CELL) continue;
          A[k * g.plane + cell_of(g, vx, vy, vz)] = to_store<S>(vs);
        }
      }
    }
  }
  if constexpr (ACC == 1) {
    if (in_region) {
      double terms[Coef<Q>::N];
      objective_terms<Q>(ob, (double)d, odr, oax, oay, oaz, oP, terms);
      accumulate_terms<Coef<Q>::N>(acc.obj, ob.rplane, r, terms);
    }
  }
  if constexpr (ACC == 2) {
    if (in_region) acc.obj[Coef<Q>::J * ob.rplane + r] += omea;
  }
}

template <int Q, typename S, bool ODD, int ACC, bool HRR, bool NT, bool NTW = NT>
__device__ __forceinline__ void primal_sweep(const Geo& g, const Coll& c, const ObjBox& ob, S* __restrict__ A,
                                             const typename Prec<S>::Dd* __restrict__ dpor,
                                             S* __restrict__ ghost, const Acc& acc) {
  if constexpr (sweep_runs<Q, S, ACC>()) {
    SWEEP_PROLOGUE_RUNS((runs_remap<Q, S, ODD, ACC>()))
    if (!valid) return;
    primal_cell<Q, S, ODD, ACC, HRR, NT, NTW>(g, c, ob, A, dpor, ghost, acc, x, y, z, tile_c0, tile_lo);
  } else {
    SWEEP_PROLOGUE_TILES
    if (!valid) return;
    primal_cell<Q, S, ODD, ACC, HRR, NT, NTW>(g, c, ob, A, dpor, ghost, acc, x, y, z, tile_c0, tile_lo);
  }
}

template <int Q, typename S, bool ODD, int ACC, bool HRR>
__global__ __launch_bounds__(256) void k_primal(const Geo g, const Coll c, const ObjBox ob,
                                                S* __restrict__ A,
                                                const typename Prec<S>::Dd* __restrict__ dpor,
                                                S* __restrict__ ghost, const Acc acc) {
  primal_sweep<Q, S, ODD, ACC, HRR, false>(g, c, ob, A, dpor, ghost, acc);
}

// The same sweep with streaming hints on the population loads and stores
// (lattices larger than the Infinity Cache, see ld_stream).
template <int Q, typename S, bool ODD, int ACC, bool HRR>
__global__ __launch_bounds__(256) void k_primal_stream(const Geo g, const Coll c, const ObjBox ob,
                                                       S* __restrict__ A,
                                                       const typename Prec<S>::Dd* __restrict__ dpor,
                                                       S* __restrict__ ghost, const Acc acc) {
  primal_sweep<Q, S, ODD, ACC, HRR, true>(g, c, ob, A, dpor, ghost, acc);
}

// Window steps of D3Q19 odd parity above the Infinity Cache: plain accesses
// to the populations (their z neighbours reuse lines one xy layer later) and
// streaming hints on the window sums, which are the cell's own and read and
// written once (1-3 % faster than plain sums on 768 x 384 x 128).
template <int Q, typename S, bool ODD, int ACC, bool HRR>
__global__ __launch_bounds__(256) void k_primal_wstream(const Geo g, const Coll c, const ObjBox ob,
                                                        S* __restrict__ A,
                                                        const typename Prec<S>::Dd* __restrict__ dpor,
                                                        S* __restrict__ ghost, const Acc acc) {
  primal_sweep<Q, S, ODD, ACC, HRR, false, true>(g, c, ob, A, dpor, ghost, acc);
}

// =========================================================================
// bandwidth probe (measurement, outside the method): a plain primal step's
// memory traffic -- every population slot and the porosity of each cell read,
// the populations written back unchanged -- on the same 256-cell runs, tile
// order and scalar-base addressing, without any arithmetic.  Its time per
// launch is the practical ceiling of an in-place sweep on this lattice.
// ODD: interior cells read and write the odd step's upstream slots (slot
// opp(k) of the neighbour at x - xi_k), every other cell its own slots.
// =========================================================================
template <int Q, typename S, bool ODD, bool NT>
__global__ __launch_bounds__(256) void k_copy_probe(const Geo g, S* __restrict__ A,
                                                    const typename Prec<S>::Dd* __restrict__ dpor,
                                                    int* __restrict__ sink) {
  SWEEP_PROLOGUE_RUNS((runs_remap<Q, S, ODD, 0>()))  // the plain step's order
  if (!valid) return;
  const auto d = at(dpor, tile_c0, tile_lo);
  S v[Q];
  const bool nb = ODD && g.slot32 && interior_cell<Q>(g, x, y, z);
  if (nb) {  // the slots of plane p at c + xi_p, addressed as the odd sweep does
    const OddSlots<Q, S> sl(g, A, tile_c0, tile_lo);
    uint64_t pb = sl.plane0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      v[p] = ld_stream<NT>(sl.slot(pb, p));
      pb = sl.next(pb);
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) v[k] = ld_stream<NT>(&at(A, k * g.plane + tile_c0, tile_lo));
  }
  __builtin_amdgcn_sched_barrier(0);
  // opaque values: a store of the value just loaded from the same address
  // would otherwise be removed as redundant
#pragma unroll
  for (int k = 0; k < Q; ++k) asm volatile("" : "+v"(v[k]));
  if (d < 0) *sink = 1;  // never taken (d is in [0, 1]); keeps the porosity load
  if (nb) {
    const OddSlots<Q, S> sl(g, A, tile_c0, tile_lo);
    uint64_t pb = sl.plane0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      st_stream<NT>(sl.slot(pb, p), v[p]);
      pb = sl.next(pb);
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) st_stream<NT>(&at(A, k * g.plane + tile_c0, tile_lo), v[k]);
  }
}

// The two-array pull pattern, measured as the alternative to the in-place AA
// propagation (a probe, not a step of the method): interior cells read slot
// k of their upstream cell c - xi_k in the lattice's array and write their
// own slot k of a second array of the same layout with streaming hints;
// other cells read their own slots.  A plain sweep's bytes again, with twice
// the population memory.  Same runs and order as the plain step.
template <int Q, typename S>
__global__ __launch_bounds__(256) void k_copy_probe_pull(const Geo g, const S* __restrict__ A, S* __restrict__ B,
                                                         const typename Prec<S>::Dd* __restrict__ dpor,
                                                         int* __restrict__ sink) {
  SWEEP_PROLOGUE_RUNS((runs_remap<Q, S, false, 0>()))
  if (!valid) return;
  const auto d = at(dpor, tile_c0, tile_lo);
  const bool nb = interior_cell<Q>(g, x, y, z);
  S v[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) v[k] = A[k * g.plane + cell - (nb ? nb_offset<Q>(g, k) : 0)];
  __builtin_amdgcn_sched_barrier(0);
  if (d < 0) *sink = 1;  // never taken (d is in [0, 1]); keeps the porosity load
#pragma unroll
  for (int k = 0; k < Q; ++k) st_stream<true>(&at(B, k * g.plane + tile_c0, tile_lo), v[k]);
}

// =========================================================================
// forward tangent (App. C): one primal step of BGK-HLBM together with its
// directional derivative fdot = (df/dd) v (FP64, no closure).  The tangent
// lives in a second AA population array and follows exactly the same
// propagation and boundaries; the pinned inlet has a zero tangent and the
// outlet's virtual values V = f^eq(1, u) carry dV = (dV/du) du.
// =========================================================================
template <int Q, bool ODD>
__device__ __forceinline__ void tangent_cell(const Geo& g, const Coll& c, double* __restrict__ A,
                                             double* __restrict__ At, const double* __restrict__ dpor,
                                             const double* __restrict__ v, double* __restrict__ ghost,
                                             double* __restrict__ ghostt, const int x, const int y,
                                             const int z) {
  using L = Lat<Q>;
  const int64_t cell = cell_of(g, x, y, z);
  const bool inout = (g.bcx == BC_INOUT);
  double s[Q], t[Q];
  if (inout && x == 0) {
    inlet_state<Q, double>(g, y, s);
    if (!ODD) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        A[L::opp[k] * g.plane + cell] = s[k];
        At[L::opp[k] * g.plane + cell] = 0.0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        push<Q, double>(g, A, x, y, z, cell, k, s[k]);
        push<Q, double>(g, At, x, y, z, cell, k, 0.0);
      }
    }
    return;
  }
  const bool interior = ODD && interior_cell<Q>(g, x, y, z);
  if (!ODD) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      s[k] = A[k * g.plane + cell];
      t[k] = At[k * g.plane + cell];
    }
  } else if (interior) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t o = L::opp[k] * g.plane + cell - nb_offset<Q>(g, k);
      s[k] = A[o];
      t[k] = At[o];
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      s[k] = pull<Q, double, double>(g, A, ghost, x, y, z, cell, k);
      t[k] = pull<Q, double, double>(g, At, ghostt, x, y, z, cell, k);
    }
  }
  double drho, jx, jy, jz, tr, tjx, tjy, tjz;
  cell_moments<Q, double>(s, drho, jx, jy, jz);
  cell_moments<Q, double>(t, tr, tjx, tjy, tjz);
  const double rho = 1.0 + drho, ir = 1.0 / rho;
  const double ux = jx * ir, uy = jy * ir, uz = jz * ir;
  // du = (dj - u drho) / rho
  const double dux = (tjx - ux * tr) * ir, duy = (tjy - uy * tr) * ir, duz = (tjz - uz * tr) * ir;
  const double d = dpor[cell], vd = v[cell];
  // u~ = d u, du~ = d du + u v
  const double tx = d * ux, ty = d * uy, tz = d * uz;
  const double dtx = d * dux + vd * ux, dty = d * duy + vd * uy, dtz = d * duz + vd * uz;
  const double tt = tx * tx + ty * ty + tz * tz;
  const double dtt = 2.0 * (tx * dtx + ty * dty + tz * dtz);
  const double omega = c.omega0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double cu = L::cx[k] * tx + L::cy[k] * ty + L::cz[k] * tz;
    const double dcu = L::cx[k] * dtx + L::cy[k] * dty + L::cz[k] * dtz;
    const double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * tt;
    const double feqs = L::w[k] * (drho + rho * poly);
    const double dfeqs = L::w[k] * (tr + tr * poly + rho * (3.0 * dcu + 9.0 * cu * dcu - 1.5 * dtt));
    const double fk = 3.0 * L::w[k] * (L::cx[k] * c.force[0] + L::cy[k] * c.force[1] + L::cz[k] * c.force[2]);
    s[k] = s[k] + omega * (feqs - s[k]) + fk;
    t[k] = t[k] + omega * (dfeqs - t[k]);
  }
  const bool outlet = inout && (x == g.nx - 1);
  const double uu = ux * ux + uy * uy + uz * uz;
  const double duu = 2.0 * (ux * dux + uy * duy + uz * duz);
  if (!ODD) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      A[L::opp[k] * g.plane + cell] = s[k];
      At[L::opp[k] * g.plane + cell] = t[k];
    }
    if (outlet) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (L::cx[k] != -1) continue;
        const double cu = L::cx[k] * ux + L::cy[k] * uy + L::cz[k] * uz;
        const double dcu = L::cx[k] * dux + L::cy[k] * duy + L::cz[k] * duz;
        const int64_t o = k * g.gplane + y + (int64_t)g.ny * z;
        ghost[o] = L::w[k] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        ghostt[o] = L::w[k] * (3.0 * dcu + 9.0 * cu * dcu - 1.5 * duu);
      }
    }
  } else if (interior) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t o = k * g.plane + cell + nb_offset<Q>(g, k);
      A[o] = s[k];
      At[o] = t[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      push<Q, double>(g, A, x, y, z, cell, k, s[k]);
      push<Q, double>(g, At, x, y, z, cell, k, t[k]);
    }
    if (outlet) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (L::cx[k] != -1) continue;
        int vx = x, vy = y + L::cy[k], vz = z + L::cz[k];
        if (classify(g, vx, vy, vz) != NB_CELL) continue;
        const double cu = L::cx[k] * ux + L::cy[k] * uy + L::cz[k] * uz;
        const double dcu = L::cx[k] * dux + L::cy[k] * duy + L::cz[k] * duz;
        const int64_t o = k * g.plane + cell_of(g, vx, vy, vz);
        A[o] = L::w[k] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        At[o] = L::w[k] * (3.0 * dcu + 9.0 * cu * dcu - 1.5 * duu);
      }
    }
  }
}

template <int Q, bool ODD>
__global__ __launch_bounds__(256) void k_tangent(const Geo g, const Coll c, double* __restrict__ A,
                                                 double* __restrict__ At, const double* __restrict__ dpor,
                                                 const double* __restrict__ v, double* __restrict__ ghost,
                                                 double* __restrict__ ghostt) {
  SWEEP_PROLOGUE_RUNS((runs_remap<Q, double, ODD, 0>()))  // the order of an FP64 plain step
  if (!valid) return;
  tangent_cell<Q, ODD>(g, c, A, At, dpor, v, ghost, ghostt, x, y, z);
}

// J(t) and dJ(t)/dd . v over the objective region: dJ/df . fdot from the
// coefficients a0 + a1.xi + a2:xi xi (J_MEA: its constant source) plus
// dJ/dd v.  Block partials: J at partials[b], the tangent at partials[nb + b].
template <int Q>
__global__ __launch_bounds__(256) void k_tangent_objective(const Geo g, const ObjBox ob,
                                                           const double* __restrict__ A,
                                                           const double* __restrict__ At,
                                                           const double* __restrict__ ghost,
                                                           const double* __restrict__ ghostt, int parity,
                                                           const double* __restrict__ dpor,
                                                           const double* __restrict__ v,
                                                           double* __restrict__ partials) {
  using C = Coef<Q>;
  __shared__ double lds[4];
  CELL_PROLOGUE
  double vj = 0.0, vt = 0.0;
  int64_t r;
  if (valid && region_index<Q>(ob, x, y, z, r)) {
    double s[Q], t[Q];
    load_state<Q, double, double>(g, A, ghost, parity, x, y, z, cell, s);
    load_state<Q, double, double>(g, At, ghostt, parity, x, y, z, cell, t);
    double terms[C::N];
    if (ob.kind == OBJ_MEA) {
      mea_terms<Q>(g, ob, x, y, z, r, s, terms);
#pragma unroll
      for (int k = 0; k < Q; ++k) vt += mea_g<Q>(g, ob, x, y, z, r, k) * t[k];
    } else {
      double dr, jx, jy, jz, P[6];
      cell_moments<Q, double>(s, dr, jx, jy, jz);
      neq_flux<Q, double>(s, dr, jx, jy, jz, 1.0 / (1.0 + dr), P);
      objective_terms<Q>(ob, dpor[cell], dr, jx, jy, jz, P, terms);
#pragma unroll
      for (int k = 0; k < Q; ++k) vt += quad_eval<Q, double>(terms + C::A0, k) * t[k];
      vt += terms[C::DJDD] * v[cell];
    }
    vj = terms[C::J];
  }
  const double a = block_sum256(vj, lds);
  const double b = block_sum256(vt, lds);
  if (threadIdx.x + blockDim.x * threadIdx.y == 0) {
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    partials[linear_block()] = a;
    partials[nb + linear_block()] = b;
  }
}

// Objective terms of one window sample over the region only (grid over the
// region box), from the canonical pre-collision state: the same values and
// arithmetic as the fused window step, for regions much smaller than the
// lattice (a drag plane, a surface box).  Launched before the step.
template <int Q, typename S, bool MEA>
__global__ __launch_bounds__(256) void k_window_region(const Geo g, const ObjBox ob, const S* __restrict__ A,
                                                       const S* __restrict__ ghost, int parity,
                                                       const typename Prec<S>::Dd* __restrict__ dpor,
                                                       double* __restrict__ acc_obj) {
  using T = typename Prec<S>::T;
  // One lane per region cell, in region order (a 1-cell-thick drag plane
  // fills every lane; a 2D grid of lattice tiles over it left one lane in 128
  // active).
  const uint32_t rn0 = (uint32_t)ob.rn[0], rn1 = (uint32_t)ob.rn[1];
  const uint32_t ri = blockIdx.x * blockDim.x + threadIdx.x;
  if (!ob.active || ri >= rn0 * rn1 * (uint32_t)ob.rn[2]) return;
  const uint32_t q = ri / rn0;
  const int x = ob.lo[0] + (int)(ri - q * rn0), y = ob.lo[1] + (int)(q % rn1), z = ob.lo[2] + (int)(q / rn1);
  int64_t r;
  if (x >= g.nx || y >= g.ny || z >= g.nz || !region_index<Q>(ob, x, y, z, r)) return;
  const int64_t cell = cell_of(g, x, y, z);
  T s[Q];
  load_state<Q, S, T>(g, A, ghost, parity, x, y, z, cell, s);
  double sd[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) sd[k] = (double)s[k];
  double terms[Coef<Q>::N];
  if constexpr (MEA) {
    mea_terms<Q>(g, ob, x, y, z, r, sd, terms);
  } else {
    double dr, ax, ay, az, P[6];
    cell_moments<Q, double>(sd, dr, ax, ay, az);
    neq_flux<Q, double>(sd, dr, ax, ay, az, 1.0 / (1.0 + dr), P);
    objective_terms<Q>(ob, (double)dpor[cell], dr, ax, ay, az, P, terms);
  }
  accumulate_terms<Coef<Q>::N>(acc_obj, ob.rplane, r, terms);
}

// The same objective terms from the copy of the region cells' pre-collision
// state and porosity that the window sweep wrote (moment-form objectives):
// one lane per region cell reading its own record, instead of one cache line
// per population and cell of the lattice.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_window_region_copy(const ObjBox ob, const T* __restrict__ rc,
                                                            double* __restrict__ acc_obj) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!ob.active || r >= (int64_t)ob.rn[0] * ob.rn[1] * ob.rn[2]) return;
  const T* rec = rc + r * region_copy_stride(Q, (int)sizeof(T));
  double sd[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) sd[k] = (double)rec[k];
  double dr, ax, ay, az, P[6], terms[Coef<Q>::N];
  cell_moments<Q, double>(sd, dr, ax, ay, az);
  neq_flux<Q, double>(sd, dr, ax, ay, az, 1.0 / (1.0 + dr), P);
  objective_terms<Q>(ob, (double)rec[Q], dr, ax, ay, az, P, terms);
  accumulate_terms<Coef<Q>::N>(acc_obj, ob.rplane, r, terms);
}

// Completes the grouped window accumulation when a run ends inside a group:
// adds the first `count` pending slots, in slot (step) order, to the FP64
// sums (the additions the group's last step would have made first).
template <int Q>
__global__ __launch_bounds__(256) void k_window_flush(const Geo g, const Acc acc, const int count) {
  using L = Lat<Q>;
  CELL_PROLOGUE
  if (!valid || (inout && x == 0)) return;  // the pinned inlet is not part of the window
  for (int j = 0; j < count; ++j) {
    const float* pv = acc.pend + j * acc.pslot;
    acc.rho[cell] = acc.rho[cell] + (double)pv[cell];
#pragma unroll
    for (int a = 0; a < L::D; ++a)
      acc.j[a * g.plane + cell] = acc.j[a * g.plane + cell] + (double)pv[(1 + a) * g.plane + cell];
    if (acc.tau) acc.tau[cell] = acc.tau[cell] + (double)pv[(L::D + 1) * g.plane + cell];
    if (acc.f) {
#pragma unroll
      for (int k = 0; k < Q; ++k)
        acc.f[k * g.plane + cell] = acc.f[k * g.plane + cell] + (double)pv[(L::D + 2 + k) * g.plane + cell];
    }
  }
}

// Packed launch: one workgroup grid covering several lattices of one stencil
// and precision (member m owns blocks [first_block, first_block + tiles)).
// Each member runs exactly the per-cell code of k_primal, so its result does
// not depend on which other lattices share the launch.
struct PackedPrimal {
  Geo g;
  Coll c;
  ObjBox ob;
  Acc acc;
  void* A;
  const void* dpor;
  void* ghost;
  int parity0;     // AA parity when the table was built
  int accumulate;  // window accumulation on
  int first_block, tiles_x, tiles_y, pad_;
};

__device__ __forceinline__ int packed_member(const int* __restrict__ first, int nm, int b) {
  int m = 0;
  while (m + 1 < nm && first[m + 1] <= b) ++m;
  return m;
}

template <int Q, typename S, bool HRR>
__global__ __launch_bounds__(256) void k_primal_packed(const PackedPrimal* __restrict__ tab,
                                                       const int* __restrict__ first, int nm, int step) {
  using Dd = typename Prec<S>::Dd;
  const int b = sweep_tile((int)blockIdx.x, (int)gridDim.x);
  const PackedPrimal& P = tab[packed_member(first, nm, b)];
  const int lb = b - P.first_block;
  const int tx = lb % P.tiles_x, r = lb / P.tiles_x;
  const int ty = r % P.tiles_y, z = r / P.tiles_y;
  const int x = tx * BX + threadIdx.x, y = ty * BY + threadIdx.y;
  if (x >= P.g.nx || y >= P.g.ny) return;
  const int64_t c0 = wave_uniform64(cell_of(P.g, tx * BX, ty * BY, z));
  const uint32_t lo = lane_offset(threadIdx.x + (uint32_t)P.g.nx * threadIdx.y);
  S* A = (S*)P.A;
  const Dd* dp = (const Dd*)P.dpor;
  S* gh = (S*)P.ghost;
  const int mode = P.accumulate ? (P.ob.kind == OBJ_MEA ? 2 : 1) : 0;
  if ((P.parity0 + step) & 1) {
    if (mode == 1)
      primal_cell<Q, S, true, 1, HRR>(P.g, P.c, P.ob, A, dp, gh, P.acc, x, y, z, c0, lo);
    else if (mode == 2)
      primal_cell<Q, S, true, 2, HRR>(P.g, P.c, P.ob, A, dp, gh, P.acc, x, y, z, c0, lo);
    else
      primal_cell<Q, S, true, 0, HRR>(P.g, P.c, P.ob, A, dp, gh, P.acc, x, y, z, c0, lo);
  } else {
    if (mode == 1)
      primal_cell<Q, S, false, 1, HRR>(P.g, P.c, P.ob, A, dp, gh, P.acc, x, y, z, c0, lo);
    else if (mode == 2)
      primal_cell<Q, S, false, 2, HRR>(P.g, P.c, P.ob, A, dp, gh, P.acc, x, y, z, c0, lo);
    else
      primal_cell<Q, S, false, 0, HRR>(P.g, P.c, P.ob, A, dp, gh, P.acc, x, y, z, c0, lo);
  }
}

// =========================================================================
// geometry, initial state, population exchange (rows a1, a2)
// =========================================================================

template <typename Dd>
__global__ __launch_bounds__(256) void k_cylinder(const Geo g, Dd* __restrict__ dpor, double xc,
                                                  double yc, double D, const double* __restrict__ noise,
                                                  int mode, double box_half, double d_solid) {
  CELL_PROLOGUE
  if (!valid) return;
  const double R = 0.5 * D;
  const double dx = x - xc, dy = y - yc;
  const double r = sqrt(dx * dx + dy * dy);
  double chi;
  if (r <= R - 1.0)
    chi = 1.0;
  else if (r >= R + 1.0)
    chi = 0.0;
  else
    chi = 0.5 * (1.0 + cos(M_PI * (r - R + 1.0) * 0.5));
  double d = 1.0 - chi;
  if (noise != nullptr && mode == 1 && chi > 0.0 && chi < 1.0) {
    d = fmin(1.0, fmax(0.0, d + noise[cell]));
  } else if (noise != nullptr && mode == 2 && fabs(dx) <= box_half && fabs(dy) <= box_half) {
    d = 1.0 - fmin(1.0, fmax(0.0, chi + noise[cell]));
  }
  // permeable cylinder: the porosity deficit scales with 1 - d_solid
  if (d_solid != 0.0) d = 1.0 - (1.0 - d) * (1.0 - d_solid);
  dpor[cell] = (Dd)d;
}

// J_MEA surface nodes of the objective region: d < 1/2 with a lattice
// neighbour d >= 1/2, one cell away from the region's faces on axes the
// region does not span completely (the functional reads every neighbour of
// a surface node, which must lie in the region as well).
template <int Q, typename Dd>
__global__ __launch_bounds__(256) void k_mea_flags(const Geo g, const ObjBox ob, const Dd* __restrict__ dpor,
                                                   unsigned char* __restrict__ flag) {
  using L = Lat<Q>;
  CELL_PROLOGUE
  if (!valid) return;
  int64_t r;
  if (!region_index<Q>(ob, x, y, z, r)) return;
  const int n3[3] = {g.nx, g.ny, g.nz}, p[3] = {x, y, z};
  bool inner = true;
  for (int a = 0; a < 3; ++a) {
    const int lo = ob.lo[a], hi = ob.lo[a] + ob.rn[a] - 1;
    if (!(lo == 0 && hi == n3[a] - 1) && (p[a] <= lo || p[a] >= hi)) inner = false;
  }
  unsigned char s = 0;
  if (inner && (double)dpor[cell] < 0.5) {
    for (int k = 1; k < Q; ++k) {
      int tx = x + L::cx[k], ty = y + L::cy[k], tz = z + L::cz[k];
      if (classify(g, tx, ty, tz) == NB_CELL && (double)dpor[cell_of(g, tx, ty, tz)] >= 0.5) s = 1;
    }
  }
  flag[r] = s;
}

// g_k(y) = (xi_k,x / A)(s(y) + s(y - xi_k)) from the surface flags.
template <int Q>
__global__ __launch_bounds__(256) void k_mea_source(const Geo g, const ObjBox ob,
                                                    const unsigned char* __restrict__ flag,
                                                    double* __restrict__ mea) {
  using L = Lat<Q>;
  CELL_PROLOGUE
  if (!valid) return;
  int64_t r;
  if (!region_index<Q>(ob, x, y, z, r)) return;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double s = (double)flag[r];
    int sx = x - L::cx[k], sy = y - L::cy[k], sz = z - L::cz[k];
    int64_t rr;
    if (classify(g, sx, sy, sz) == NB_CELL && region_index<Q>(ob, sx, sy, sz, rr)) s += (double)flag[rr];
    mea[k * ob.rplane + r] = (double)L::cx[k] / ob.u0 * s;
  }
}

template <typename Dd>
__global__ __launch_bounds__(256) void k_set_porosity(const Geo g, Dd* __restrict__ dpor,
                                                      const double* __restrict__ d, int* bad) {
  CELL_PROLOGUE
  if (!valid) return;
  const double v = d[cell];
  if (!(v >= 0.0 && v <= 1.0)) atomicOr(bad, 1);
  dpor[cell] = (Dd)v;
}

template <int Q, typename S>
__global__ __launch_bounds__(256) void k_init(const Geo g, S* __restrict__ A,
                                              const typename Prec<S>::Dd* __restrict__ dpor,
                                              double rho0, const double* __restrict__ u, int64_t n) {
  using L = Lat<Q>;
  CELL_PROLOGUE
  if (!valid) return;
  double s[Q];
  if (inout && x == 0) {
    inlet_state<Q, double>(g, y, s);
  } else {
    double v[3] = {0.0, 0.0, 0.0};
    if (u != nullptr) {
      v[0] = u[cell];
      v[1] = u[n + cell];
      v[2] = u[2 * n + cell];
    } else if (inout) {
      v[0] = inlet_velocity<double>(g, y);
    }
    const double d = (double)dpor[cell];
    for (int a = 0; a < 3; ++a) v[a] *= d;
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const double cu = L::cx[k] * v[0] + L::cy[k] * v[1] + L::cz[k] * v[2];
      s[k] = L::w[k] * ((rho0 - 1.0) + rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * vv));
    }
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) A[k * g.plane + cell] = to_store<S>(s[k]);
}

template <int Q, typename S>
__global__ __launch_bounds__(256) void k_gather(const Geo g, const S* __restrict__ A,
                                                const S* __restrict__ ghost, int parity,
                                                double* __restrict__ out, int64_t n) {
  using L = Lat<Q>;
  using T = typename Prec<S>::T;
  CELL_PROLOGUE
  if (!valid) return;
  T s[Q];
  if (inout && x == 0)
    inlet_state<Q, T>(g, y, s);
  else
    load_state<Q, S, T>(g, A, ghost, parity, x, y, z, cell, s);
#pragma unroll
  for (int k = 0; k < Q; ++k) out[k * n + cell] = (double)s[k] + L::w[k];
}

template <int Q, typename S>
__global__ __launch_bounds__(256) void k_scatter(const Geo g, S* __restrict__ A,
                                                 const double* __restrict__ in, int64_t n) {
  using L = Lat<Q>;
  CELL_PROLOGUE
  if (!valid) return;
#pragma unroll
  for (int k = 0; k < Q; ++k) A[k * g.plane + cell] = to_store<S>(in[k * n + cell] - L::w[k]);
}

template <int Q, typename S>
__global__ __launch_bounds__(256) void k_moments(const Geo g, const S* __restrict__ A,
                                                 const S* __restrict__ ghost, int parity,
                                                 double* __restrict__ rho, double* __restrict__ u,
                                                 int64_t n) {
  using T = typename Prec<S>::T;
  CELL_PROLOGUE
  if (!valid) return;
  T s[Q];
  if (inout && x == 0)
    inlet_state<Q, T>(g, y, s);
  else
    load_state<Q, S, T>(g, A, ghost, parity, x, y, z, cell, s);
  double sd[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) sd[k] = (double)s[k];
  double dr, jx, jy, jz;
  cell_moments<Q, double>(sd, dr, jx, jy, jz);
  const double r = 1.0 + dr;
  if (rho) rho[cell] = r;
  if (u) {
    u[cell] = jx / r;
    u[n + cell] = jy / r;
    u[2 * n + cell] = jz / r;
  }
}

// field: 2 mean rho, 3 mean u, 5 mean tau
template <int Q>
__global__ __launch_bounds__(256) void k_mean_fields(const Geo g, int field, const double* acc_rho,
                                                     const double* acc_j, const double* acc_tau,
                                                     double inv, double* __restrict__ out, int64_t n) {
  CELL_PROLOGUE
  if (!valid) return;
  const double r = 1.0 + acc_rho[cell] * inv;
  if (field == 2) {
    out[cell] = r;
  } else if (field == 3) {
    out[cell] = acc_j[cell] * inv / r;
    out[n + cell] = acc_j[g.plane + cell] * inv / r;
    out[2 * n + cell] = (Lat<Q>::D == 3) ? acc_j[2 * g.plane + cell] * inv / r : 0.0;
  } else {
    out[cell] = acc_tau ? acc_tau[cell] * inv : 0.0;
  }
}

// =========================================================================
// reductions: steady check, objective
// =========================================================================

template <int Q, typename S>
__global__ __launch_bounds__(256) void k_steady_check(const Geo g, const S* __restrict__ A,
                                                      const S* __restrict__ ghost, int parity,
                                                      double* __restrict__ usnap, int first,
                                                      double* __restrict__ partials) {
  using T = typename Prec<S>::T;
  __shared__ double lds[4];
  CELL_PROLOGUE
  double dmax = 0.0, umax = 0.0;
  bool bad = false;
  if (valid && !(inout && x == 0)) {
    T s[Q];
    load_state<Q, S, T>(g, A, ghost, parity, x, y, z, cell, s);
    double sd[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) sd[k] = (double)s[k];
    double dr, jx, jy, jz;
    cell_moments<Q, double>(sd, dr, jx, jy, jz);
    const double r = 1.0 + dr;
    const double u[3] = {jx / r, jy / r, jz / r};
    for (int a = 0; a < Lat<Q>::D; ++a) {
      if (!isfinite(u[a])) bad = true;
      if (!first) dmax = fmax(dmax, fabs(u[a] - usnap[a * g.plane + cell]));
      umax = fmax(umax, fabs(u[a]));
      usnap[a * g.plane + cell] = u[a];
    }
    if (!isfinite(r)) bad = true;
  }
  if (bad || first) dmax = INFINITY;
  const double a = block_max256(dmax, lds);
  const double b = block_max256(umax, lds);
  const int t = threadIdx.x + blockDim.x * threadIdx.y;
  if (t == 0) {
    partials[2 * linear_block()] = a;
    partials[2 * linear_block() + 1] = b;
  }
}

// which = 0: J of the current state; 1: window-mean J (from accumulated terms)
template <int Q, typename S>
__global__ __launch_bounds__(256) void k_objective(const Geo g, const ObjBox ob, const S* __restrict__ A,
                                                   const S* __restrict__ ghost, int parity,
                                                   const typename Prec<S>::Dd* __restrict__ dpor,
                                                   int which, const double* __restrict__ acc_obj,
                                                   double inv, double* __restrict__ partials) {
  using T = typename Prec<S>::T;
  __shared__ double lds[4];
  CELL_PROLOGUE
  double v = 0.0;
  int64_t r;
  if (valid && region_index<Q>(ob, x, y, z, r)) {
    if (which == 1) {
      v = acc_obj[Coef<Q>::J * ob.rplane + r] * inv;
    } else {
      T s[Q];
      load_state<Q, S, T>(g, A, ghost, parity, x, y, z, cell, s);
      double sd[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) sd[k] = (double)s[k];
      double terms[Coef<Q>::N];
      if (ob.kind == OBJ_MEA) {
        mea_terms<Q>(g, ob, x, y, z, r, sd, terms);
      } else {
        double dr, jx, jy, jz, P[6];
        cell_moments<Q, double>(sd, dr, jx, jy, jz);
        neq_flux<Q, double>(sd, dr, jx, jy, jz, 1.0 / (1.0 + dr), P);
        objective_terms<Q>(ob, (double)dpor[cell], dr, jx, jy, jz, P, terms);
      }
      v = terms[Coef<Q>::J];
    }
  }
  const double sum = block_sum256(v, lds);
  if (threadIdx.x + blockDim.x * threadIdx.y == 0) partials[linear_block()] = sum;
}

__global__ __launch_bounds__(256) void k_finalize_sum(const double* __restrict__ partials, int n,
                                                      double* __restrict__ out) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += partials[i];
  const double s = block_sum256(v, lds);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ __launch_bounds__(256) void k_finalize_max2(const double* __restrict__ partials, int n,
                                                       double* __restrict__ out) {
  __shared__ double lds[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double pa = partials[2 * i], pb = partials[2 * i + 1];
    a = (pa != pa) ? INFINITY : fmax(a, pa);
    b = (pb != pb) ? INFINITY : fmax(b, pb);
  }
  const double ra = block_max256(a, lds);
  const double rb = block_max256(b, lds);
  if (threadIdx.x == 0) {
    out[0] = ra;
    out[1] = rb;
  }
}

// =========================================================================
// adjoint preparation (row a7): freeze the Jacobian data at the steady or
// window-mean state (Eqs. adjoint_steady / adjoint_unsteady)
// =========================================================================

struct PrepIn {
  const double* acc_rho;
  const double* acc_j;
  const double* acc_f;
  const double* acc_tau;
  const double* acc_obj;
  double inv;
  int source;      // 0 steady (current state), 1 window mean
  int smag, turb;  // closure present, 0 frozen / 1 differentiated
  int hrr;         // HRRLBM collision: its own frozen-coefficient layout
  double tau0, tau_adj, kS;
};

template <int Q, typename S, typename SA>
__global__ __launch_bounds__(256) void k_adjoint_prep(const Geo g, const ObjBox ob, const PrepIn pin,
                                                      const S* __restrict__ A,
                                                      const S* __restrict__ ghost, int parity,
                                                      const typename Prec<S>::Dd* __restrict__ dpor,
                                                      SA* __restrict__ prep, double* __restrict__ src,
                                                      double* __restrict__ gdat,
                                                      double* __restrict__ oprep) {
  using L = Lat<Q>;
  using T = typename Prec<S>::T;
  constexpr int D = L::D;
  CELL_PROLOGUE
  if (!valid || (inout && x == 0)) return;
  double fs[Q];  // shifted populations f - w of the frozen state
  double drho, jx, jy, jz;
  const bool need_f = (pin.source == 0) || (pin.smag && pin.turb == 1) || pin.hrr;
  if (pin.source == 1) {
    drho = pin.acc_rho[cell] * pin.inv;
    jx = pin.acc_j[cell] * pin.inv;
    jy = pin.acc_j[g.plane + cell] * pin.inv;
    jz = (D == 3) ? pin.acc_j[2 * g.plane + cell] * pin.inv : 0.0;
    if (need_f) {
#pragma unroll
      for (int k = 0; k < Q; ++k) fs[k] = pin.acc_f[k * g.plane + cell] * pin.inv;
    }
  } else {
    T s[Q];
    load_state<Q, S, T>(g, A, ghost, parity, x, y, z, cell, s);
#pragma unroll
    for (int k = 0; k < Q; ++k) fs[k] = (double)s[k];
    cell_moments<Q, double>(fs, drho, jx, jy, jz);
  }
  const double rho = 1.0 + drho, ir = 1.0 / rho;
  const double u[3] = {jx * ir, jy * ir, jz * ir};
  const double d = (double)dpor[cell];
  const double ut[3] = {d * u[0], d * u[1], d * u[2]};
  const double ta = pin.tau_adj;
  double P[6] = {0, 0, 0, 0, 0, 0};
  if (pin.smag && need_f) neq_flux<Q, double>(fs, drho, jx, jy, jz, ir, P);
  double tau_used;
  if (!pin.smag) {
    tau_used = ta;
  } else if (pin.turb == 1) {
    tau_used = 0.5 * (ta + sqrt(ta * ta + pin.kS * sqrt(frob2(P))));
  } else {
    double tmean;
    if (pin.source == 1)
      tmean = pin.acc_tau[cell] * pin.inv;
    else
      tmean = 0.5 * (pin.tau0 + sqrt(pin.tau0 * pin.tau0 + pin.kS * sqrt(frob2(P))));
    tau_used = ta + (tmean - pin.tau0);
  }
  const double omega = 1.0 / tau_used;

  if (pin.hrr) {
    // rho, j, d, omega, a2 = sum xi xi (f - w) - drho/3 I - rho u~u~ and, with
    // the differentiated closure, (1/tau^2) dtau/dPi = cc Pi
    prep[cell] = (SA)rho;
    const double jv[3] = {jx, jy, jz};
    for (int a = 0; a < D; ++a) prep[(1 + a) * g.plane + cell] = (SA)jv[a];
    prep[(D + 1) * g.plane + cell] = (SA)d;
    prep[(D + 2) * g.plane + cell] = (SA)omega;
    double S6[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      S6[0] += L::cx[k] * L::cx[k] * fs[k];
      S6[1] += L::cy[k] * L::cy[k] * fs[k];
      S6[2] += L::cz[k] * L::cz[k] * fs[k];
      S6[3] += L::cx[k] * L::cy[k] * fs[k];
      S6[4] += L::cx[k] * L::cz[k] * fs[k];
      S6[5] += L::cy[k] * L::cz[k] * fs[k];
    }
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int m6 = 0; m6 < 6; ++m6) {
      const int m = sym_index<Q>(m6);
      if (m < 0) continue;
      const double a2 = S6[m6] - (m6 < 3 ? drho / 3.0 : 0.0) - rho * ut[ia[m6]] * ut[ib[m6]];
      prep[(D + 3 + m) * g.plane + cell] = (SA)a2;
    }
    if (pin.smag && pin.turb == 1) {
      const double Pn = sqrt(frob2(P));
      double cc = 0.0;
      if (Pn > 0.0) cc = pin.kS / (4.0 * sqrt(ta * ta + pin.kS * Pn) * Pn * tau_used * tau_used);
      for (int m6 = 0; m6 < 6; ++m6) {
        const int m = sym_index<Q>(m6);
        if (m >= 0) prep[(D + 3 + L::NSYM + m) * g.plane + cell] = (SA)(cc * P[m6]);
      }
    }
  } else {
  for (int a = 0; a < D; ++a) prep[a * g.plane + cell] = (SA)ut[a];
  prep[D * g.plane + cell] = (SA)d;
  prep[(D + 1) * g.plane + cell] = (SA)omega;
  if (pin.smag && pin.turb == 1) {
    // f^neq_j = f_j - f^eq_j(rho, d u) and the coefficients of
    // (1/tau^2) dtau/df_i = b0 + b1.xi_i + b2:xi_i xi_i.
    const double tt = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const double cu = L::cx[k] * ut[0] + L::cy[k] * ut[1] + L::cz[k] * ut[2];
      const double feqs = L::w[k] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * tt));
      prep[(D + 2 + k) * g.plane + cell] = (SA)(fs[k] - feqs);
    }
    const double Pn = sqrt(frob2(P));
    double cc = 0.0;
    if (Pn > 0.0) cc = pin.kS / (4.0 * sqrt(ta * ta + pin.kS * Pn) * Pn * tau_used * tau_used);
    const double Pm[3][3] = {{P[0], P[3], P[4]}, {P[3], P[1], P[5]}, {P[4], P[5], P[2]}};
    double Pu[3], uPu = 0.0;
    for (int a = 0; a < 3; ++a) {
      Pu[a] = Pm[a][0] * u[0] + Pm[a][1] * u[1] + Pm[a][2] * u[2];
      uPu += u[a] * Pu[a];
    }
    const double tr = P[0] + P[1] + P[2];
    const int64_t bo = (D + 2 + Q);
    prep[bo * g.plane + cell] = (SA)(cc * (uPu - tr / 3.0));
    for (int a = 0; a < D; ++a) prep[(bo + 1 + a) * g.plane + cell] = (SA)(-2.0 * cc * Pu[a]);
    for (int m6 = 0; m6 < 6; ++m6) {
      const int m = sym_index<Q>(m6);
      if (m >= 0) prep[(bo + 1 + D + m) * g.plane + cell] = (SA)(cc * P[m6]);
    }
  }
  }
  gdat[cell] = rho;
  for (int a = 0; a < D; ++a) gdat[(1 + a) * g.plane + cell] = u[a];
  gdat[(D + 1) * g.plane + cell] = omega;
  if (inout && x == g.nx - 1) {
    const int64_t o = y + (int64_t)g.ny * z;
    oprep[o] = rho;
    for (int a = 0; a < D; ++a) oprep[(1 + a) * g.gplane + o] = u[a];
  }
  int64_t r;
  if (region_index<Q>(ob, x, y, z, r)) {
    if (pin.source == 1) {
#pragma unroll
      for (int m = 0; m < Coef<Q>::N; ++m) src[m * ob.rplane + r] = pin.acc_obj[m * ob.rplane + r] * pin.inv;
    } else {
      double terms[Coef<Q>::N];
      if (ob.kind == OBJ_MEA) {
        mea_terms<Q>(g, ob, x, y, z, r, fs, terms);
      } else {
        double Pq[6];
        neq_flux<Q, double>(fs, drho, jx, jy, jz, ir, Pq);
        objective_terms<Q>(ob, d, drho, jx, jy, jz, Pq, terms);
      }
#pragma unroll
      for (int m = 0; m < Coef<Q>::N; ++m) src[m * ob.rplane + r] = terms[m];
    }
  }
}

// =========================================================================
// adjoint sweep (row a8): lambda_i = sum_j dC_j/df_i phi_j - dJ/df_i at each
// cell (closed form in the weighted adjoint moments), then phi = S^T lambda
// through the relabelled AA propagation.
// =========================================================================

struct AdjC {
  int les;       // per-cell omega
  int diff;      // differentiated closure term
  double omega0;
};

// Adjoint values of a cell as read by an even step / the gradient: canonical
// slots, with the outlet's outgoing directions zero unless bounce-back wrote them.
template <int Q, typename SA>
__device__ __forceinline__ void adjoint_zero_outlet(const Geo& g, int x, int y, int z, SA (&ph)[Q]) {
  using L = Lat<Q>;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (L::cx[k] != -1) continue;
    int sx = x - L::cx[k], sy = y - L::cy[k], sz = z - L::cz[k];
    if (classify(g, sx, sy, sz) != NB_BOUNCE) ph[k] = (SA)0;
  }
}
template <int Q, typename SA>
__device__ __forceinline__ void adjoint_read_canonical(const Geo& g, const SA* __restrict__ A, int x,
                                                       int y, int z, int64_t cell, bool outlet,
                                                       SA (&ph)[Q]) {
  using L = Lat<Q>;
#pragma unroll
  for (int k = 0; k < Q; ++k) ph[k] = ld_stream(&A[k * g.plane + cell]);
  if (outlet) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (L::cx[k] != -1) continue;
      int sx = x - L::cx[k], sy = y - L::cy[k], sz = z - L::cz[k];
      if (classify(g, sx, sy, sz) != NB_BOUNCE) ph[k] = (SA)0;
    }
  }
}

// ---- adjoint of the HRRLBM collision ---------------------------------------
// The HRR collision depends on f only through rho, j and S = sum xi xi f, so
// lambda_i = sum_j phi_j dC_j/df_i = G_rho + xi_i.G_j + xi_i xi_i : G_S with
// G the gradient of Phi = sum_j phi_j C_j(rho, j, S) at the frozen state.
// In the weighted Hermite moments of phi (m0, m1, M2 = sum w phi H2,
// M3_t = sum w phi H_t):
//   Phi = A + (1 - omega) B,
//   A = rho m0 + 3 d j.m1 + 4.5 rho u~.M2.u~ + 13.5 rho sum_t u~_a^2 u~_b M3_t,
//   B = 3 (1 - d) j.m1 + 4.5 a2:M2 + 13.5 sum_t a3_t M3_t,
// differentiated by hand through u~ = d j / rho, a2 = S - rho/3 I - rho u~u~
// and a3; the differentiated closure adds B (1/tau^2) dtau/dPi : dPi.

// Hermite moments of the canonical adjoint phi_i = ph[opp(i)] (xi_opp(k) = -xi_k).
template <int Q, typename T>
__device__ __forceinline__ void hrr_phi_moments(const T (&ph)[Q], T& m0, T (&m1)[3], T (&M2)[3][3],
                                                T (&M3)[H3Types<Q>::N]) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  m0 = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m1[a] = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) M2[a][b] = 0;
  }
#pragma unroll
  for (int t = 0; t < H3Types<Q>::N; ++t) M3[t] = 0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const T wp = (T)L::w[k] * ph[k];
    m0 += wp;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (lat_c<Q>(k, a) != 0) m1[a] -= (T)lat_c<Q>(k, a) * wp;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const T h = (T)(lat_c<Q>(k, a) * lat_c<Q>(k, b)) - (a == b ? (T)(1.0 / 3.0) : (T)0);
        if (h != (T)0) M2[a][b] += h * wp;
      }
    }
#pragma unroll
    for (int t = 0; t < H3Types<Q>::N; ++t) {
      const T h = (T)h3<Q>(k, t);
      if (h != (T)0) M3[t] -= h * wp;  // H_t is odd in xi
    }
  }
}

template <int Q, typename T, bool NT = false>
__device__ __forceinline__ void sym_read(const T* __restrict__ p, int64_t plane, int64_t cell, int base,
                                         T (&M)[3][3]) {
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[a][b] = 0;
#pragma unroll
  for (int m6 = 0; m6 < 6; ++m6) {
    const int m = sym_index<Q>(m6);
    if (m < 0) continue;
    const T v = ld_stream<NT>(&p[(base + m) * plane + cell]);
    M[ia[m6]][ib[m6]] = v;
    M[ib[m6]][ia[m6]] = v;
  }
}

// NT: streaming hints on the frozen per-cell data (lattices above the
// Infinity Cache, both adjoint steps).
template <int Q, typename T, bool NT = false>
__device__ __forceinline__ void hrr_adjoint(const T (&ph)[Q], const T* __restrict__ prep, int64_t plane,
                                            int64_t cell, bool diff, T (&lam)[Q]) {
  using L = Lat<Q>;
  using H = H3Types<Q>;
  constexpr int D = L::D;
  T m0, m1[3], M2[3][3], M3[H::N];
  hrr_phi_moments<Q, T>(ph, m0, m1, M2, M3);
  const T rho = ld_stream<NT>(&prep[cell]);
  T j[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) j[a] = ld_stream<NT>(&prep[(1 + a) * plane + cell]);
  const T d = ld_stream<NT>(&prep[(D + 1) * plane + cell]);
  const T omega = ld_stream<NT>(&prep[(D + 2) * plane + cell]);
  T a2[3][3];
  sym_read<Q, T, NT>(prep, plane, cell, D + 3, a2);
  const T ir = (T)1 / rho;
  const T u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
  const T ut[3] = {d * u[0], d * u[1], d * u[2]};
  T M2ut[3], jm1 = 0, utM2ut = 0, trM2 = 0, a2M2 = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    M2ut[a] = M2[a][0] * ut[0] + M2[a][1] * ut[1] + M2[a][2] * ut[2];
    jm1 += j[a] * m1[a];
    trM2 += M2[a][a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    utM2ut += ut[a] * M2ut[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) a2M2 += a2[a][b] * M2[a][b];
  }
  const T om1 = (T)1 - omega;
  // A part
  T Gr = m0 - (T)4.5 * utM2ut;
  T Gj[3], GS[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Gj[a] = (T)3 * d * m1[a] + (T)9 * d * M2ut[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) GS[a][b] = 0;
  }
  // B part (times 1 - omega) and B itself
  T B = (T)3 * ((T)1 - d) * jm1 + (T)4.5 * a2M2;
  T GrB = (T)4.5 * (utM2ut - trM2 / (T)3);
  T GjB[3], GSB[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    GjB[a] = (T)3 * ((T)1 - d) * m1[a] - (T)9 * d * M2ut[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) GSB[a][b] = (T)4.5 * M2[a][b];
  }
#pragma unroll
  for (int t = 0; t < H::N; ++t) {
    const int a = H::a[t], b = H::b[t];
    const T m3 = M3[t];
    const T a3 = (T)2 * ut[a] * a2[a][b] + ut[b] * a2[a][a];
    Gr -= (T)27 * ut[a] * ut[a] * ut[b] * m3;
    Gj[a] += (T)27 * d * ut[a] * ut[b] * m3;
    Gj[b] += (T)13.5 * d * ut[a] * ut[a] * m3;
    B += (T)13.5 * a3 * m3;
    GrB += (T)13.5 * m3 * (-a3 * ir + (T)3 * ut[a] * ut[a] * ut[b] - ut[b] / (T)3);
    GjB[a] += (T)13.5 * m3 * ((T)2 * d * ir * a2[a][b] - (T)4 * d * ut[a] * ut[b]);
    GjB[b] += (T)13.5 * m3 * (d * ir * a2[a][a] - (T)2 * d * ut[a] * ut[a]);
    GSB[a][b] += (T)27 * ut[a] * m3;
    GSB[a][a] += (T)13.5 * ut[b] * m3;
  }
  Gr += om1 * GrB;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Gj[a] += om1 * GjB[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) GS[a][b] = om1 * GSB[a][b];
  }
  if (diff) {  // omega = 1/tau_eff(Pi), Pi = S - rho/3 I - j j / rho
    T q[3][3];
    sym_read<Q, T, NT>(prep, plane, cell, D + 3 + L::NSYM, q);
    T qu[3], uqu = 0, trq = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qu[a] = q[a][0] * u[0] + q[a][1] * u[1] + q[a][2] * u[2];
      trq += q[a][a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) uqu += u[a] * qu[a];
    Gr += B * (uqu - trq / (T)3);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Gj[a] -= (T)2 * B * qu[a];
#pragma unroll
      for (int b = 0; b < 3; ++b) GS[a][b] += B * q[a][b];
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    T v = Gr;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (lat_c<Q>(i, a) == 0) continue;
      v += (T)lat_c<Q>(i, a) * Gj[a];
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (lat_c<Q>(i, b) != 0) v += (T)(lat_c<Q>(i, a) * lat_c<Q>(i, b)) * GS[a][b];
    }
    lam[i] = v;
  }
}

// Sum_i phi_i dC_i/dd of the HRRLBM collision at the frozen state (gradient
// assembly): u~ = d u and a2 depend on d; the closure does not.
template <int Q>
__device__ __forceinline__ double hrr_dphi_dd(const double (&ph)[Q], const double* pr, double d) {
  using H = H3Types<Q>;
  constexpr int D = Lat<Q>::D;
  double m0, m1[3], M2[3][3], M3[H::N];
  hrr_phi_moments<Q, double>(ph, m0, m1, M2, M3);
  (void)m0;
  const double rho = pr[0];
  const double u[3] = {pr[1] / rho, pr[2] / rho, D == 3 ? pr[3] / rho : 0.0};
  const double omega = pr[D + 2];
  double a2[3][3];
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) a2[a][b] = 0.0;
  for (int m6 = 0; m6 < 6; ++m6) {
    const int m = sym_index<Q>(m6);
    if (m < 0) continue;
    a2[ia[m6]][ib[m6]] = a2[ib[m6]][ia[m6]] = pr[D + 3 + m];
  }
  double um1 = 0, uM2u = 0;
  for (int a = 0; a < 3; ++a) {
    um1 += u[a] * m1[a];
    for (int b = 0; b < 3; ++b) uM2u += u[a] * M2[a][b] * u[b];
  }
  double dA = 3.0 * rho * um1 + 9.0 * d * rho * uM2u;
  double dB = -3.0 * rho * um1 - 9.0 * d * rho * uM2u;
  for (int t = 0; t < H::N; ++t) {
    const int a = H::a[t], b = H::b[t];
    dA += 40.5 * d * d * rho * u[a] * u[a] * u[b] * M3[t];
    dB += 13.5 * M3[t] * (2.0 * u[a] * a2[a][b] + u[b] * a2[a][a] - 6.0 * d * d * rho * u[a] * u[a] * u[b]);
  }
  return dA + (1.0 - omega) * dB;
}

template <int Q, typename SA, bool ODD, bool HRR, bool MEA, bool NT = false, bool NTP = NT>
__device__ __forceinline__ void adjoint_cell(const Geo& g, const ObjBox& ob, const AdjC& ac, SA* __restrict__ A,
                                             const SA* __restrict__ prep, const double* __restrict__ src,
                                             const double* __restrict__ oprep, const SA* __restrict__ pv_in,
                                             SA* __restrict__ pv_out, const int x, const int y, const int z,
                                             const int64_t c0, const uint32_t lo) {
  using L = Lat<Q>;
  using T = SA;
  constexpr int D = L::D;
  const int64_t cell = c0 + lo;
  const bool inout = (g.bcx == BC_INOUT);
  // inlet: no dependence on the state, lambda = 0; outlet: no adjoint inflow
  // from beyond x = nx-1.  As in the primal sweep, the inlet and outlet cells
  // of rows away from walls and periodic seams share the interior path of
  // the odd step (fast lanes).
  const bool inlet = inout && x == 0, outlet = inout && (x == g.nx - 1);
  bool fast = true;
  if constexpr (ODD) {
    const bool rows = y > 0 && y < g.ny - 1 && (D == 2 || (z > 0 && z < g.nz - 1));
    fast = g.slot32 && rows && ((x > 0 && x < g.nx - 1) || inlet || outlet);
  }
  if (inlet && !fast) {  // odd step, inlet cell of a wall row
#pragma unroll
    for (int k = 0; k < Q; ++k) push<Q, SA>(g, A, x, y, z, cell, k, (SA)0);
    return;
  }
  // Frozen data of the BGK adjoint, requested before phi: the inlet and
  // outlet overrides of phi below have to wait for its loads, so a load
  // issued after them would start a second memory round trip.
  T tx = (T)0, ty = (T)0, tz = (T)0, d = (T)0, omega = (T)0;
  if constexpr (!HRR) {
    tx = ld_stream<NTP>(&at(prep, c0, lo));
    ty = ld_stream<NTP>(&at(prep, g.plane + c0, lo));
    if constexpr (D == 3) tz = ld_stream<NTP>(&at(prep, 2 * g.plane + c0, lo));
    d = ld_stream<NTP>(&at(prep, D * g.plane + c0, lo));
    // per-cell omega (LES): plane D + 1; otherwise the load repeats d's
    // (no branch between the loads) and the constant is taken
    const T om = ld_stream<NTP>(&at(prep, (ac.les ? D + 1 : D) * g.plane + c0, lo));
    omega = ac.les ? om : (T)ac.omega0;
  }
  T ph[Q];  // phihat_k = phi_opp(k)
  if (!ODD) {
#pragma unroll
    for (int k = 0; k < Q; ++k) ph[k] = ld_stream<NT>(&at(A, k * g.plane + c0, lo));
    __builtin_amdgcn_sched_barrier(0);
    if (outlet) adjoint_zero_outlet<Q, SA>(g, x, y, z, ph);
  } else if (fast) {
    // as in the primal sweep: every fast lane requests all its slots; the
    // inlet's values are replaced below, the outlet's from beyond x = nx-1 here
    const OddSlots<Q, SA> sl(g, A, c0, lo);
    uint64_t pb = sl.plane0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      ph[L::opp[p]] = ld_stream(sl.slot(pb, p));
      pb = sl.next(pb);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (outlet) {
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (L::cx[k] == -1) ph[k] = (T)0;
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) {  // beyond the outlet: no adjoint inflow
      int sx = x, sy = y, sz = z;
      bool bounce, leaves;
      neighbour(g, -L::cx[k], -L::cy[k], -L::cz[k], sx, sy, sz, bounce, leaves);
      const int64_t ia = bounce ? k * g.plane + cell : L::opp[k] * g.plane + cell_of(g, sx, sy, sz);
      const T v = A[leaves ? k * g.plane + cell : ia];
      ph[k] = leaves ? (T)0 : v;
    }
  }
  if (inlet) {
#pragma unroll
    for (int k = 0; k < Q; ++k) ph[k] = (T)0;
  }
  T lam[Q];
  if constexpr (HRR) {
    hrr_adjoint<Q, T, NTP>(ph, prep, g.plane, cell, ac.diff != 0, lam);
  } else {
    // Weighted moments of phi (phi_i = ph[opp i], xi_opp(k) = -xi_k) over the
    // opposite pairs: m0 = sum w phi, m1 = sum w phi xi, M2 = sum w phi xi xi;
    // terms with zero lattice coefficients are never formed.
    T m0 = (T)L::w[0] * ph[0];
    T m1[3] = {0, 0, 0}, m2[6] = {0, 0, 0, 0, 0, 0};
    bool h1[3] = {false, false, false}, h2[6] = {false, false, false, false, false, false};
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      if (L::opp[k] < k) continue;
      const int o = L::opp[k];
      const T w = (T)L::w[k];
      const T wp = w * (ph[k] + ph[o]);
      const T wq = w * (ph[k] - ph[o]);
      m0 += wp;
      const int c[3] = {L::cx[k], L::cy[k], L::cz[k]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (c[a] == 0) continue;
        const T t = c[a] > 0 ? -wq : wq;
        m1[a] = h1[a] ? m1[a] + t : t;
        h1[a] = true;
      }
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const int cf = c[ia[m]] * c[ib[m]];
        if (cf == 0) continue;
        const T t = cf > 0 ? wp : -wp;
        m2[m] = h2[m] ? m2[m] + t : t;
        h2[m] = true;
      }
    }
    const T mxx = m2[0], myy = m2[1], mzz = m2[2], mxy = m2[3], mxz = m2[4], myz = m2[5];
    T tt, m2tx, m2ty, m2tz, tmt;
    if constexpr (D == 3) {
      tt = tx * tx + ty * ty + tz * tz;
      m2tx = mxx * tx + mxy * ty + mxz * tz;
      m2ty = mxy * tx + myy * ty + myz * tz;
      m2tz = mxz * tx + myz * ty + mzz * tz;
      tmt = tx * m2tx + ty * m2ty + tz * m2tz;
    } else {
      tt = tx * tx + ty * ty;
      m2tx = mxx * tx + mxy * ty;
      m2ty = mxy * tx + myy * ty;
      m2tz = (T)0;
      tmt = tx * m2tx + ty * m2ty;
    }
    // sum_j phi_j d f^eq_j / d f_i = Phr + Phj . xi_i, scaled by omega
    const T oPhr = omega * (m0 * ((T)1 + (T)1.5 * tt) - (T)4.5 * tmt);
    const T od = omega * d;
    const T oPjx = od * ((T)3 * m1[0] + (T)9 * m2tx - (T)3 * m0 * tx);
    const T oPjy = od * ((T)3 * m1[1] + (T)9 * m2ty - (T)3 * m0 * ty);
    const T oPjz = (D == 3) ? od * ((T)3 * m1[2] + (T)9 * m2tz - (T)3 * m0 * tz) : (T)0;
    const T omc = (T)1 - omega;
    lam[0] = omc * ph[0] + oPhr;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      if (L::opp[k] < k) continue;
      const int o = L::opp[k];
      const T e = csum<T>(L::cx[k], L::cy[k], L::cz[k], oPjx, oPjy, oPjz);
      lam[k] = omc * ph[o] + (oPhr + e);
      lam[o] = omc * ph[k] + (oPhr - e);
    }
    if (ac.diff) {  // differentiated Smagorinsky: (sum_j phi_j f^neq_j) (1/tau^2) dtau/df_i
      T sd = ph[0] * (T)ld_stream<NTP>(&at(prep, (D + 2 + L::opp[0]) * g.plane + c0, lo));
#pragma unroll
      for (int k = 1; k < Q; ++k) sd += ph[k] * (T)ld_stream<NTP>(&at(prep, (D + 2 + L::opp[k]) * g.plane + c0, lo));
      T b[Coef<Q>::NB];
#pragma unroll
      for (int m = 0; m < Coef<Q>::NB; ++m) b[m] = ld_stream<NTP>(&at(prep, (D + 2 + Q + m) * g.plane + c0, lo));
#pragma unroll
      for (int i = 0; i < Q; ++i) lam[i] += sd * quad_eval<Q, T>(b, i);
    }
  }
  if (outlet) {  // virtual column: sum_j dV_j/df_i phiV_j = (xi_i - u).Psi / rho
    const int64_t o = y + (int64_t)g.ny * z;
    // weighted moments of the virtual column's adjoint values (directions
    // with xi_x = -1), zero coefficients skipped
    T v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // v0, v1 (x y z), v2 (xx yy zz xy xz yz)
    bool hv[10] = {false, false, false, false, false, false, false, false, false, false};
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (L::cx[k] != -1) continue;
      const T wp = (T)L::w[k] * pv_in[k * g.gplane + o];
      const int cf[10] = {1, L::cx[k], L::cy[k], L::cz[k], L::cx[k] * L::cx[k], L::cy[k] * L::cy[k],
                          L::cz[k] * L::cz[k], L::cx[k] * L::cy[k], L::cx[k] * L::cz[k], L::cy[k] * L::cz[k]};
#pragma unroll
      for (int m = 0; m < 10; ++m) {
        if (cf[m] == 0) continue;
        const T t = cf[m] > 0 ? wp : -wp;
        v[m] = hv[m] ? v[m] + t : t;
        hv[m] = true;
      }
    }
    const T v0 = v[0], v1x = v[1], v1y = v[2], v1z = v[3], vxx = v[4], vyy = v[5], vzz = v[6], vxy = v[7],
            vxz = v[8], vyz = v[9];
    const T ro = (T)oprep[o];
    const T uox = (T)oprep[g.gplane + o];
    const T uoy = (T)oprep[2 * g.gplane + o];
    const T uoz = (D == 3) ? (T)oprep[3 * g.gplane + o] : (T)0;
    const T Psx = (T)3 * v1x + (T)9 * (vxx * uox + vxy * uoy + vxz * uoz) - (T)3 * v0 * uox;
    const T Psy = (T)3 * v1y + (T)9 * (vxy * uox + vyy * uoy + vyz * uoz) - (T)3 * v0 * uoy;
    const T Psz = (T)3 * v1z + (T)9 * (vxz * uox + vyz * uoy + vzz * uoz) - (T)3 * v0 * uoz;
    const T iro = (T)1 / ro;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      lam[i] += (((T)L::cx[i] - uox) * Psx + ((T)L::cy[i] - uoy) * Psy + ((T)L::cz[i] - uoz) * Psz) * iro;
  }
  int64_t r;
  if (region_index<Q>(ob, x, y, z, r)) {
    T a[1 + D + L::NSYM];
#pragma unroll
    for (int m = 0; m < 1 + D + L::NSYM; ++m) a[m] = (T)src[(Coef<Q>::A0 + m) * ob.rplane + r];
#pragma unroll
    for (int i = 0; i < Q; ++i) lam[i] -= quad_eval<Q, T>(a, i);
    if constexpr (MEA) {
#pragma unroll
      for (int i = 0; i < Q; ++i) lam[i] -= (T)mea_g<Q>(g, ob, x, y, z, r, i);
    }
  }

  if (inlet) {  // lambda = 0 at the pinned inlet
#pragma unroll
    for (int k = 0; k < Q; ++k) lam[k] = (T)0;
  }

  if (!ODD) {
#pragma unroll
    for (int i = 0; i < Q; ++i) st_stream<NT>(&at(A, i * g.plane + c0, lo), lam[i]);
  } else if (fast) {
    const OddSlots<Q, SA> sl(g, A, c0, lo);
    uint64_t pb = sl.plane0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      // values leaving through the inlet or outlet end are dropped
      if (!((L::cx[p] == -1 && inlet) || (L::cx[p] == 1 && outlet))) st_stream(sl.slot(pb, p), lam[L::opp[p]]);
      pb = sl.next(pb);
    }
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) push<Q, SA>(g, A, x, y, z, cell, k, lam[L::opp[k]]);
  }
  if (outlet) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (L::cx[k] != -1) continue;
      int vx = x, vy = y - L::cy[k], vz = z - L::cz[k];
      if (classify(g, vx, vy, vz) != NB_CELL) continue;
      pv_out[k * g.gplane + vy + (int64_t)g.ny * vz] = lam[k];
    }
  }
}

template <int Q, typename SA, bool ODD, bool HRR, bool MEA>
__global__ __launch_bounds__(256) void k_adjoint(const Geo g, const ObjBox ob, const AdjC ac,
                                                 SA* __restrict__ A, const SA* __restrict__ prep,
                                                 const double* __restrict__ src,
                                                 const double* __restrict__ oprep,
                                                 const SA* __restrict__ pv_in, SA* __restrict__ pv_out) {
  if constexpr (adjoint_runs<Q, SA>()) {
    SWEEP_PROLOGUE_RUNS(false)
    if (!valid) return;
    adjoint_cell<Q, SA, ODD, HRR, MEA>(g, ob, ac, A, prep, src, oprep, pv_in, pv_out, x, y, z, tile_c0, tile_lo);
  } else {
    SWEEP_PROLOGUE_TILES
    if (!valid) return;
    adjoint_cell<Q, SA, ODD, HRR, MEA>(g, ob, ac, A, prep, src, oprep, pv_in, pv_out, x, y, z, tile_c0, tile_lo);
  }
}

// The even adjoint step with streaming hints on the phi accesses (lattices
// larger than the Infinity Cache, see ld_stream; 4-5 % faster there for
// D2Q9, 1 % for D3Q19, 9 % slower on a cache-resident lattice).
template <int Q, typename SA, bool HRR, bool MEA>
__global__ __launch_bounds__(256) void k_adjoint_stream(const Geo g, const ObjBox ob, const AdjC ac,
                                                        SA* __restrict__ A, const SA* __restrict__ prep,
                                                        const double* __restrict__ src,
                                                        const double* __restrict__ oprep,
                                                        const SA* __restrict__ pv_in, SA* __restrict__ pv_out) {
  if constexpr (adjoint_runs<Q, SA>()) {
    SWEEP_PROLOGUE_RUNS(false)
    if (!valid) return;
    adjoint_cell<Q, SA, false, HRR, MEA, true>(g, ob, ac, A, prep, src, oprep, pv_in, pv_out, x, y, z, tile_c0,
                                               tile_lo);
  } else {
    SWEEP_PROLOGUE_TILES
    if (!valid) return;
    adjoint_cell<Q, SA, false, HRR, MEA, true>(g, ob, ac, A, prep, src, oprep, pv_in, pv_out, x, y, z, tile_c0,
                                               tile_lo);
  }
}
// The odd step above the Infinity Cache: plain accesses to phi, streaming
// hints on the frozen per-cell data, which is the cell's own and read once
// per sweep (2-6 % faster than plain loads on the 8192 x 4096 and
// 768 x 384 x 128 lattices).
template <int Q, typename SA, bool HRR, bool MEA>
__global__ __launch_bounds__(256) void k_adjoint_pstream(const Geo g, const ObjBox ob, const AdjC ac,
                                                         SA* __restrict__ A, const SA* __restrict__ prep,
                                                         const double* __restrict__ src,
                                                         const double* __restrict__ oprep,
                                                         const SA* __restrict__ pv_in, SA* __restrict__ pv_out) {
  if constexpr (adjoint_runs<Q, SA>()) {
    SWEEP_PROLOGUE_RUNS(false)
    if (!valid) return;
    adjoint_cell<Q, SA, true, HRR, MEA, false, true>(g, ob, ac, A, prep, src, oprep, pv_in, pv_out, x, y, z,
                                                     tile_c0, tile_lo);
  } else {
    SWEEP_PROLOGUE_TILES
    if (!valid) return;
    adjoint_cell<Q, SA, true, HRR, MEA, false, true>(g, ob, ac, A, prep, src, oprep, pv_in, pv_out, x, y, z,
                                                     tile_c0, tile_lo);
  }
}

struct PackedAdjoint {
  Geo g;
  ObjBox ob;
  AdjC ac;
  void* A;
  const void* prep;
  const double* src;
  const double* oprep;
  void* pv[2];
  int iter0;   // adjoint iterations done when the table was built
  int pvcur0;  // outlet buffer holding the latest values at that time
  int first_block, tiles_x, tiles_y, pad_;
};

template <int Q, typename SA, bool HRR>
__global__ __launch_bounds__(256) void k_adjoint_packed(const PackedAdjoint* __restrict__ tab,
                                                        const int* __restrict__ first, int nm, int step) {
  const int b = sweep_tile((int)blockIdx.x, (int)gridDim.x);
  const PackedAdjoint& P = tab[packed_member(first, nm, b)];
  const int lb = b - P.first_block;
  const int tx = lb % P.tiles_x, r = lb / P.tiles_x;
  const int ty = r % P.tiles_y, z = r / P.tiles_y;
  const int x = tx * BX + threadIdx.x, y = ty * BY + threadIdx.y;
  if (x >= P.g.nx || y >= P.g.ny) return;
  const int64_t c0 = wave_uniform64(cell_of(P.g, tx * BX, ty * BY, z));
  const uint32_t lo = lane_offset(threadIdx.x + (uint32_t)P.g.nx * threadIdx.y);
  const int cur = (P.pvcur0 + step) & 1;
  const SA* pin = (const SA*)P.pv[cur];
  SA* pout = (SA*)P.pv[cur ^ 1];
  SA* A = (SA*)P.A;
  const SA* pr = (const SA*)P.prep;
  const bool odd = ((P.iter0 + step) & 1) != 0;
  if (P.ob.kind == OBJ_MEA) {
    if (odd)
      adjoint_cell<Q, SA, true, HRR, true>(P.g, P.ob, P.ac, A, pr, P.src, P.oprep, pin, pout, x, y, z, c0, lo);
    else
      adjoint_cell<Q, SA, false, HRR, true>(P.g, P.ob, P.ac, A, pr, P.src, P.oprep, pin, pout, x, y, z, c0, lo);
  } else {
    if (odd)
      adjoint_cell<Q, SA, true, HRR, false>(P.g, P.ob, P.ac, A, pr, P.src, P.oprep, pin, pout, x, y, z, c0, lo);
    else
      adjoint_cell<Q, SA, false, HRR, false>(P.g, P.ob, P.ac, A, pr, P.src, P.oprep, pin, pout, x, y, z, c0, lo);
  }
}

// Residual: max |phi - snapshot| and max |phi| over the state cells.
template <int Q, typename SA>
__global__ __launch_bounds__(256) void k_adjoint_residual(const Geo g, const SA* __restrict__ A,
                                                          SA* __restrict__ snap, int first,
                                                          double* __restrict__ partials) {
  __shared__ double lds[4];
  CELL_PROLOGUE
  double dmax = 0.0, pmax = 0.0;
  bool bad = false;
  if (valid && !(inout && x == 0)) {
    SA ph[Q];
    adjoint_read_canonical<Q, SA>(g, A, x, y, z, cell, inout && x == g.nx - 1, ph);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const double v = (double)ph[k];
      if (!isfinite(v)) bad = true;
      if (!first) dmax = fmax(dmax, fabs(v - (double)snap[k * g.plane + cell]));
      pmax = fmax(pmax, fabs(v));
      snap[k * g.plane + cell] = ph[k];
    }
  }
  if (bad || first) dmax = INFINITY;
  const double a = block_max256(dmax, lds);
  const double b = block_max256(pmax, lds);
  if (threadIdx.x + blockDim.x * threadIdx.y == 0) {
    partials[2 * linear_block()] = a;
    partials[2 * linear_block() + 1] = b;
  }
}

// Gradient (row a9): dJ/dd = dJ/dd|explicit - sum_i phi_i dC_i/dd, with
// sum_i phi_i dC_i/dd = omega rho [3 m1.u + 9 d u.m2.u - 3 d m0 |u|^2].
template <int Q, typename SA, typename Dd>
__global__ __launch_bounds__(256) void k_gradient(const Geo g, const ObjBox ob, const SA* __restrict__ A,
                                                  const Dd* __restrict__ dpor,
                                                  const double* __restrict__ gdat,
                                                  const double* __restrict__ src,
                                                  const SA* __restrict__ prep, int hrr,
                                                  double* __restrict__ out) {
  using L = Lat<Q>;
  constexpr int D = L::D;
  CELL_PROLOGUE
  if (!valid) return;
  if (inout && x == 0) {
    out[cell] = 0.0;
    return;
  }
  SA ph[Q];
  adjoint_read_canonical<Q, SA>(g, A, x, y, z, cell, inout && x == g.nx - 1, ph);
  if (hrr) {
    double phd[Q], pr[D + 3 + Lat<Q>::NSYM];
#pragma unroll
    for (int k = 0; k < Q; ++k) phd[k] = (double)ph[k];
#pragma unroll
    for (int m = 0; m < D + 3 + Lat<Q>::NSYM; ++m) pr[m] = (double)prep[m * g.plane + cell];
    double dJdd = 0.0;
    int64_t r;
    if (region_index<Q>(ob, x, y, z, r)) dJdd = src[Coef<Q>::DJDD * ob.rplane + r];
    out[cell] = dJdd - hrr_dphi_dd<Q>(phd, pr, (double)dpor[cell]);
    return;
  }
  double m0 = 0, m1[3] = {0, 0, 0}, m2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double wp = L::w[k] * (double)ph[k];
    const int c[3] = {-L::cx[k], -L::cy[k], -L::cz[k]};  // direction of phi_opp(k)
    m0 += wp;
    for (int a = 0; a < 3; ++a) {
      m1[a] += c[a] * wp;
      for (int b = 0; b < 3; ++b) m2[a][b] += c[a] * c[b] * wp;
    }
  }
  const double rho = gdat[cell];
  const double u[3] = {gdat[g.plane + cell], gdat[2 * g.plane + cell],
                       D == 3 ? gdat[3 * g.plane + cell] : 0.0};
  const double omega = gdat[(D + 1) * g.plane + cell];
  const double d = (double)dpor[cell];
  double m1u = 0, um2u = 0, uu = 0;
  for (int a = 0; a < 3; ++a) {
    m1u += m1[a] * u[a];
    uu += u[a] * u[a];
    for (int b = 0; b < 3; ++b) um2u += u[a] * m2[a][b] * u[b];
  }
  double dJdd = 0.0;
  int64_t r;
  if (region_index<Q>(ob, x, y, z, r)) dJdd = src[Coef<Q>::DJDD * ob.rplane + r];
  out[cell] = dJdd - omega * rho * (3.0 * m1u + 9.0 * d * um2u - 3.0 * d * m0 * uu);
}

// Adjoint populations in the canonical layout (phi_i on post-collision slots).
template <int Q, typename SA>
__global__ __launch_bounds__(256) void k_adjoint_gather(const Geo g, const SA* __restrict__ A,
                                                        double* __restrict__ out, int64_t n) {
  using L = Lat<Q>;
  CELL_PROLOGUE
  if (!valid) return;
  if (inout && x == 0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i * n + cell] = 0.0;
    return;
  }
  SA ph[Q];
  adjoint_read_canonical<Q, SA>(g, A, x, y, z, cell, inout && x == g.nx - 1, ph);
#pragma unroll
  for (int i = 0; i < Q; ++i) out[i * n + cell] = (double)ph[L::opp[i]];
}

}  // namespace hlbm
