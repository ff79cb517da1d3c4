// hlbm_launch.hip -- host-side launchers of the gfx950 kernels: grid shape
// and template dispatch over stencil, precision, collision and window mode.

#include "hlbm_kernels.hpp"

namespace hlbm {

Geo make_geo(const hlbm_lattice_s* L) {
  Geo g;
  g.nx = L->desc.nx;
  g.ny = L->desc.ny;
  g.nz = L->desc.nz;
  g.tiles_x = (g.nx + BX - 1) / BX;
  g.tiles_y = (g.ny + BY - 1) / BY;
  g.bcx = L->desc.bc_x;
  g.bcy = L->desc.bc_y;
  g.bcz = L->desc.stencil == HLBM_D2Q9 ? BC_PERIODIC : L->desc.bc_z;
  g.plane = L->plane;
  g.gplane = L->gplane;
  g.inlet_profile = L->desc.inlet_profile;
  g.u_in = L->desc.u_in;
  g.slot32 = (3 * (int64_t)g.nx + 256) * 8 < ((int64_t)1 << 32);
  return g;
}

ObjBox make_obj(const hlbm_lattice_s* L) {
  ObjBox o;
  o.active = L->obj_set;
  o.kind = L->obj_kind;
  for (int a = 0; a < 3; ++a) {
    o.lo[a] = L->lo[a];
    o.rn[a] = L->rn[a];
  }
  o.rplane = L->rplane;
  o.u0 = L->u0;
  o.p0 = L->p0;
  o.tau0 = L->desc.tau;
  o.mea = L->mea_src;
  return o;
}

Coll make_coll(const hlbm_lattice_s* L) {
  Coll c;
  c.tau0 = L->desc.tau;
  c.omega0 = 1.0 / L->desc.tau;
  c.kS = 18.0 * sqrt(2.0) * L->desc.smagorinsky_cs * L->desc.smagorinsky_cs;
  c.smag = L->desc.smagorinsky_cs > 0.0;
  for (int a = 0; a < 3; ++a) c.force[a] = L->desc.force[a];
  c.probe_cell = -1;
  c.probe_out = nullptr;
  if (L->probe_buf != nullptr && L->probe_cap > 0) {
    c.probe_cell = L->probe_cell;
    c.probe_out = L->probe_buf + (L->probe_n % L->probe_cap);
  }
  return c;
}

dim3 cell_grid(const hlbm_lattice_s* L) {
  return dim3((L->desc.nx + BX - 1) / BX, (L->desc.ny + BY - 1) / BY, L->desc.nz);
}

static const dim3 kBlock(BX, BY, 1);
static const dim3 kSweepBlock(SWEEP_BLOCK, 1, 1);

// 1D grids of the sweep kernels: runs of SWEEP_BLOCK consecutive cells
// (plain primal steps, tangent) or one workgroup per BX x BY tile (window
// steps, adjoint); see the sweep prologues.
static dim3 sweep_grid(const hlbm_lattice_s* L) {
  return dim3((unsigned)((L->n + SWEEP_BLOCK - 1) / SWEEP_BLOCK), 1, 1);
}
static dim3 tile_grid(const hlbm_lattice_s* L) {
  const dim3 c = cell_grid(L);
  return dim3(c.x * c.y * c.z, 1, 1);
}

// The collision model is a template parameter: the HRR collision needs far
// more registers, which would lower the occupancy of the BGK sweeps if both
// shared one kernel.
template <int Q, typename S, int ACC, bool HRR>
static void primal_variant(hlbm_lattice_s* L) {
  using Dd = typename Prec<S>::Dd;
  const Geo g = make_geo(L);
  const Coll c = make_coll(L);
  const ObjBox ob = make_obj(L);
  Acc acc{L->acc_rho, L->acc_j, L->desc.track_mean_populations ? L->acc_f : nullptr,
          c.smag ? L->acc_tau : nullptr, L->acc_obj};
  if constexpr (ACC != 0) {  // grouped window accumulation (FP32 and FP16 lattices)
    if (L->acc_pend) {
      acc.pend = L->acc_pend;
      acc.pslot = pend_slot_elems(L);
      if (L->pend_n < PEND_GROUP - 1) {  // a group's first steps: store the values
        acc.pend_out = L->pend_n++;
      } else {  // its last step: add the stored values, then its own
        acc.pend_in = 1;
        L->pend_n = 0;
      }
    }
  }
  if constexpr (ACC == 3) acc.rcopy = L->obj_kind != HLBM_OBJ_MEA ? L->rcopy : nullptr;
  S* A = (S*)L->f;
  const Dd* dp = (const Dd*)L->dpor;
  S* gh = (S*)L->ghost;
  constexpr bool runs = sweep_runs<Q, S, ACC>();  // lane map of the sweep (runs or tiles)
  const dim3 grid = runs ? sweep_grid(L) : tile_grid(L);
  const dim3 block = runs ? kSweepBlock : kBlock;
  // Streaming hints (lattices above the Infinity Cache): both D2Q9 steps;
  // only the D3Q19 even step, whose accesses are the cell's own slots (the
  // odd step's z neighbours reuse lines one xy layer later and ran 7 %
  // slower with the hints); the D3Q19 odd window step on its window sums.
  if (L->stream_nt) {
    if (L->parity == 0) {
      k_primal_stream<Q, S, false, ACC, HRR><<<grid, block, 0, L->stream>>>(g, c, ob, A, dp, gh, acc);
      return;
    }
    if constexpr (Q == 9) {
      k_primal_stream<Q, S, true, ACC, HRR><<<grid, block, 0, L->stream>>>(g, c, ob, A, dp, gh, acc);
      return;
    }
    if constexpr (ACC != 0) {  // D3Q19 odd window step: streaming hints on the window sums only
      k_primal_wstream<Q, S, true, ACC, HRR><<<grid, block, 0, L->stream>>>(g, c, ob, A, dp, gh, acc);
      return;
    }
  }
  if (L->parity == 0)
    k_primal<Q, S, false, ACC, HRR><<<grid, block, 0, L->stream>>>(g, c, ob, A, dp, gh, acc);
  else
    k_primal<Q, S, true, ACC, HRR><<<grid, block, 0, L->stream>>>(g, c, ob, A, dp, gh, acc);
}

// Window steps: the objective terms are fused into the sweep when the
// region is a sizeable part of the lattice, and accumulated by a separate
// region pass (before the step, from the same pre-collision state) when it is
// small, so that the sweep keeps the register budget of a plain step.
template <int Q, typename S, bool HRR>
static void primal_mode(hlbm_lattice_s* L, int accumulate) {
  if (!accumulate) {
    primal_variant<Q, S, 0, HRR>(L);
    return;
  }
  const bool mea = L->obj_set && L->obj_kind == HLBM_OBJ_MEA;
  const int64_t rcells = (int64_t)L->rn[0] * L->rn[1] * L->rn[2];
  if (L->obj_set && rcells * 8 <= L->n) {
    using Dd = typename Prec<S>::Dd;
    using T = typename Prec<S>::T;
    const dim3 rg((unsigned)((rcells + 255) / 256));  // one lane per region cell
    if (!mea && L->rcopy) {  // the sweep copies the region cells' state, the pass follows it
      primal_variant<Q, S, 3, HRR>(L);
      k_window_region_copy<Q, T><<<rg, 256, 0, L->stream>>>(make_obj(L), (const T*)L->rcopy, L->acc_obj);
      return;
    }
    if (mea)
      k_window_region<Q, S, true><<<rg, 256, 0, L->stream>>>(make_geo(L), make_obj(L), (const S*)L->f,
                                                                (const S*)L->ghost, L->parity,
                                                                (const Dd*)L->dpor, L->acc_obj);
    else
      k_window_region<Q, S, false><<<rg, 256, 0, L->stream>>>(make_geo(L), make_obj(L), (const S*)L->f,
                                                                 (const S*)L->ghost, L->parity,
                                                                 (const Dd*)L->dpor, L->acc_obj);
    primal_variant<Q, S, 3, HRR>(L);
  } else if (mea) {
    primal_variant<Q, S, 2, HRR>(L);
  } else {
    primal_variant<Q, S, 1, HRR>(L);
  }
}

template <int Q, typename S>
static hipError_t primal_impl(hlbm_lattice_s* L, int accumulate) {
  if (L->desc.collision == HLBM_COLL_HRR)
    primal_mode<Q, S, true>(L, accumulate);
  else
    primal_mode<Q, S, false>(L, accumulate);
  return hipGetLastError();
}

#define HLBM_DISPATCH(L, FN, ...)                                             \
  do {                                                                        \
    const int key_ = (L)->desc.stencil * 3 + (L)->desc.precision;            \
    switch (key_) {                                                           \
      case 0: return FN<9, double>(__VA_ARGS__);                              \
      case 1: return FN<9, float>(__VA_ARGS__);                               \
      case 2: return FN<9, _Float16>(__VA_ARGS__);                            \
      case 3: return FN<19, double>(__VA_ARGS__);                             \
      case 4: return FN<19, float>(__VA_ARGS__);                              \
      case 5: return FN<19, _Float16>(__VA_ARGS__);                           \
      default: return hipErrorInvalidValue;                                   \
    }                                                                         \
  } while (0)

hipError_t launch_primal_step(hlbm_lattice_s* L, int accumulate) {
  HLBM_DISPATCH(L, primal_impl, L, accumulate);
}

int64_t pend_slot_elems(const hlbm_lattice_s* L) {
  return L->plane * (2 + L->dim + (L->desc.track_mean_populations ? L->q : 0));
}

hipError_t launch_window_flush(hlbm_lattice_s* L, int count) {
  const Geo g = make_geo(L);
  Acc acc{L->acc_rho, L->acc_j, L->desc.track_mean_populations ? L->acc_f : nullptr,
          make_coll(L).smag ? L->acc_tau : nullptr, L->acc_obj};
  acc.pend = L->acc_pend;
  acc.pslot = pend_slot_elems(L);
  if (L->q == 9)
    k_window_flush<9><<<cell_grid(L), kBlock, 0, L->stream>>>(g, acc, count);
  else
    k_window_flush<19><<<cell_grid(L), kBlock, 0, L->stream>>>(g, acc, count);
  return hipGetLastError();
}

template <int Q, typename S>
static hipError_t init_impl(hlbm_lattice_s* L, double rho0, const double* u_dev) {
  k_init<Q, S><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (S*)L->f,
                                                       (const typename Prec<S>::Dd*)L->dpor, rho0,
                                                       u_dev, L->n);
  return hipGetLastError();
}
hipError_t launch_init(hlbm_lattice_s* L, double rho0, const double* u_dev) {
  HLBM_DISPATCH(L, init_impl, L, rho0, u_dev);
}

hipError_t launch_cylinder(hlbm_lattice_s* L, double xc, double yc, double D,
                           const double* noise_dev, int mode, double box_half, double d_solid) {
  if (L->desc.precision == HLBM_FP64)
    k_cylinder<double><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (double*)L->dpor, xc, yc,
                                                               D, noise_dev, mode, box_half, d_solid);
  else
    k_cylinder<float><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (float*)L->dpor, xc, yc, D,
                                                              noise_dev, mode, box_half, d_solid);
  return hipGetLastError();
}

hipError_t launch_mea_flags(hlbm_lattice_s* L) {
  const Geo g = make_geo(L);
  const ObjBox ob = make_obj(L);
  const bool f64 = L->desc.precision == HLBM_FP64;
  unsigned char* fl = L->mea_flag;
  if (L->desc.stencil == HLBM_D2Q9) {
    if (f64)
      k_mea_flags<9, double><<<cell_grid(L), kBlock, 0, L->stream>>>(g, ob, (const double*)L->dpor, fl);
    else
      k_mea_flags<9, float><<<cell_grid(L), kBlock, 0, L->stream>>>(g, ob, (const float*)L->dpor, fl);
    k_mea_source<9><<<cell_grid(L), kBlock, 0, L->stream>>>(g, ob, fl, L->mea_src);
  } else {
    if (f64)
      k_mea_flags<19, double><<<cell_grid(L), kBlock, 0, L->stream>>>(g, ob, (const double*)L->dpor, fl);
    else
      k_mea_flags<19, float><<<cell_grid(L), kBlock, 0, L->stream>>>(g, ob, (const float*)L->dpor, fl);
    k_mea_source<19><<<cell_grid(L), kBlock, 0, L->stream>>>(g, ob, fl, L->mea_src);
  }
  return hipGetLastError();
}

hipError_t launch_tangent_step(hlbm_lattice_s* L) {
  const Geo g = make_geo(L);
  const Coll c = make_coll(L);
  double* A = (double*)L->f;
  double* gh = (double*)L->ghost;
  const double* dp = (const double*)L->dpor;
  const dim3 grid = sweep_grid(L);
  const bool odd = L->parity != 0;
  if (L->desc.stencil == HLBM_D2Q9) {
    if (odd)
      k_tangent<9, true><<<grid, kSweepBlock, 0, L->stream>>>(g, c, A, L->tan_f, dp, L->tan_v, gh, L->tan_ghost);
    else
      k_tangent<9, false><<<grid, kSweepBlock, 0, L->stream>>>(g, c, A, L->tan_f, dp, L->tan_v, gh, L->tan_ghost);
  } else {
    if (odd)
      k_tangent<19, true><<<grid, kSweepBlock, 0, L->stream>>>(g, c, A, L->tan_f, dp, L->tan_v, gh, L->tan_ghost);
    else
      k_tangent<19, false><<<grid, kSweepBlock, 0, L->stream>>>(g, c, A, L->tan_f, dp, L->tan_v, gh, L->tan_ghost);
  }
  return hipGetLastError();
}

hipError_t launch_tangent_objective(hlbm_lattice_s* L, double* partials, int* nblocks) {
  const dim3 grid = cell_grid(L);
  *nblocks = (int)(grid.x * grid.y * grid.z);
  const Geo g = make_geo(L);
  const ObjBox ob = make_obj(L);
  const double* A = (const double*)L->f;
  const double* gh = (const double*)L->ghost;
  const double* dp = (const double*)L->dpor;
  if (L->desc.stencil == HLBM_D2Q9)
    k_tangent_objective<9><<<grid, kBlock, 0, L->stream>>>(g, ob, A, L->tan_f, gh, L->tan_ghost, L->parity, dp,
                                                          L->tan_v, partials);
  else
    k_tangent_objective<19><<<grid, kBlock, 0, L->stream>>>(g, ob, A, L->tan_f, gh, L->tan_ghost, L->parity, dp,
                                                           L->tan_v, partials);
  return hipGetLastError();
}

hipError_t launch_set_porosity(hlbm_lattice_s* L, const double* d_dev, int* bad_dev) {
  if (L->desc.precision == HLBM_FP64)
    k_set_porosity<double><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (double*)L->dpor, d_dev,
                                                                   bad_dev);
  else
    k_set_porosity<float><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (float*)L->dpor, d_dev,
                                                                  bad_dev);
  return hipGetLastError();
}

template <int Q, typename S>
static hipError_t gather_impl(hlbm_lattice_s* L, double* out) {
  k_gather<Q, S><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (const S*)L->f,
                                                         (const S*)L->ghost, L->parity, out, L->n);
  return hipGetLastError();
}
hipError_t launch_gather(hlbm_lattice_s* L, double* out_dev) { HLBM_DISPATCH(L, gather_impl, L, out_dev); }

template <int Q, typename S>
static hipError_t scatter_impl(hlbm_lattice_s* L, const double* in) {
  k_scatter<Q, S><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (S*)L->f, in, L->n);
  return hipGetLastError();
}
hipError_t launch_scatter(hlbm_lattice_s* L, const double* in_dev) {
  HLBM_DISPATCH(L, scatter_impl, L, in_dev);
}

template <int Q, typename S>
static hipError_t moments_impl(hlbm_lattice_s* L, double* rho, double* u) {
  k_moments<Q, S><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (const S*)L->f,
                                                          (const S*)L->ghost, L->parity, rho, u, L->n);
  return hipGetLastError();
}
hipError_t launch_moments(hlbm_lattice_s* L, double* rho_dev, double* u_dev) {
  HLBM_DISPATCH(L, moments_impl, L, rho_dev, u_dev);
}

hipError_t launch_mean_fields(hlbm_lattice_s* L, int field, double* out_dev) {
  const double inv = L->nsamp ? 1.0 / (double)L->nsamp : 0.0;
  if (L->desc.stencil == HLBM_D2Q9)
    k_mean_fields<9><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), field, L->acc_rho, L->acc_j,
                                                             L->acc_tau, inv, out_dev, L->n);
  else
    k_mean_fields<19><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), field, L->acc_rho, L->acc_j,
                                                              L->acc_tau, inv, out_dev, L->n);
  return hipGetLastError();
}

static int grid_blocks(const dim3& g) { return (int)(g.x * g.y * g.z); }

template <int Q, typename S>
static hipError_t steady_impl(hlbm_lattice_s* L, int first, double* partials, int* nb) {
  const dim3 grid = cell_grid(L);
  *nb = grid_blocks(grid);
  k_steady_check<Q, S><<<grid, kBlock, 0, L->stream>>>(make_geo(L), (const S*)L->f, (const S*)L->ghost,
                                                       L->parity, L->usnap, first, partials);
  return hipGetLastError();
}
hipError_t launch_steady_check(hlbm_lattice_s* L, int first, double* partials, int* nblocks) {
  HLBM_DISPATCH(L, steady_impl, L, first, partials, nblocks);
}

template <int Q, typename S>
static hipError_t objective_impl(hlbm_lattice_s* L, int which, double* partials, int* nb) {
  const dim3 grid = cell_grid(L);
  *nb = grid_blocks(grid);
  const double inv = L->nsamp ? 1.0 / (double)L->nsamp : 0.0;
  k_objective<Q, S><<<grid, kBlock, 0, L->stream>>>(make_geo(L), make_obj(L), (const S*)L->f,
                                                    (const S*)L->ghost, L->parity,
                                                    (const typename Prec<S>::Dd*)L->dpor, which,
                                                    L->acc_obj, inv, partials);
  return hipGetLastError();
}
hipError_t launch_objective(hlbm_lattice_s* L, int which, double* partials, int* nblocks) {
  HLBM_DISPATCH(L, objective_impl, L, which, partials, nblocks);
}

hipError_t launch_finalize_sum(hlbm_lattice_s* L, const double* partials, int n, double* out) {
  k_finalize_sum<<<1, 256, 0, L->stream>>>(partials, n, out);
  return hipGetLastError();
}
hipError_t launch_finalize_max2(hlbm_lattice_s* L, const double* partials, int n, double* out) {
  k_finalize_max2<<<1, 256, 0, L->stream>>>(partials, n, out);
  return hipGetLastError();
}

// adjoint storage type: FP64 form -> double, FP32/FP16S forms -> float
template <typename S>
struct AdjT {
  using type = float;
};
template <>
struct AdjT<double> {
  using type = double;
};

template <int Q, typename S>
static hipError_t prep_impl(hlbm_lattice_s* L, int source, double tau_adj, int turb) {
  using SA = typename AdjT<S>::type;
  PrepIn pin;
  pin.acc_rho = L->acc_rho;
  pin.acc_j = L->acc_j;
  pin.acc_f = L->acc_f;
  pin.acc_tau = L->acc_tau;
  pin.acc_obj = L->acc_obj;
  pin.inv = L->nsamp ? 1.0 / (double)L->nsamp : 0.0;
  pin.source = source;
  pin.smag = L->desc.smagorinsky_cs > 0.0;
  pin.turb = turb;
  pin.tau0 = L->desc.tau;
  pin.tau_adj = tau_adj;
  pin.kS = 18.0 * sqrt(2.0) * L->desc.smagorinsky_cs * L->desc.smagorinsky_cs;
  pin.hrr = L->desc.collision == HLBM_COLL_HRR;
  k_adjoint_prep<Q, S, SA><<<cell_grid(L), kBlock, 0, L->stream>>>(
      make_geo(L), make_obj(L), pin, (const S*)L->f, (const S*)L->ghost, L->parity,
      (const typename Prec<S>::Dd*)L->dpor, (SA*)L->prep, L->src, L->gdat, L->oprep);
  return hipGetLastError();
}
hipError_t launch_adjoint_prep(hlbm_lattice_s* L, int source, double tau_adj, int turb) {
  HLBM_DISPATCH(L, prep_impl, L, source, tau_adj, turb);
}

template <int Q, typename S>
static hipError_t adjoint_impl(hlbm_lattice_s* L) {
  using SA = typename AdjT<S>::type;
  AdjC ac;
  ac.les = L->adj_les;
  ac.diff = L->adj_diff;
  ac.omega0 = L->adj_omega;  // used when the relaxation time is uniform (no closure)
  const Geo g = make_geo(L);
  const ObjBox ob = make_obj(L);
  SA* A = (SA*)L->phi;
  const SA* pin = (const SA*)L->pv[L->pvcur];
  SA* pout = (SA*)L->pv[L->pvcur ^ 1];
  const SA* prep = (const SA*)L->prep;
  const bool odd = (L->adj_iters & 1) != 0;
  const bool hrr = L->desc.collision == HLBM_COLL_HRR, mea = L->obj_kind == HLBM_OBJ_MEA;
  constexpr bool runs = adjoint_runs<Q, SA>();  // lane map of the sweep (runs or tiles)
  const dim3 grid = runs ? sweep_grid(L) : tile_grid(L);
  const dim3 block = runs ? kSweepBlock : kBlock;
#define HLBM_ADJ(KERNEL, ...) \
  KERNEL<Q, SA, __VA_ARGS__><<<grid, block, 0, L->stream>>>(g, ob, ac, A, prep, L->src, L->oprep, pin, pout)
  // Streaming hints above the Infinity Cache: on phi and the frozen data in
  // the even step, on the frozen data only in the odd step.
  if (L->stream_nt && !odd) {
    if (hrr) {
      if (mea) HLBM_ADJ(k_adjoint_stream, true, true); else HLBM_ADJ(k_adjoint_stream, true, false);
    } else {
      if (mea) HLBM_ADJ(k_adjoint_stream, false, true); else HLBM_ADJ(k_adjoint_stream, false, false);
    }
  } else if (L->stream_nt) {
    if (hrr) {
      if (mea) HLBM_ADJ(k_adjoint_pstream, true, true); else HLBM_ADJ(k_adjoint_pstream, true, false);
    } else {
      if (mea) HLBM_ADJ(k_adjoint_pstream, false, true); else HLBM_ADJ(k_adjoint_pstream, false, false);
    }
  } else if (hrr) {
    if (mea) {
      if (odd) HLBM_ADJ(k_adjoint, true, true, true); else HLBM_ADJ(k_adjoint, false, true, true);
    } else {
      if (odd) HLBM_ADJ(k_adjoint, true, true, false); else HLBM_ADJ(k_adjoint, false, true, false);
    }
  } else {
    if (mea) {
      if (odd) HLBM_ADJ(k_adjoint, true, false, true); else HLBM_ADJ(k_adjoint, false, false, true);
    } else {
      if (odd) HLBM_ADJ(k_adjoint, true, false, false); else HLBM_ADJ(k_adjoint, false, false, false);
    }
  }
#undef HLBM_ADJ
  return hipGetLastError();
}
hipError_t launch_adjoint_step(hlbm_lattice_s* L) {
  HLBM_DISPATCH(L, adjoint_impl, L);
}

template <int Q, typename S>
static hipError_t residual_impl(hlbm_lattice_s* L, int first, double* partials, int* nb) {
  using SA = typename AdjT<S>::type;
  const dim3 grid = cell_grid(L);
  *nb = grid_blocks(grid);
  k_adjoint_residual<Q, SA><<<grid, kBlock, 0, L->stream>>>(make_geo(L), (const SA*)L->phi, (SA*)L->snap,
                                                            first, partials);
  return hipGetLastError();
}
hipError_t launch_adjoint_residual(hlbm_lattice_s* L, int first, double* partials, int* nblocks) {
  HLBM_DISPATCH(L, residual_impl, L, first, partials, nblocks);
}

template <int Q, typename S>
static hipError_t gradient_impl(hlbm_lattice_s* L, double* g_dev) {
  using SA = typename AdjT<S>::type;
  k_gradient<Q, SA, typename Prec<S>::Dd><<<cell_grid(L), kBlock, 0, L->stream>>>(
      make_geo(L), make_obj(L), (const SA*)L->phi, (const typename Prec<S>::Dd*)L->dpor, L->gdat, L->src,
      (const SA*)L->prep, L->desc.collision == HLBM_COLL_HRR, g_dev);
  return hipGetLastError();
}
hipError_t launch_gradient(hlbm_lattice_s* L, double* g_dev) { HLBM_DISPATCH(L, gradient_impl, L, g_dev); }

template <int Q, typename S>
static hipError_t adjoint_gather_impl(hlbm_lattice_s* L, double* out) {
  using SA = typename AdjT<S>::type;
  k_adjoint_gather<Q, SA><<<cell_grid(L), kBlock, 0, L->stream>>>(make_geo(L), (const SA*)L->phi, out, L->n);
  return hipGetLastError();
}
hipError_t launch_adjoint_gather(hlbm_lattice_s* L, double* out_dev) {
  HLBM_DISPATCH(L, adjoint_gather_impl, L, out_dev);
}

template <int Q, typename S>
static hipError_t copy_probe_impl(hlbm_lattice_s* L, int pattern, int streaming, int* sink, void* second) {
  const Geo g = make_geo(L);
  S* A = (S*)L->f;
  const typename Prec<S>::Dd* dp = (const typename Prec<S>::Dd*)L->dpor;
  const dim3 grid = sweep_grid(L);
  if (pattern == 2) {
    k_copy_probe_pull<Q, S><<<grid, kSweepBlock, 0, L->stream>>>(g, A, (S*)second, dp, sink);
  } else if (pattern == 0) {
    if (streaming)
      k_copy_probe<Q, S, false, true><<<grid, kSweepBlock, 0, L->stream>>>(g, A, dp, sink);
    else
      k_copy_probe<Q, S, false, false><<<grid, kSweepBlock, 0, L->stream>>>(g, A, dp, sink);
  } else {
    if (streaming)
      k_copy_probe<Q, S, true, true><<<grid, kSweepBlock, 0, L->stream>>>(g, A, dp, sink);
    else
      k_copy_probe<Q, S, true, false><<<grid, kSweepBlock, 0, L->stream>>>(g, A, dp, sink);
  }
  return hipGetLastError();
}
hipError_t launch_copy_probe(hlbm_lattice_s* L, int pattern, int streaming, int* sink_dev, void* second) {
  HLBM_DISPATCH(L, copy_probe_impl, L, pattern, streaming, sink_dev, second);
}

}  // namespace hlbm

// =========================================================================
// packed launches (groups of small lattices)
// =========================================================================

namespace hlbm {

int tiles_x_of(const hlbm_lattice_s* L) { return (L->desc.nx + BX - 1) / BX; }
int tiles_y_of(const hlbm_lattice_s* L) { return (L->desc.ny + BY - 1) / BY; }

void fill_packed_primal(const hlbm_lattice_s* L, int accumulate, int first_block, void* out) {
  PackedPrimal* P = (PackedPrimal*)out;
  P->g = make_geo(L);
  P->c = make_coll(L);
  P->c.probe_cell = -1;  // the probe is not recorded in packed launches
  P->c.probe_out = nullptr;
  P->ob = make_obj(L);
  const bool smag = L->desc.smagorinsky_cs > 0.0;
  P->acc = Acc{L->acc_rho, L->acc_j, L->desc.track_mean_populations ? L->acc_f : nullptr,
               smag ? L->acc_tau : nullptr, L->acc_obj};
  P->A = L->f;
  P->dpor = L->dpor;
  P->ghost = L->ghost;
  P->parity0 = L->parity;
  P->accumulate = accumulate;
  P->first_block = first_block;
  P->tiles_x = tiles_x_of(L);
  P->tiles_y = tiles_y_of(L);
  P->pad_ = 0;
}

void fill_packed_adjoint(const hlbm_lattice_s* L, int first_block, void* out) {
  PackedAdjoint* P = (PackedAdjoint*)out;
  P->g = make_geo(L);
  P->ob = make_obj(L);
  P->ac.les = L->adj_les;
  P->ac.diff = L->adj_diff;
  P->ac.omega0 = L->adj_omega;
  P->A = L->phi;
  P->prep = L->prep;
  P->src = L->src;
  P->oprep = L->oprep;
  P->pv[0] = L->pv[0];
  P->pv[1] = L->pv[1];
  P->iter0 = (int)(L->adj_iters & 1);
  P->pvcur0 = L->pvcur;
  P->first_block = first_block;
  P->tiles_x = tiles_x_of(L);
  P->tiles_y = tiles_y_of(L);
  P->pad_ = 0;
}

size_t packed_primal_size() { return sizeof(PackedPrimal); }
size_t packed_adjoint_size() { return sizeof(PackedAdjoint); }

template <int Q, typename S>
static void primal_packed(hipStream_t st, bool hrr, const PackedPrimal* t, const int* first, int nm, int blocks,
                          int step) {
  const dim3 grid((unsigned)blocks);
  if (hrr)
    k_primal_packed<Q, S, true><<<grid, kBlock, 0, st>>>(t, first, nm, step);
  else
    k_primal_packed<Q, S, false><<<grid, kBlock, 0, st>>>(t, first, nm, step);
}

hipError_t launch_primal_packed(hipStream_t st, int stencil, int precision, int collision, const void* tab,
                                const int* first, int nm, int blocks, int step) {
  const PackedPrimal* t = (const PackedPrimal*)tab;
  const bool hrr = collision == HLBM_COLL_HRR;
  switch (stencil * 3 + precision) {
    case 0: primal_packed<9, double>(st, hrr, t, first, nm, blocks, step); break;
    case 1: primal_packed<9, float>(st, hrr, t, first, nm, blocks, step); break;
    case 2: primal_packed<9, _Float16>(st, hrr, t, first, nm, blocks, step); break;
    case 3: primal_packed<19, double>(st, hrr, t, first, nm, blocks, step); break;
    case 4: primal_packed<19, float>(st, hrr, t, first, nm, blocks, step); break;
    case 5: primal_packed<19, _Float16>(st, hrr, t, first, nm, blocks, step); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int Q, typename SA>
static void adjoint_packed(hipStream_t st, bool hrr, const PackedAdjoint* t, const int* first, int nm, int blocks,
                           int step) {
  const dim3 grid((unsigned)blocks);
  if (hrr)
    k_adjoint_packed<Q, SA, true><<<grid, kBlock, 0, st>>>(t, first, nm, step);
  else
    k_adjoint_packed<Q, SA, false><<<grid, kBlock, 0, st>>>(t, first, nm, step);
}

hipError_t launch_adjoint_packed(hipStream_t st, int stencil, int precision, int collision, const void* tab,
                                 const int* first, int nm, int blocks, int step) {
  const PackedAdjoint* t = (const PackedAdjoint*)tab;
  const bool f64 = precision == HLBM_FP64, hrr = collision == HLBM_COLL_HRR;
  if (stencil == HLBM_D2Q9) {
    if (f64)
      adjoint_packed<9, double>(st, hrr, t, first, nm, blocks, step);
    else
      adjoint_packed<9, float>(st, hrr, t, first, nm, blocks, step);
  } else {
    if (f64)
      adjoint_packed<19, double>(st, hrr, t, first, nm, blocks, step);
    else
      adjoint_packed<19, float>(st, hrr, t, first, nm, blocks, step);
  }
  return hipGetLastError();
}

}  // namespace hlbm
