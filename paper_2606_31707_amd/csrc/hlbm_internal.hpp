// hlbm_internal.hpp -- host-side lattice state shared by the C ABI and the
// kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <unordered_map>

#include "../../include/hlbm.h"
#include "hlbm_device.hpp"
#include "hlbm_host.hpp"

struct hlbm_lattice_s {
  hlbm_desc desc;
  int q = 0, dim = 0, ncoef = 0, nb = 0;
  int64_t n = 0;       // cells
  int64_t plane = 0;   // padded plane stride (elements)
  int64_t gplane = 0;  // padded (y, z) plane stride of the outlet buffers
  size_t ssize = 0;    // bytes per stored population
  size_t dsize = 0;    // bytes per porosity value
  hipStream_t stream = nullptr;

  // primal state
  void* f = nullptr;      // q * plane stored populations (AA pattern, in place)
  void* dpor = nullptr;   // plane porosity values
  void* ghost = nullptr;  // q * gplane outlet virtual values (even -> odd step)
  bool stream_nt = false;  // streaming load/store hints in the sweeps
  int parity = 0;         // 0: canonical layout; 1: after an even (local) step
  int64_t steps = 0;

  // window (FP64)
  double* acc_rho = nullptr;  // plane: sum of (rho - 1)
  double* acc_j = nullptr;    // dim * plane
  double* acc_f = nullptr;    // q * plane: sum of f_i - w_i (optional)
  double* acc_tau = nullptr;  // plane: sum of tau_eff (with the closure)
  double* acc_obj = nullptr;  // ncoef * rplane
  int64_t nsamp = 0;
  // FP32 and FP16 lattices: PEND_GROUP - 1 slots of (2 + dim [+ q]) FP32
  // planes holding the values of the first window steps of a group, added
  // to the sums by the group's last step (or by a flush at the end of a
  // run); pend_n: slots filled
  float* acc_pend = nullptr;
  int pend_n = 0;

  // objective region
  int obj_set = 0, obj_kind = 0;
  int lo[3] = {0, 0, 0}, rn[3] = {1, 1, 1};
  int64_t rplane = 0;
  double u0 = 0.0, p0 = 1.0 / 3.0;
  void* rcopy = nullptr;              // rplane records: region cells' pre-collision state (region_copy_used)
  unsigned char* mea_flag = nullptr;  // rplane: J_MEA surface nodes of the region
  double* mea_src = nullptr;          // q * rplane: J_MEA's constant dJ/df_k over the region
  int mea_dirty = 1;                  // flags to rebuild (porosity or region changed)

  // adjoint
  void* phi = nullptr;    // q * plane (double for FP64, float otherwise)
  void* prep = nullptr;   // per-cell frozen coefficients (adjoint type)
  int nprep = 0;          // planes in prep
  double* src = nullptr;  // ncoef * rplane: adjoint source and dJ/dd on the region
  double* gdat = nullptr; // (dim + 2) * plane: rho, u, omega for the gradient
  double* oprep = nullptr;// (1 + dim) * gplane: rho, u of the outlet column
  void* pv[2] = {nullptr, nullptr};  // q * gplane: adjoint on the outlet virtual slots
  int pvcur = 0;
  void* snap = nullptr;   // q * plane residual snapshot
  size_t asize = 0;       // bytes per adjoint value
  int adj_ready = 0;
  int adj_diff = 0;       // differentiated closure term active
  int adj_les = 0;        // per-cell omega
  double adj_omega = 0.0; // 1/tau_adj when uniform
  int64_t adj_iters = 0;

  // reductions
  double* red = nullptr;      // partials
  int64_t red_cap = 0;
  double* red_host = nullptr; // pinned
  double* usnap = nullptr;    // dim * plane steady-check snapshot
  int usnap_valid = 0;

  // profiling: launches of each sweep kind timed in blocks of up to
  // prof_every back-to-back launches, by events recorded on the stream
  // before the first and after the last launch of a block; a ring of event
  // pairs is read back lazily, so timing adds no host synchronization
  static constexpr int kProfSlots = 64;
  int64_t prof_every = 0;
  int64_t prof_sampled[3] = {0, 0, 0};  // launches timed per kind
  double prof_ms[3] = {0.0, 0.0, 0.0};
  hipEvent_t prof_ev[kProfSlots][2] = {};
  int prof_slot_kind[kProfSlots] = {};     // -1: free
  int64_t prof_slot_n[kProfSlots] = {};    // launches in the slot's block
  int prof_next = 0;                       // next slot of the ring
  int prof_open = -1;                      // slot of the open block, -1: none
  int prof_open_kind = -1;

  // forward tangent (FP64): fdot in the AA layout, its outlet buffer, v,
  // and the device record of (J, dJ/dd . v)
  double* tan_f = nullptr;
  double* tan_ghost = nullptr;
  double* tan_v = nullptr;
  double* tan_rec = nullptr;
  int64_t tan_rec_cap = 0;

  // velocity probe
  int64_t probe_cell = -1;
  double* probe_buf = nullptr;
  int64_t probe_cap = 0, probe_n = 0;

  // every device buffer the handle owns, with its size (hlbm_device_bytes)
  std::unordered_map<void*, size_t> allocs;

  // device the handle was created on, and the device address of that GPU's
  // copy of the library's scratch array (the allocation-free entry point)
  int device = 0;
  int* noalloc_scratch = nullptr;
};

namespace hlbm {

// Per-launch collision parameters.
struct Coll {
  double tau0, omega0;
  double kS;      // 18 sqrt(2) Cs^2
  int smag;       // closure on
  double force[3];
  int64_t probe_cell;  // cell whose u_y is recorded (-1: none)
  double* probe_out;   // destination of this step's probe value
};

struct ObjBox {
  int active, kind;
  int lo[3], rn[3];
  int64_t rplane;
  double u0, p0, tau0;           // J_MEA: u0 carries the surface area A
  const double* mea;             // J_MEA: dJ/df_k over the region, plane k (else null)
};

struct Acc {
  double* rho;
  double* j;
  double* f;
  double* tau;
  double* obj;
  // Grouped accumulation (FP32 arithmetic): the pending values of the
  // first PEND_GROUP - 1 window steps of a group, PEND_GROUP - 1 slots of
  // pslot elements, each the FP32 planes drho, j (dim), tau_eff, f (q, when
  // tracked); null where every step adds to the sums at once.  pend_out:
  // the slot this step stores its values in (-1: none); pend_in != 0: this
  // step adds all PEND_GROUP - 1 slots, in slot order, before its own values.
  float* pend = nullptr;
  int64_t pslot = 0;
  int pend_out = -1;
  int pend_in = 0;
  // Window steps with a small moment-form objective region: the sweep
  // stores each region cell's pre-collision populations and porosity here
  // (one record of region_copy_stride arithmetic-type values per region
  // cell, region order) for the region pass that follows it; null otherwise.
  void* rcopy = nullptr;
};


Geo make_geo(const hlbm_lattice_s* L);
ObjBox make_obj(const hlbm_lattice_s* L);
Coll make_coll(const hlbm_lattice_s* L);
dim3 cell_grid(const hlbm_lattice_s* L);

// launchers (return hipError_t of the launch)
hipError_t launch_init(hlbm_lattice_s* L, double rho0, const double* u_dev);
// adds the first `count` pending slots of the grouped window accumulation
// to the sums; elements per pending slot
hipError_t launch_window_flush(hlbm_lattice_s* L, int count);
int64_t pend_slot_elems(const hlbm_lattice_s* L);
hipError_t launch_cylinder(hlbm_lattice_s* L, double xc, double yc, double D,
                           const double* noise_dev, int mode, double box_half, double d_solid);
hipError_t launch_set_porosity(hlbm_lattice_s* L, const double* d_dev, int* bad_dev);
hipError_t launch_mea_flags(hlbm_lattice_s* L);
hipError_t launch_tangent_step(hlbm_lattice_s* L);
hipError_t launch_tangent_objective(hlbm_lattice_s* L, double* partials, int* nblocks);
hipError_t launch_primal_step(hlbm_lattice_s* L, int accumulate);
hipError_t launch_gather(hlbm_lattice_s* L, double* out_dev);
hipError_t launch_scatter(hlbm_lattice_s* L, const double* in_dev);
hipError_t launch_moments(hlbm_lattice_s* L, double* rho_dev, double* u_dev);
hipError_t launch_mean_fields(hlbm_lattice_s* L, int field, double* out_dev);
hipError_t launch_steady_check(hlbm_lattice_s* L, int first, double* partials, int* nblocks);
hipError_t launch_objective(hlbm_lattice_s* L, int which, double* partials, int* nblocks);
hipError_t launch_finalize_sum(hlbm_lattice_s* L, const double* partials, int n, double* out);
hipError_t launch_finalize_max2(hlbm_lattice_s* L, const double* partials, int n, double* out);
hipError_t launch_adjoint_prep(hlbm_lattice_s* L, int source, double tau_adj, int turb);
hipError_t launch_adjoint_step(hlbm_lattice_s* L);
hipError_t launch_adjoint_residual(hlbm_lattice_s* L, int first, double* partials, int* nblocks);
hipError_t launch_gradient(hlbm_lattice_s* L, double* g_dev);
hipError_t launch_adjoint_gather(hlbm_lattice_s* L, double* out_dev);
// pattern 2 writes to `second`, an array of the population array's size
hipError_t launch_copy_probe(hlbm_lattice_s* L, int pattern, int streaming, int* sink_dev, void* second);

// packed launches over groups of lattices
int tiles_x_of(const hlbm_lattice_s* L);
int tiles_y_of(const hlbm_lattice_s* L);
size_t packed_primal_size();
size_t packed_adjoint_size();
void fill_packed_primal(const hlbm_lattice_s* L, int accumulate, int first_block, void* out);
void fill_packed_adjoint(const hlbm_lattice_s* L, int first_block, void* out);
hipError_t launch_primal_packed(hipStream_t st, int stencil, int precision, int collision, const void* tab,
                                const int* first, int nm, int blocks, int step);
hipError_t launch_adjoint_packed(hipStream_t st, int stencil, int precision, int collision, const void* tab,
                                 const int* first, int nm, int blocks, int step);

}  // namespace hlbm

// A group of lattices stepped by packed launches (see hlbm_group_* in hlbm.h).
struct hlbm_group_s {
  hipStream_t stream = nullptr;
  int stencil = -1, precision = -1, collision = 0;
  int n_primal = 0, n_adjoint = 0;
  int blocks_primal = 0, blocks_adjoint = 0;
  void* tab_primal = nullptr;   // device tables
  void* tab_adjoint = nullptr;
  int* first_primal = nullptr;  // device first-block arrays
  int* first_adjoint = nullptr;
  size_t cap_primal = 0, cap_adjoint = 0;  // members the device tables hold
  int64_t steps_since_set = 0;
  // the last multi-step run of packed launches, captured as a HIP graph
  // (kernel nodes only) and replayed while the launch arguments repeat
  hipGraphExec_t gexec = nullptr;
  uint64_t gkey[13] = {};  // launch arguments the graph was captured with
  bool graph_ok = true;    // false after a failed capture: plain launches
  hlbm_lattice_s** members = nullptr;
  int32_t* modes = nullptr;
  int64_t* counts0 = nullptr;  // each member's step (or adjoint iteration) count at the set
  int count = 0;
};
