// hlbm_api.hip -- C ABI of the gfx950 HLBM mean-flow adjoint library: lattice
// lifetime, argument checks, and the host-side loops of the three phases of
// the paper's Algorithm 1 (primal with window, adjoint, gradient assembly).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hlbm_host.hpp"
#include "hlbm_internal.hpp"
#include "hlbm_stop.hpp"

using namespace hlbm;

namespace {

thread_local std::string g_last_error;

hlbm_status fail(hlbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(HLBM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define CHECK_LAT(L)                                              \
  do {                                                            \
    if ((L) == nullptr) return fail(HLBM_E_INVALID, "null lattice"); \
  } while (0)

hlbm_status dev_alloc(void** p, size_t bytes) {
  if (*p) return HLBM_OK;
  hipError_t e = hipMalloc(p, bytes ? bytes : 256);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(HLBM_E_OOM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  return HLBM_OK;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

// Buffers owned by a lattice are allocated and freed through these, which
// keep the handle's record of its device memory.
hlbm_status lat_alloc(hlbm_lattice_s* L, void** p, size_t bytes) {
  if (*p) return HLBM_OK;
  hlbm_status s = dev_alloc(p, bytes);
  if (s == HLBM_OK) L->allocs[*p] = bytes ? bytes : 256;
  return s;
}
void lat_free(hlbm_lattice_s* L, void* p) {
  if (!p) return;
  L->allocs.erase(p);
  dev_free(p);
}

// Scratch of the allocation-free entry point (hlbm_set_porosity_noalloc): a
// library-owned device array that every GPU the library runs on holds, each
// its own copy, until the process ends.  In host code `scratch` names a
// host-side stand-in, not a device address: the address of a device's copy
// is looked up once per device (with that device current, when the first
// lattice is created on it) and only that address reaches kernels and copies.
constexpr int kScratchInts = 64;  // 256 bytes
__device__ __align__(256) int scratch[kScratchInts];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch_addr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
hlbm_status scratch_address(int device, int** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return fail(HLBM_E_DEVICE, "device ordinal %d out of range", device);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(HLBM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch_addr[device] = (int*)p;
  }
  *out = g_scratch_addr[device];
  return HLBM_OK;
}

// Clears n ints (a kernel rather than a memset: safe under stream capture).
__global__ void k_clear_ints(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hlbm_status validate_desc(const hlbm_desc* d) {
  const char* why = desc_problem(d);
  return why ? fail(HLBM_E_INVALID, "%s", why) : HLBM_OK;
}

// device scratch for host <-> device exchange of FP64 arrays
hlbm_status staging(hlbm_lattice_s* L, const double* in, int64_t count, int mem, double** dev,
                    bool* owned) {
  *owned = false;
  if (mem == HLBM_MEM_DEVICE) {
    *dev = const_cast<double*>(in);
    return HLBM_OK;
  }
  void* p = nullptr;
  hlbm_status s = dev_alloc(&p, sizeof(double) * (size_t)count);
  if (s != HLBM_OK) return s;
  *dev = (double*)p;
  *owned = true;
  if (in) {
    hipError_t e = hipMemcpyAsync(p, in, sizeof(double) * count, hipMemcpyHostToDevice, L->stream);
    if (e != hipSuccess) {
      dev_free(p);
      return fail(HLBM_E_DEVICE, "H2D copy: %s", hipGetErrorString(e));
    }
  }
  return HLBM_OK;
}

hlbm_status finish_out(hlbm_lattice_s* L, double* dev, double* out, int64_t count, int mem, bool owned) {
  hipError_t e = hipSuccess;
  if (mem == HLBM_MEM_HOST) e = hipMemcpyAsync(out, dev, sizeof(double) * count, hipMemcpyDeviceToHost, L->stream);
  hipError_t e2 = hipStreamSynchronize(L->stream);
  if (owned) dev_free(dev);
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "D2H copy: %s", hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(HLBM_E_DEVICE, "stream sync: %s", hipGetErrorString(e2));
  return HLBM_OK;
}

// J_MEA reads its surface flags; they follow the porosity and the region.
hlbm_status ensure_mea(hlbm_lattice_s* L) {
  if (!L->obj_set || L->obj_kind != HLBM_OBJ_MEA || !L->mea_dirty) return HLBM_OK;
  hipError_t e = launch_mea_flags(L);
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "J_MEA surface flags: %s", hipGetErrorString(e));
  L->mea_dirty = 0;
  return HLBM_OK;
}

hlbm_status ensure_window(hlbm_lattice_s* L) {
  const int64_t P = L->plane;
  hlbm_status s;
  bool fresh = L->acc_rho == nullptr;
  if ((s = lat_alloc(L, (void**)&L->acc_rho, sizeof(double) * P)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, (void**)&L->acc_j, sizeof(double) * P * L->dim)) != HLBM_OK) return s;
  if (L->desc.track_mean_populations && (s = lat_alloc(L, (void**)&L->acc_f, sizeof(double) * P * L->q)) != HLBM_OK)
    return s;
  if (L->desc.smagorinsky_cs > 0.0 && (s = lat_alloc(L, (void**)&L->acc_tau, sizeof(double) * P)) != HLBM_OK) return s;
  // FP32 arithmetic: the pending slots of the grouped accumulation (each
  // written by a window step before it is read)
  if (L->desc.precision != HLBM_FP64 &&
      (s = lat_alloc(L, (void**)&L->acc_pend, sizeof(float) * pend_slot_elems(L) * (PEND_GROUP - 1))) != HLBM_OK)
    return s;
  if (fresh) {
    HIP_TRY(hipMemsetAsync(L->acc_rho, 0, sizeof(double) * P, L->stream));
    HIP_TRY(hipMemsetAsync(L->acc_j, 0, sizeof(double) * P * L->dim, L->stream));
    if (L->acc_f) HIP_TRY(hipMemsetAsync(L->acc_f, 0, sizeof(double) * P * L->q, L->stream));
    if (L->acc_tau) HIP_TRY(hipMemsetAsync(L->acc_tau, 0, sizeof(double) * P, L->stream));
  }
  return HLBM_OK;
}

hlbm_status ensure_partials(hlbm_lattice_s* L, int64_t nvals) {
  if (L->red_cap >= nvals) return HLBM_OK;
  lat_free(L, L->red);
  L->red = nullptr;
  L->red_cap = 0;
  hlbm_status s = lat_alloc(L, (void**)&L->red, sizeof(double) * (size_t)nvals);
  if (s == HLBM_OK) L->red_cap = nvals;
  return s;
}

int64_t n_blocks(hlbm_lattice_s* L) {
  dim3 g = cell_grid(L);
  return (int64_t)g.x * g.y * g.z;
}

// Reduces partials to up to two doubles on the host.
hlbm_status reduce_to_host(hlbm_lattice_s* L, int nblocks, int pairs, double* out) {
  double* res = L->red + 2 * n_blocks(L);  // result slots after the partials
  if (pairs)
    HIP_TRY(launch_finalize_max2(L, L->red, nblocks, res));
  else
    HIP_TRY(launch_finalize_sum(L, L->red, nblocks, res));
  HIP_TRY(hipMemcpyAsync(L->red_host, res, sizeof(double) * 2, hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(hipStreamSynchronize(L->stream));
  out[0] = L->red_host[0];
  if (pairs) out[1] = L->red_host[1];
  return HLBM_OK;
}

void reset_window_counts(hlbm_lattice_s* L) { L->nsamp = 0; }

hlbm_status zero_window(hlbm_lattice_s* L) {
  const int64_t P = L->plane;
  if (L->acc_rho) HIP_TRY(hipMemsetAsync(L->acc_rho, 0, sizeof(double) * P, L->stream));
  if (L->acc_j) HIP_TRY(hipMemsetAsync(L->acc_j, 0, sizeof(double) * P * L->dim, L->stream));
  if (L->acc_f) HIP_TRY(hipMemsetAsync(L->acc_f, 0, sizeof(double) * P * L->q, L->stream));
  if (L->acc_tau) HIP_TRY(hipMemsetAsync(L->acc_tau, 0, sizeof(double) * P, L->stream));
  if (L->acc_obj) HIP_TRY(hipMemsetAsync(L->acc_obj, 0, sizeof(double) * L->rplane * L->ncoef, L->stream));
  L->nsamp = 0;
  L->pend_n = 0;
  return HLBM_OK;
}

// Completes the grouped accumulation of a run that ended inside a group (the
// sums are whole again outside hlbm_run_primal).
hlbm_status flush_window(hlbm_lattice_s* L) {
  if (L->pend_n == 0) return HLBM_OK;
  const int count = L->pend_n;
  L->pend_n = 0;
  HIP_TRY(launch_window_flush(L, count));
  return HLBM_OK;
}

// Adds a finished timing block to its kind's statistics and frees the slot.
hlbm_status prof_collect(hlbm_lattice_s* L, int slot) {
  const int kind = L->prof_slot_kind[slot];
  if (kind < 0) return HLBM_OK;
  HIP_TRY(hipEventSynchronize(L->prof_ev[slot][1]));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, L->prof_ev[slot][0], L->prof_ev[slot][1]));
  L->prof_ms[kind] += ms;
  L->prof_sampled[kind] += L->prof_slot_n[slot];
  L->prof_slot_kind[slot] = -1;
  return HLBM_OK;
}

// Collects every block (closing none): statistics up to the last closed block.
hlbm_status prof_collect_all(hlbm_lattice_s* L) {
  for (int i = 0; i < hlbm_lattice_s::kProfSlots; ++i) {
    if (i == L->prof_open) continue;
    hlbm_status s = prof_collect(L, i);
    if (s != HLBM_OK) return s;
  }
  return HLBM_OK;
}

// Launches one sweep of the given kind.  With profiling on, the launches are
// timed in blocks of up to prof_every back-to-back launches of one kind; a
// block never extends past the caller's run of `remaining` consecutive sweeps
// (other kernels follow it), so the block time per launch is the sweep's
// duration in a steady stream of launches, dispatch gaps included.
template <typename F>
hlbm_status timed_launch(hlbm_lattice_s* L, int kind, int64_t remaining, F&& launch) {
  if (L->prof_every <= 0) {
    hipError_t e = launch();
    if (e != hipSuccess) return fail(HLBM_E_DEVICE, "sweep launch: %s", hipGetErrorString(e));
    return HLBM_OK;
  }
  hlbm_status s;
  if (L->prof_open >= 0 && L->prof_open_kind != kind) {  // left open by a failed run
    HIP_TRY(hipEventRecord(L->prof_ev[L->prof_open][1], L->stream));
    L->prof_slot_kind[L->prof_open] = L->prof_open_kind;
    L->prof_open = -1;
  }
  if (L->prof_open < 0) {  // open a block in the next slot of the ring
    const int slot = L->prof_next;
    L->prof_next = (slot + 1) % hlbm_lattice_s::kProfSlots;
    if ((s = prof_collect(L, slot)) != HLBM_OK) return s;  // long finished
    HIP_TRY(hipEventRecord(L->prof_ev[slot][0], L->stream));
    L->prof_open = slot;
    L->prof_open_kind = kind;
    L->prof_slot_n[slot] = 0;
  }
  hipError_t e = launch();
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "sweep launch: %s", hipGetErrorString(e));
  const int slot = L->prof_open;
  L->prof_slot_n[slot] += 1;
  if (L->prof_slot_n[slot] >= L->prof_every || remaining <= 1) {  // close the block
    HIP_TRY(hipEventRecord(L->prof_ev[slot][1], L->stream));
    L->prof_slot_kind[slot] = L->prof_open_kind;
    L->prof_open = -1;
    L->prof_open_kind = -1;
  }
  return HLBM_OK;
}
}  // namespace

extern "C" {

const char* hlbm_last_error(void) { return g_last_error.c_str(); }

const char* hlbm_status_string(hlbm_status s) {
  switch (s) {
    case HLBM_OK: return "ok";
    case HLBM_W_NOT_CONVERGED: return "not converged";
    case HLBM_E_INVALID: return "invalid argument";
    case HLBM_E_OOM: return "out of device memory";
    case HLBM_E_STATE: return "call order violated";
    case HLBM_E_DIVERGED: return "diverged";
    case HLBM_E_DEVICE: return "device error";
  }
  return "unknown status";
}

hlbm_status hlbm_footprint_bytes(const hlbm_desc* desc, int with_window, int with_adjoint, int64_t region_cells,
                                 int32_t objective, uint64_t* bytes) {
  hlbm_status s = validate_desc(desc);
  if (s != HLBM_OK) return s;
  if (!bytes) return fail(HLBM_E_INVALID, "null output");
  const char* why = footprint_of(desc, with_window, with_adjoint, region_cells, objective, BX, BY, bytes);
  return why ? fail(HLBM_E_INVALID, "%s", why) : HLBM_OK;
}

hlbm_status hlbm_device_bytes(hlbm_lattice L, uint64_t* bytes) {
  CHECK_LAT(L);
  if (!bytes) return fail(HLBM_E_INVALID, "null output");
  uint64_t b = 0;
  for (const auto& kv : L->allocs) b += kv.second;
  *bytes = b;
  return HLBM_OK;
}

hlbm_status hlbm_create(const hlbm_desc* desc, hlbm_lattice* out) {
  if (!out) return fail(HLBM_E_INVALID, "null output handle");
  *out = nullptr;
  hlbm_status s = validate_desc(desc);
  if (s != HLBM_OK) return s;
  hlbm_lattice_s* L = new hlbm_lattice_s();
  L->desc = *desc;
  if (L->desc.stencil == HLBM_D2Q9) L->desc.bc_z = HLBM_BC_PERIODIC;
  L->q = q_of(desc->stencil);
  L->dim = dim_of(desc->stencil);
  L->ncoef = ncoef_of(desc->stencil);
  L->nb = nb_of(desc->stencil);
  L->n = (int64_t)desc->nx * desc->ny * desc->nz;
  L->ssize = ssize_of(desc->precision);
  L->dsize = dsize_of(desc->precision);
  L->asize = asize_of(desc->precision);
  L->plane = plane_stride(L->n, L->ssize);
  L->gplane = round_up((int64_t)desc->ny * desc->nz, 128);
  // every kernel indexes plane k at k * plane + cell with cell < n
  if (L->plane < L->n || L->gplane < (int64_t)desc->ny * desc->nz) {
    const long long pl = (long long)L->plane, nn = (long long)L->n;
    delete L;
    return fail(HLBM_E_INVALID, "internal: plane stride %lld < %lld cells", pl, nn);
  }
  L->stream = (hipStream_t)desc->stream;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
      delete L;
      return fail(HLBM_E_DEVICE, "hipGetDevice failed");
    }
    L->device = dev;
    if ((s = scratch_address(dev, &L->noalloc_scratch)) != HLBM_OK) {
      delete L;
      return s;
    }
  }
  // streaming hints for BGK primal sweeps over lattices larger than the
  // 256 MiB Infinity Cache (D2Q9 measured 160 MB slower with them, 320 MB
  // faster); which steps take them is decided per stencil at launch
  const int64_t sweep_bytes = (int64_t)(L->ssize * L->q + L->dsize) * L->plane;
  L->stream_nt = desc->cache_policy == HLBM_CACHE_STREAMING ||
                 (desc->cache_policy == HLBM_CACHE_AUTO && sweep_bytes > ((int64_t)256 << 20));
  auto bail = [&](hlbm_status st) {
    hlbm_destroy(L);
    return st;
  };
  if ((s = lat_alloc(L, &L->f, L->ssize * L->q * L->plane)) != HLBM_OK) return bail(s);
  if ((s = lat_alloc(L, &L->dpor, L->dsize * L->plane)) != HLBM_OK) return bail(s);
  if ((s = lat_alloc(L, &L->ghost, L->ssize * L->q * L->gplane)) != HLBM_OK) return bail(s);
  if ((s = ensure_partials(L, 2 * n_blocks(L) + 8)) != HLBM_OK) return bail(s);
  if (hipHostMalloc((void**)&L->red_host, 4 * sizeof(double)) != hipSuccess)
    return bail(fail(HLBM_E_OOM, "pinned host allocation failed"));
  for (int i = 0; i < hlbm_lattice_s::kProfSlots; ++i) {
    L->prof_slot_kind[i] = -1;
    if (hipEventCreate(&L->prof_ev[i][0]) != hipSuccess || hipEventCreate(&L->prof_ev[i][1]) != hipSuccess)
      return bail(fail(HLBM_E_DEVICE, "event creation failed"));
  }
  if (hipMemsetAsync(L->ghost, 0, L->ssize * L->q * L->gplane, L->stream) != hipSuccess)
    return bail(fail(HLBM_E_DEVICE, "memset failed"));
  // d = 1 everywhere: a cylinder of negative diameter leaves chi = 0
  if (launch_cylinder(L, 0.0, 0.0, -10.0, nullptr, 0, 0.0, 0.0) != hipSuccess)
    return bail(fail(HLBM_E_DEVICE, "porosity fill failed"));
  if (launch_init(L, 1.0, nullptr) != hipSuccess) return bail(fail(HLBM_E_DEVICE, "init failed"));
  if (hipStreamSynchronize(L->stream) != hipSuccess) return bail(fail(HLBM_E_DEVICE, "sync failed"));
  *out = L;
  return HLBM_OK;
}

void hlbm_destroy(hlbm_lattice L) {
  if (!L) return;
  (void)hipStreamSynchronize(L->stream);
  void* bufs[] = {L->f,   L->dpor,  L->ghost, L->acc_rho, L->acc_j, L->acc_f, L->acc_tau, L->acc_obj, L->acc_pend,
                  L->phi, L->prep,  L->src,   L->gdat,    L->oprep, L->pv[0], L->pv[1],   L->snap,
                  L->red, L->usnap, L->probe_buf, L->mea_flag, L->mea_src, L->rcopy, L->tan_f, L->tan_ghost,
                  L->tan_v, L->tan_rec};
  for (void* p : bufs) dev_free(p);
  if (L->red_host) (void)hipHostFree(L->red_host);
  for (int i = 0; i < hlbm_lattice_s::kProfSlots; ++i)
    for (int j = 0; j < 2; ++j)
      if (L->prof_ev[i][j]) (void)hipEventDestroy(L->prof_ev[i][j]);
  delete L;
}

hlbm_status hlbm_synchronize(hlbm_lattice L) {
  CHECK_LAT(L);
  HIP_TRY(hipStreamSynchronize(L->stream));
  return HLBM_OK;
}

hlbm_status hlbm_set_porosity(hlbm_lattice L, const double* d, int64_t n, int32_t mem) {
  CHECK_LAT(L);
  if (!d || n != L->n) return fail(HLBM_E_INVALID, "porosity needs %lld values", (long long)L->n);
  if (mem == HLBM_MEM_HOST) {
    for (int64_t i = 0; i < n; ++i)
      if (!(d[i] >= 0.0 && d[i] <= 1.0)) return fail(HLBM_E_INVALID, "porosity[%lld] = %g outside [0, 1]", (long long)i, d[i]);
  }
  double* dev;
  bool owned;
  hlbm_status s = staging(L, d, n, mem, &dev, &owned);
  if (s != HLBM_OK) return s;
  int* bad = nullptr;
  if ((s = dev_alloc((void**)&bad, sizeof(int))) != HLBM_OK) {
    if (owned) dev_free(dev);
    return s;
  }
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), L->stream);
  if (e == hipSuccess) e = launch_set_porosity(L, dev, bad);
  int hbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  dev_free(bad);
  if (owned) dev_free(dev);
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "set_porosity: %s", hipGetErrorString(e));
  if (hbad) return fail(HLBM_E_INVALID, "porosity outside [0, 1] or not finite");
  L->adj_ready = 0;
  L->mea_dirty = 1;
  return HLBM_OK;
}

hlbm_status hlbm_set_porosity_noalloc(hlbm_lattice L, const double* d, int64_t n) {
  CHECK_LAT(L);
  if (!d || n != L->n) return fail(HLBM_E_INVALID, "porosity needs %lld device values", (long long)L->n);
  int* flag = L->noalloc_scratch;  // element 0 of this device's scratch array
  if (!flag) return fail(HLBM_E_STATE, "no scratch address for the lattice's device");
  k_clear_ints<<<1, 64, 0, L->stream>>>(flag, 1);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_set_porosity(L, d, flag);
  if (e == hipSuccess) e = hipMemcpyAsync(L->red_host, flag, sizeof(int), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "set_porosity_noalloc: %s", hipGetErrorString(e));
  int bad = 0;
  std::memcpy(&bad, L->red_host, sizeof(int));
  L->adj_ready = 0;
  L->mea_dirty = 1;
  if (bad) return fail(HLBM_E_INVALID, "porosity outside [0, 1] or not finite");
  return HLBM_OK;
}

hlbm_status hlbm_build_cylinder(hlbm_lattice L, double xc, double yc, double D, const double* noise, int64_t n,
                                int32_t mem, int32_t noise_mode, double box_half, double d_solid) {
  CHECK_LAT(L);
  if (!std::isfinite(xc) || !std::isfinite(yc) || !(D > 0.0) || !std::isfinite(D))
    return fail(HLBM_E_INVALID, "bad cylinder parameters");
  if (!(d_solid >= 0.0 && d_solid < 1.0)) return fail(HLBM_E_INVALID, "d_solid must be in [0, 1)");
  if (noise_mode < HLBM_NOISE_NONE || noise_mode > HLBM_NOISE_BOX) return fail(HLBM_E_INVALID, "bad noise mode");
  if (noise && n != L->n) return fail(HLBM_E_INVALID, "noise needs %lld values", (long long)L->n);
  double* dev = nullptr;
  bool owned = false;
  if (noise) {
    hlbm_status s = staging(L, noise, n, mem, &dev, &owned);
    if (s != HLBM_OK) return s;
  }
  hipError_t e = launch_cylinder(L, xc, yc, D, dev, noise ? noise_mode : 0, box_half, d_solid);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (owned) dev_free(dev);
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "build_cylinder: %s", hipGetErrorString(e));
  L->adj_ready = 0;
  L->mea_dirty = 1;
  return HLBM_OK;
}

hlbm_status hlbm_init_equilibrium(hlbm_lattice L, double rho0, const double* u, int64_t n, int32_t mem) {
  CHECK_LAT(L);
  if (!(rho0 > 0.0) || !std::isfinite(rho0)) return fail(HLBM_E_INVALID, "rho0 must be positive");
  if (u && n != 3 * L->n) return fail(HLBM_E_INVALID, "u needs 3n = %lld values", (long long)(3 * L->n));
  double* dev = nullptr;
  bool owned = false;
  if (u) {
    hlbm_status s = staging(L, u, 3 * L->n, mem, &dev, &owned);
    if (s != HLBM_OK) return s;
  }
  hipError_t e = launch_init(L, rho0, dev);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (owned) dev_free(dev);
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "init: %s", hipGetErrorString(e));
  L->parity = 0;
  L->steps = 0;
  L->usnap_valid = 0;
  L->adj_ready = 0;
  return zero_window(L);
}

hlbm_status hlbm_set_populations(hlbm_lattice L, const double* f, int64_t n_values, int32_t mem) {
  CHECK_LAT(L);
  if (!f || n_values != L->q * L->n) return fail(HLBM_E_INVALID, "populations need q*n values");
  double* dev;
  bool owned;
  hlbm_status s = staging(L, f, n_values, mem, &dev, &owned);
  if (s != HLBM_OK) return s;
  hipError_t e = launch_scatter(L, dev);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (owned) dev_free(dev);
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "set_populations: %s", hipGetErrorString(e));
  L->parity = 0;
  L->usnap_valid = 0;
  L->adj_ready = 0;
  return HLBM_OK;
}

hlbm_status hlbm_get_populations(hlbm_lattice L, double* f, int64_t n_values, int32_t mem) {
  CHECK_LAT(L);
  if (!f || n_values != L->q * L->n) return fail(HLBM_E_INVALID, "populations need q*n values");
  double* dev;
  bool owned;
  hlbm_status s = staging(L, mem == HLBM_MEM_DEVICE ? f : nullptr, n_values, mem, &dev, &owned);
  if (s != HLBM_OK) return s;
  hipError_t e = launch_gather(L, dev);
  if (e != hipSuccess) {
    if (owned) dev_free(dev);
    return fail(HLBM_E_DEVICE, "gather: %s", hipGetErrorString(e));
  }
  return finish_out(L, dev, f, n_values, mem, owned);
}

hlbm_status hlbm_set_objective(hlbm_lattice L, int32_t kind, const int32_t lo[3], const int32_t hi[3], double u0,
                               double p0) {
  CHECK_LAT(L);
  if (kind < HLBM_OBJ_FFA || kind > HLBM_OBJ_MEA) return fail(HLBM_E_INVALID, "bad objective kind");
  if (kind == HLBM_OBJ_MEA && !(u0 > 0.0)) return fail(HLBM_E_INVALID, "J_MEA needs the surface area A > 0 in u0");
  if (!lo || !hi) return fail(HLBM_E_INVALID, "null region");
  const int nn[3] = {L->desc.nx, L->desc.ny, L->desc.nz};
  for (int a = 0; a < 3; ++a)
    if (lo[a] < 0 || hi[a] >= nn[a] || lo[a] > hi[a]) return fail(HLBM_E_INVALID, "region outside the lattice");
  if (L->desc.bc_x == HLBM_BC_INLET_OUTLET && lo[0] < 1)
    return fail(HLBM_E_INVALID, "region may not include the inlet column");
  if (!std::isfinite(u0) || !std::isfinite(p0)) return fail(HLBM_E_INVALID, "u0/p0 not finite");
  int rn[3];
  for (int a = 0; a < 3; ++a) rn[a] = hi[a] - lo[a] + 1;
  const int64_t rp = round_up((int64_t)rn[0] * rn[1] * rn[2], 128);
  if (rp > L->rplane) {
    lat_free(L, L->acc_obj);
    lat_free(L, L->src);
    lat_free(L, L->mea_flag);
    lat_free(L, L->mea_src);
    lat_free(L, L->rcopy);
    L->mea_src = nullptr;
    L->acc_obj = nullptr;
    L->src = nullptr;
    L->mea_flag = nullptr;
    L->rcopy = nullptr;
    L->rplane = 0;
  }
  hlbm_status s;
  if ((s = lat_alloc(L, (void**)&L->acc_obj, sizeof(double) * rp * L->ncoef)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, (void**)&L->src, sizeof(double) * rp * L->ncoef)) != HLBM_OK) return s;
  L->mea_dirty = 1;
  L->rplane = rp > L->rplane ? rp : L->rplane;
  if (kind == HLBM_OBJ_MEA) {  // sized for the plane stride the kernels index with
    lat_free(L, L->mea_flag);
    lat_free(L, L->mea_src);
    L->mea_flag = nullptr;
    L->mea_src = nullptr;
    if ((s = lat_alloc(L, (void**)&L->mea_flag, L->rplane)) != HLBM_OK) return s;
    if ((s = lat_alloc(L, (void**)&L->mea_src, sizeof(double) * L->q * L->rplane)) != HLBM_OK) return s;
  }
  if (region_copy_used((int64_t)rn[0] * rn[1] * rn[2], L->n, kind)) {
    if ((s = lat_alloc(L, &L->rcopy, L->asize * (size_t)region_copy_stride(L->q, (int)L->asize) * (size_t)L->rplane)) !=
        HLBM_OK)
      return s;
  } else {
    lat_free(L, L->rcopy);
    L->rcopy = nullptr;
  }
  L->obj_kind = kind;
  for (int a = 0; a < 3; ++a) {
    L->lo[a] = lo[a];
    L->rn[a] = rn[a];
  }
  L->u0 = u0;
  L->p0 = p0;
  L->obj_set = 1;
  L->adj_ready = 0;
  // a new objective starts a new window
  return zero_window(L);
}

hlbm_status hlbm_window_reset(hlbm_lattice L) {
  CHECK_LAT(L);
  L->adj_ready = 0;
  return zero_window(L);
}

hlbm_status hlbm_window_count(hlbm_lattice L, int64_t* samples) {
  CHECK_LAT(L);
  if (!samples) return fail(HLBM_E_INVALID, "null output");
  *samples = L->nsamp;
  return HLBM_OK;
}

hlbm_status hlbm_profile_enable(hlbm_lattice L, int32_t every) {
  CHECK_LAT(L);
  if (every < 0) return fail(HLBM_E_INVALID, "every must be >= 0");
  // drop what is pending: an open block is closed at its next launch only,
  // so discard it and every recorded block
  HIP_TRY(hipStreamSynchronize(L->stream));
  for (int i = 0; i < hlbm_lattice_s::kProfSlots; ++i) L->prof_slot_kind[i] = -1;
  L->prof_open = -1;
  L->prof_open_kind = -1;
  L->prof_every = every;
  for (int k = 0; k < 3; ++k) {
    L->prof_sampled[k] = 0;
    L->prof_ms[k] = 0.0;
  }
  return HLBM_OK;
}

hlbm_status hlbm_profile_get(hlbm_lattice L, int32_t kind, double* mean_us, int64_t* sampled) {
  CHECK_LAT(L);
  if (kind < 0 || kind > 2) return fail(HLBM_E_INVALID, "kind must be 0, 1 or 2");
  hlbm_status s = prof_collect_all(L);
  if (s != HLBM_OK) return s;
  const int64_t n = L->prof_sampled[kind];
  if (mean_us) *mean_us = n ? 1e3 * L->prof_ms[kind] / (double)n : 0.0;
  if (sampled) *sampled = n;
  return HLBM_OK;
}

hlbm_status hlbm_set_probe(hlbm_lattice L, int32_t x, int32_t y, int32_t z, int64_t capacity) {
  CHECK_LAT(L);
  if (capacity < 0) return fail(HLBM_E_INVALID, "capacity must be >= 0");
  if (capacity == 0) {
    HIP_TRY(hipStreamSynchronize(L->stream));
    lat_free(L, L->probe_buf);
    L->probe_buf = nullptr;
    L->probe_cap = L->probe_n = 0;
    L->probe_cell = -1;
    return HLBM_OK;
  }
  if (x < 0 || x >= L->desc.nx || y < 0 || y >= L->desc.ny || z < 0 || z >= L->desc.nz)
    return fail(HLBM_E_INVALID, "probe outside the lattice");
  if (capacity != L->probe_cap) {
    HIP_TRY(hipStreamSynchronize(L->stream));
    lat_free(L, L->probe_buf);
    L->probe_buf = nullptr;
    hlbm_status s = lat_alloc(L, (void**)&L->probe_buf, sizeof(double) * (size_t)capacity);
    if (s != HLBM_OK) return s;
  }
  L->probe_cap = capacity;
  L->probe_n = 0;
  L->probe_cell = (int64_t)x + (int64_t)L->desc.nx * ((int64_t)y + (int64_t)L->desc.ny * z);
  return HLBM_OK;
}

hlbm_status hlbm_get_probe(hlbm_lattice L, double* out, int64_t capacity, int64_t* count) {
  CHECK_LAT(L);
  if (!out || !count) return fail(HLBM_E_INVALID, "null output");
  if (!L->probe_buf) return fail(HLBM_E_STATE, "no probe set");
  const int64_t n = L->probe_n < L->probe_cap ? L->probe_n : L->probe_cap;
  if (capacity < n) return fail(HLBM_E_INVALID, "output holds %lld values, %lld needed", (long long)capacity, (long long)n);
  std::vector<double> ring((size_t)L->probe_cap);
  HIP_TRY(hipMemcpyAsync(ring.data(), L->probe_buf, sizeof(double) * L->probe_cap, hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(hipStreamSynchronize(L->stream));
  const int64_t start = (L->probe_n <= L->probe_cap) ? 0 : (L->probe_n % L->probe_cap);
  for (int64_t i = 0; i < n; ++i) out[i] = ring[(size_t)((start + i) % L->probe_cap)];
  *count = n;
  return HLBM_OK;
}


hlbm_status hlbm_run_primal(hlbm_lattice L, int64_t n_steps, int32_t accumulate, double steady_tol,
                            int64_t check_every, int64_t* steps_done) {
  CHECK_LAT(L);
  if (steps_done) *steps_done = 0;
  if (n_steps < 0) return fail(HLBM_E_INVALID, "negative step count");
  if (!(steady_tol >= 0.0)) return fail(HLBM_E_INVALID, "steady_tol must be >= 0");
  if (check_every <= 0) check_every = 100;
  hlbm_status s;
  if ((s = ensure_mea(L)) != HLBM_OK) return s;
  if (accumulate) {
    if ((s = ensure_window(L)) != HLBM_OK) return s;
  }
  if (steady_tol > 0.0) {
    if ((s = lat_alloc(L, (void**)&L->usnap, sizeof(double) * L->plane * L->dim)) != HLBM_OK) return s;
  }
  const int64_t nb = n_blocks(L);
  // snapshot of u at the start of a steady run
  if (steady_tol > 0.0) {
    int nbl = 0;
    HIP_TRY(launch_steady_check(L, 1, L->red, &nbl));
    L->usnap_valid = 1;
  }
  (void)nb;
  int64_t done = 0;
  hlbm_status result = HLBM_OK;
  bool converged = false;
  // chunks between checks are timed as one batch
  while (done < n_steps) {
    int64_t chunk = n_steps - done;
    if (steady_tol > 0.0 && chunk > check_every) chunk = check_every;
    for (int64_t k = 0; k < chunk; ++k) {
      s = timed_launch(L, accumulate ? 1 : 0, chunk - k,
                       [&]() { return launch_primal_step(L, accumulate); });
      if (s != HLBM_OK) return s;
      L->parity ^= 1;
      L->steps += 1;
      if (accumulate) L->nsamp += 1;
      if (L->probe_buf) L->probe_n += 1;
    }
    done += chunk;
    if (steady_tol > 0.0) {
      int nbl = 0;
      HIP_TRY(launch_steady_check(L, 0, L->red, &nbl));
      double mm[2];
      if ((s = reduce_to_host(L, nbl, 1, mm)) != HLBM_OK) return s;
      if (!std::isfinite(mm[0]) || !std::isfinite(mm[1])) {
        if (steps_done) *steps_done = done;
        if ((s = flush_window(L)) != HLBM_OK) return s;
        return fail(HLBM_E_DIVERGED, "non-finite velocity after %lld steps", (long long)L->steps);
      }
      if (mm[0] <= steady_tol * mm[1]) {
        converged = true;
        break;
      }
    }
  }
  if (steps_done) *steps_done = done;
  if ((s = flush_window(L)) != HLBM_OK) return s;
  if (steady_tol > 0.0 && !converged) result = HLBM_W_NOT_CONVERGED;
  L->adj_ready = 0;
  return result;
}

hlbm_status hlbm_run_tangent(hlbm_lattice L, const double* v, int64_t n, int32_t mem, int64_t n_steps,
                             int64_t record_every, double* out) {
  CHECK_LAT(L);
  if (L->desc.precision != HLBM_FP64) return fail(HLBM_E_INVALID, "the tangent runs on FP64 lattices");
  if (L->desc.smagorinsky_cs > 0.0) return fail(HLBM_E_INVALID, "the tangent has no Smagorinsky closure");
  if (L->desc.collision != HLBM_COLL_BGK) return fail(HLBM_E_INVALID, "the tangent is written for the BGK collision");
  if (!L->obj_set) return fail(HLBM_E_STATE, "no objective set");
  if (!v || n != L->n) return fail(HLBM_E_INVALID, "v needs %lld values", (long long)L->n);
  if (n_steps < 0 || record_every < 1) return fail(HLBM_E_INVALID, "bad step counts");
  const int64_t nrec = n_steps / record_every;
  if (nrec > 0 && !out) return fail(HLBM_E_INVALID, "null output");
  hlbm_status s;
  if ((s = ensure_mea(L)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, (void**)&L->tan_f, sizeof(double) * L->q * L->plane)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, (void**)&L->tan_ghost, sizeof(double) * L->q * L->gplane)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, (void**)&L->tan_v, sizeof(double) * L->plane)) != HLBM_OK) return s;
  if (nrec > L->tan_rec_cap) {
    lat_free(L, L->tan_rec);
    L->tan_rec = nullptr;
    L->tan_rec_cap = 0;
    if ((s = lat_alloc(L, (void**)&L->tan_rec, sizeof(double) * 2 * nrec)) != HLBM_OK) return s;
    L->tan_rec_cap = nrec;
  }
  HIP_TRY(hipMemcpyAsync(L->tan_v, v, sizeof(double) * L->n,
                         mem == HLBM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, L->stream));
  // seeding: fdot = 0 at the current state
  HIP_TRY(hipMemsetAsync(L->tan_f, 0, sizeof(double) * L->q * L->plane, L->stream));
  HIP_TRY(hipMemsetAsync(L->tan_ghost, 0, sizeof(double) * L->q * L->gplane, L->stream));
  const int64_t nb = n_blocks(L);
  int64_t r = 0;
  for (int64_t k = 0; k < n_steps; ++k) {
    HIP_TRY(launch_tangent_step(L));
    L->parity ^= 1;
    L->steps += 1;
    if ((k + 1) % record_every == 0) {
      int nbl = 0;
      HIP_TRY(launch_tangent_objective(L, L->red, &nbl));
      HIP_TRY(launch_finalize_sum(L, L->red, nbl, L->tan_rec + 2 * r));
      HIP_TRY(launch_finalize_sum(L, L->red + nb, nbl, L->tan_rec + 2 * r + 1));
      r += 1;
    }
  }
  if (nrec > 0)
    HIP_TRY(hipMemcpyAsync(out, L->tan_rec, sizeof(double) * 2 * nrec, hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(hipStreamSynchronize(L->stream));
  L->adj_ready = 0;
  L->usnap_valid = 0;
  return HLBM_OK;
}

hlbm_status hlbm_get_objective(hlbm_lattice L, int32_t which, double* J) {
  CHECK_LAT(L);
  if (!J) return fail(HLBM_E_INVALID, "null output");
  if (!L->obj_set) return fail(HLBM_E_STATE, "no objective set");
  if (which == 1 && L->nsamp == 0) return fail(HLBM_E_STATE, "empty window");
  if (which != 0 && which != 1) return fail(HLBM_E_INVALID, "which must be 0 or 1");
  hlbm_status s = ensure_mea(L);
  if (s != HLBM_OK) return s;
  int nbl = 0;
  HIP_TRY(launch_objective(L, which, L->red, &nbl));
  return reduce_to_host(L, nbl, 0, J);
}

hlbm_status hlbm_solve_adjoint(hlbm_lattice L, const hlbm_adjoint_opts* o, hlbm_adjoint_report* rep) {
  CHECK_LAT(L);
  if (!o || o->struct_size != sizeof(hlbm_adjoint_opts)) return fail(HLBM_E_INVALID, "bad adjoint options");
  if (rep) {
    rep->iters = 0;
    rep->residual = -1.0;
  }
  if (o->source != HLBM_SOURCE_STEADY && o->source != HLBM_SOURCE_MEAN) return fail(HLBM_E_INVALID, "bad source");
  if (o->turb != HLBM_TURB_FROZEN && o->turb != HLBM_TURB_DIFFERENTIATED) return fail(HLBM_E_INVALID, "bad turb");
  if (o->max_iters < 0 || !(o->tol >= 0.0)) return fail(HLBM_E_INVALID, "bad iteration limits");
  const double tau_adj = o->tau_adj > 0.0 ? o->tau_adj : L->desc.tau;
  if (!(tau_adj > 0.5)) return fail(HLBM_E_INVALID, "tau_adj must exceed 1/2");
  if (!L->obj_set) return fail(HLBM_E_STATE, "no objective set");
  {
    hlbm_status s0 = ensure_mea(L);
    if (s0 != HLBM_OK) return s0;
  }
  const bool smag = L->desc.smagorinsky_cs > 0.0;
  if (o->source == HLBM_SOURCE_MEAN) {
    if (L->nsamp == 0 || !L->acc_rho) return fail(HLBM_E_STATE, "mean-flow adjoint needs a non-empty window");
    if (smag && o->turb == HLBM_TURB_DIFFERENTIATED && !L->acc_f)
      return fail(HLBM_E_STATE, "differentiated closure needs track_mean_populations");
    if (L->desc.collision == HLBM_COLL_HRR && !L->acc_f)
      return fail(HLBM_E_STATE, "the HRR mean-flow adjoint needs track_mean_populations (mean second moments)");
  }
  const int P = 0;
  (void)P;
  const int64_t plane = L->plane;
  const size_t as = L->asize;
  hlbm_status s;
  const int nprep = L->dim + 2 + L->q + L->nb;
  if ((s = lat_alloc(L, &L->phi, as * L->q * plane)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, &L->prep, as * nprep * plane)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, (void**)&L->gdat, sizeof(double) * (L->dim + 2) * plane)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, (void**)&L->oprep, sizeof(double) * (1 + L->dim) * L->gplane)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, &L->pv[0], as * L->q * L->gplane)) != HLBM_OK) return s;
  if ((s = lat_alloc(L, &L->pv[1], as * L->q * L->gplane)) != HLBM_OK) return s;
  if (o->tol > 0.0 && (s = lat_alloc(L, &L->snap, as * L->q * plane)) != HLBM_OK) return s;
  L->nprep = nprep;
  const bool turb_diff = smag && o->turb == HLBM_TURB_DIFFERENTIATED;
  if (o->restart || !L->adj_ready || L->adj_diff != (int)turb_diff) {
    HIP_TRY(hipMemsetAsync(L->prep, 0, as * nprep * plane, L->stream));
    HIP_TRY(hipMemsetAsync(L->gdat, 0, sizeof(double) * (L->dim + 2) * plane, L->stream));
    HIP_TRY(hipMemsetAsync(L->src, 0, sizeof(double) * L->rplane * L->ncoef, L->stream));
    HIP_TRY(launch_adjoint_prep(L, o->source, tau_adj, o->turb));
    HIP_TRY(hipMemsetAsync(L->phi, 0, as * L->q * plane, L->stream));
    HIP_TRY(hipMemsetAsync(L->pv[0], 0, as * L->q * L->gplane, L->stream));
    HIP_TRY(hipMemsetAsync(L->pv[1], 0, as * L->q * L->gplane, L->stream));
    L->pvcur = 0;
    L->adj_iters = 0;
    L->adj_ready = 1;
    L->adj_les = smag ? 1 : 0;
    L->adj_diff = turb_diff ? 1 : 0;
    L->adj_omega = 1.0 / tau_adj;
  }
  int64_t iters = o->max_iters + (o->max_iters & 1);
  int64_t M = o->check_every > 0 ? o->check_every : 100;
  M += (M & 1);
  hlbm_status result = HLBM_OK;
  double res = -1.0;
  if (o->tol > 0.0) {
    int nbl = 0;
    HIP_TRY(launch_adjoint_residual(L, 1, L->red, &nbl));
  }
  int64_t done = 0;
  bool converged = false;
  double min_res = HUGE_VAL;
  while (done < iters) {
    int64_t chunk = iters - done;
    if (o->tol > 0.0 && chunk > M) chunk = M;
    for (int64_t k = 0; k < chunk; ++k) {
      s = timed_launch(L, 2, chunk - k, [&]() { return launch_adjoint_step(L); });
      if (s != HLBM_OK) return s;
      L->pvcur ^= 1;
      L->adj_iters += 1;
    }
    done += chunk;
    if (o->tol > 0.0) {
      int nbl = 0;
      HIP_TRY(launch_adjoint_residual(L, 0, L->red, &nbl));
      double mm[2];
      if ((s = reduce_to_host(L, nbl, 1, mm)) != HLBM_OK) return s;
      const StopDecision dec = adjoint_stop(mm[0], mm[1], o->tol, &min_res, &res);
      if (dec == STOP_DIVERGED) {
        if (rep) {
          rep->iters = done;
          rep->residual = res;
        }
        return fail(HLBM_E_DIVERGED, "adjoint diverged after %lld iterations (residual %g, smallest %g)",
                    (long long)L->adj_iters, res, min_res);
      }
      if (dec == STOP_CONVERGED) {
        converged = true;
        break;
      }
    }
  }
  if (o->tol > 0.0) HIP_TRY(hipStreamSynchronize(L->stream));
  if (rep) {
    rep->iters = done;
    rep->residual = res;
  }
  if (o->tol > 0.0 && !converged) result = HLBM_W_NOT_CONVERGED;
  return result;
}

hlbm_status hlbm_get_gradient(hlbm_lattice L, double* g, int64_t n, int32_t mem) {
  CHECK_LAT(L);
  if (!g || n != L->n) return fail(HLBM_E_INVALID, "gradient needs n values");
  if (!L->adj_ready) return fail(HLBM_E_STATE, "solve the adjoint first");
  double* dev;
  bool owned;
  hlbm_status s = staging(L, mem == HLBM_MEM_DEVICE ? g : nullptr, n, mem, &dev, &owned);
  if (s != HLBM_OK) return s;
  hipError_t e = launch_gradient(L, dev);
  if (e != hipSuccess) {
    if (owned) dev_free(dev);
    return fail(HLBM_E_DEVICE, "gradient: %s", hipGetErrorString(e));
  }
  return finish_out(L, dev, g, n, mem, owned);
}

hlbm_status hlbm_get_adjoint(hlbm_lattice L, double* phi, int64_t n_values, int32_t mem) {
  CHECK_LAT(L);
  if (!phi || n_values != L->q * L->n) return fail(HLBM_E_INVALID, "adjoint needs q*n values");
  if (!L->adj_ready) return fail(HLBM_E_STATE, "solve the adjoint first");
  double* dev;
  bool owned;
  hlbm_status s = staging(L, mem == HLBM_MEM_DEVICE ? phi : nullptr, n_values, mem, &dev, &owned);
  if (s != HLBM_OK) return s;
  hipError_t e = launch_adjoint_gather(L, dev);
  if (e != hipSuccess) {
    if (owned) dev_free(dev);
    return fail(HLBM_E_DEVICE, "adjoint gather: %s", hipGetErrorString(e));
  }
  return finish_out(L, dev, phi, n_values, mem, owned);
}

}  // extern "C"

namespace {
template <typename Dd>
__global__ void k_porosity_out(const Dd* __restrict__ d, double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)d[i];
}
}  // namespace

extern "C" hlbm_status hlbm_get_field(hlbm_lattice L, int32_t field, double* out, int64_t n_values, int32_t mem) {
  CHECK_LAT(L);
  if (!out) return fail(HLBM_E_INVALID, "null output");
  const bool vec = (field == HLBM_FIELD_U || field == HLBM_FIELD_MEAN_U);
  if (field < HLBM_FIELD_RHO || field > HLBM_FIELD_MEAN_TAU) return fail(HLBM_E_INVALID, "bad field");
  const int64_t need = vec ? 3 * L->n : L->n;
  if (n_values != need) return fail(HLBM_E_INVALID, "field needs %lld values", (long long)need);
  if ((field == HLBM_FIELD_MEAN_RHO || field == HLBM_FIELD_MEAN_U || field == HLBM_FIELD_MEAN_TAU) &&
      (L->nsamp == 0 || !L->acc_rho))
    return fail(HLBM_E_STATE, "empty window");
  if (field == HLBM_FIELD_MEAN_TAU && !L->acc_tau) return fail(HLBM_E_STATE, "no Smagorinsky closure");
  double* dev;
  bool owned;
  hlbm_status s = staging(L, mem == HLBM_MEM_DEVICE ? out : nullptr, need, mem, &dev, &owned);
  if (s != HLBM_OK) return s;
  hipError_t e = hipSuccess;
  if (field == HLBM_FIELD_RHO)
    e = launch_moments(L, dev, nullptr);
  else if (field == HLBM_FIELD_U)
    e = launch_moments(L, nullptr, dev);
  else if (field == HLBM_FIELD_POROSITY) {
    const int64_t nb = (L->n + 255) / 256;
    if (L->desc.precision == HLBM_FP64)
      k_porosity_out<double><<<dim3((unsigned)nb), dim3(256), 0, L->stream>>>((const double*)L->dpor, dev, L->n);
    else
      k_porosity_out<float><<<dim3((unsigned)nb), dim3(256), 0, L->stream>>>((const float*)L->dpor, dev, L->n);
    e = hipGetLastError();
  } else {
    e = launch_mean_fields(L, field, dev);
  }
  if (e != hipSuccess) {
    if (owned) dev_free(dev);
    return fail(HLBM_E_DEVICE, "get_field: %s", hipGetErrorString(e));
  }
  return finish_out(L, dev, out, need, mem, owned);
}

extern "C" hlbm_status hlbm_bytes_per_update(hlbm_lattice L, double* primal, double* primal_window, double* adjoint) {
  CHECK_LAT(L);
  const double q = L->q, dim = L->dim;
  const double ss = (double)L->ssize, ds = (double)L->dsize, as = (double)L->asize;
  const double rfrac = L->obj_set ? (double)L->rn[0] * L->rn[1] * L->rn[2] / (double)L->n : 0.0;
  const bool smag = L->desc.smagorinsky_cs > 0.0;
  // primal: read + write every population once, read d
  const double p = 2.0 * q * ss + ds;
  // window: FP64 read-modify-write of the m dense sums rho, j (+ f, tau) and
  // the region terms; with the grouped accumulation (FP32 arithmetic) one
  // read-modify-write per group of K steps, the first K - 1 writing m FP32
  // values that the last reads: (16 + 8 (K - 1)) / K per sum and step
  double m = 1.0 + dim;
  if (L->desc.track_mean_populations) m += q;
  if (smag) m += 1.0;
  const double K = PEND_GROUP;
  double pw = p + (L->desc.precision != HLBM_FP64 ? (16.0 + 8.0 * (K - 1.0)) / K : 16.0) * m;
  pw += rfrac * 16.0 * L->ncoef;
  // adjoint: read + write phi, read the frozen coefficients and the source
  const double nsym = dim == 2 ? 3.0 : 6.0;
  double a = 2.0 * q * as;
  if (L->desc.collision == HLBM_COLL_HRR) {
    a += as * (dim + 3.0 + nsym);  // rho, j, d, omega, a2
    if (L->adj_diff) a += as * nsym;
  } else {
    a += as * (dim + 1.0);  // u~, d
    if (smag) a += as;      // omega per cell
    if (L->adj_diff) a += as * (q + L->nb);
  }
  a += rfrac * 8.0 * (L->obj_kind == HLBM_OBJ_MEA ? q : L->ncoef - 2);
  if (primal) *primal = p;
  if (primal_window) *primal_window = pw;
  if (adjoint) *adjoint = a;
  return HLBM_OK;
}

extern "C" hlbm_status hlbm_copy_probe(hlbm_lattice L, int32_t pattern, int32_t streaming, int64_t n_launches,
                                       double* us_per_launch) {
  CHECK_LAT(L);
  if (pattern < 0 || pattern > 2) return fail(HLBM_E_INVALID, "pattern must be 0, 1 or 2");
  if (n_launches < 1 || !us_per_launch) return fail(HLBM_E_INVALID, "need n_launches >= 1 and an output");
  // pattern 2 writes a second population array, held only for this call
  void* second = nullptr;
  if (pattern == 2) {
    hlbm_status s = dev_alloc(&second, L->ssize * (size_t)L->q * (size_t)L->plane);
    if (s != HLBM_OK) return s;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipEventRecord(ev[0], L->stream);
  // the porosity test that guards the sink is never true (d is in [0, 1])
  for (int64_t k = 0; k < n_launches && e == hipSuccess; ++k)
    e = launch_copy_probe(L, pattern, streaming != 0, (int*)L->red, second);
  if (e == hipSuccess) e = hipEventRecord(ev[1], L->stream);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  if (ev[0]) (void)hipEventDestroy(ev[0]);
  if (ev[1]) (void)hipEventDestroy(ev[1]);
  if (second) {
    (void)hipStreamSynchronize(L->stream);
    dev_free(second);
  }
  if (e != hipSuccess) return fail(HLBM_E_DEVICE, "copy probe: %s", hipGetErrorString(e));
  *us_per_launch = 1e3 * (double)ms / (double)n_launches;
  return HLBM_OK;
}

extern "C" hlbm_status hlbm_reconfigure(hlbm_lattice L, double tau, double cs, double u_in) {
  CHECK_LAT(L);
  hlbm_desc d = L->desc;
  d.tau = tau;
  d.smagorinsky_cs = cs;
  d.u_in = u_in;
  hlbm_status s = validate_desc(&d);
  if (s != HLBM_OK) return s;
  if (cs > 0.0 && L->desc.smagorinsky_cs == 0.0 && L->acc_rho && !L->acc_tau) {
    if ((s = lat_alloc(L, (void**)&L->acc_tau, sizeof(double) * L->plane)) != HLBM_OK) return s;
    HIP_TRY(hipMemsetAsync(L->acc_tau, 0, sizeof(double) * L->plane, L->stream));
  }
  L->desc.tau = tau;
  L->desc.smagorinsky_cs = cs;
  L->desc.u_in = u_in;
  L->adj_ready = 0;
  return HLBM_OK;
}

extern "C" hlbm_status hlbm_group_create(void* stream, hlbm_group* out) {
  if (!out) return fail(HLBM_E_INVALID, "null output");
  hlbm_group_s* g = new hlbm_group_s();
  g->stream = (hipStream_t)stream;
  *out = g;
  return HLBM_OK;
}

extern "C" void hlbm_group_destroy(hlbm_group g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  dev_free(g->tab_primal);
  dev_free(g->tab_adjoint);
  dev_free(g->first_primal);
  dev_free(g->first_adjoint);
  delete[] g->members;
  delete[] g->modes;
  delete[] g->counts0;
  delete g;
}

extern "C" hlbm_status hlbm_group_set(hlbm_group g, const hlbm_lattice* lats, const int32_t* modes, int32_t count) {
  if (!g) return fail(HLBM_E_INVALID, "null group");
  if (count < 0 || (count > 0 && (!lats || !modes))) return fail(HLBM_E_INVALID, "bad member list");
  for (int i = 0; i < count; ++i) {
    hlbm_lattice_s* L = lats[i];
    if (!L) return fail(HLBM_E_INVALID, "null member %d", i);
    if (modes[i] < HLBM_GROUP_PRIMAL || modes[i] > HLBM_GROUP_ADJOINT) return fail(HLBM_E_INVALID, "bad mode");
    if (L->desc.stencil != lats[0]->desc.stencil || L->desc.precision != lats[0]->desc.precision ||
        L->desc.collision != lats[0]->desc.collision)
      return fail(HLBM_E_INVALID, "members must share stencil, precision and collision model");
    if (modes[i] == HLBM_GROUP_ADJOINT && !L->adj_ready)
      return fail(HLBM_E_STATE, "member %d: adjoint not prepared", i);
    for (int j = 0; j < i; ++j)
      if (lats[j] == L) return fail(HLBM_E_INVALID, "member %d listed twice", i);
  }
  HIP_TRY(hipStreamSynchronize(g->stream));
  hlbm_status s;
  for (int i = 0; i < count; ++i) {
    if ((s = ensure_mea(lats[i])) != HLBM_OK) return s;
    if (modes[i] == HLBM_GROUP_PRIMAL_WINDOW && (s = ensure_window(lats[i])) != HLBM_OK) return s;
    HIP_TRY(hipStreamSynchronize(lats[i]->stream));
  }
  const size_t ps = packed_primal_size(), as = packed_adjoint_size();
  std::vector<unsigned char> tp, ta;
  std::vector<int> fp, fa;
  int bp = 0, ba = 0;
  for (int i = 0; i < count; ++i) {
    hlbm_lattice_s* L = lats[i];
    const int blocks = tiles_x_of(L) * tiles_y_of(L) * L->desc.nz;
    if (modes[i] == HLBM_GROUP_ADJOINT) {
      ta.resize(ta.size() + as);
      fill_packed_adjoint(L, ba, ta.data() + ta.size() - as);
      fa.push_back(ba);
      ba += blocks;
    } else {
      tp.resize(tp.size() + ps);
      fill_packed_primal(L, modes[i] == HLBM_GROUP_PRIMAL_WINDOW, bp, tp.data() + tp.size() - ps);
      fp.push_back(bp);
      bp += blocks;
    }
  }
  auto upload = [&](std::vector<unsigned char>& t, std::vector<int>& f, size_t esz, void** tab, int** first,
                    size_t* cap) -> hlbm_status {
    const size_t m = f.size();
    if (m == 0) return HLBM_OK;
    if (m > *cap) {
      dev_free(*tab);
      dev_free(*first);
      *tab = nullptr;
      *first = nullptr;
      *cap = 0;
      hlbm_status st;
      if ((st = dev_alloc(tab, esz * m)) != HLBM_OK) return st;
      if ((st = dev_alloc((void**)first, sizeof(int) * m)) != HLBM_OK) return st;
      *cap = m;
    }
    HIP_TRY(hipMemcpyAsync(*tab, t.data(), esz * m, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(*first, f.data(), sizeof(int) * m, hipMemcpyHostToDevice, g->stream));
    return HLBM_OK;
  };
  if ((s = upload(tp, fp, ps, &g->tab_primal, &g->first_primal, &g->cap_primal)) != HLBM_OK) return s;
  if ((s = upload(ta, fa, as, &g->tab_adjoint, &g->first_adjoint, &g->cap_adjoint)) != HLBM_OK) return s;
  HIP_TRY(hipStreamSynchronize(g->stream));  // host tables go out of scope
  delete[] g->members;
  delete[] g->modes;
  delete[] g->counts0;
  g->members = count ? new hlbm_lattice_s*[count] : nullptr;
  g->modes = count ? new int32_t[count] : nullptr;
  g->counts0 = count ? new int64_t[count] : nullptr;
  for (int i = 0; i < count; ++i) {
    g->members[i] = lats[i];
    g->modes[i] = modes[i];
    g->counts0[i] = modes[i] == HLBM_GROUP_ADJOINT ? lats[i]->adj_iters : lats[i]->steps;
  }
  g->count = count;
  g->n_primal = (int)fp.size();
  g->n_adjoint = (int)fa.size();
  g->blocks_primal = bp;
  g->blocks_adjoint = ba;
  g->stencil = count ? lats[0]->desc.stencil : -1;
  g->precision = count ? lats[0]->desc.precision : -1;
  g->collision = count ? lats[0]->desc.collision : 0;
  g->steps_since_set = 0;
  return HLBM_OK;
}

namespace {
// The n packed launches of a step run (each step one primal and/or one
// adjoint launch; AA parity from the step count since the last set).
hipError_t enqueue_group_steps(hlbm_group_s* g, int64_t n) {
  for (int64_t k = 0; k < n; ++k) {
    const int step = (int)((g->steps_since_set + k) & 1);
    hipError_t e;
    if (g->n_primal > 0 &&
        (e = launch_primal_packed(g->stream, g->stencil, g->precision, g->collision, g->tab_primal,
                                  g->first_primal, g->n_primal, g->blocks_primal, step)) != hipSuccess)
      return e;
    if (g->n_adjoint > 0 &&
        (e = launch_adjoint_packed(g->stream, g->stencil, g->precision, g->collision, g->tab_adjoint,
                                   g->first_adjoint, g->n_adjoint, g->blocks_adjoint, step)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Runs of at least this many steps on a group's own stream are launched as
// one HIP graph: the host then enqueues one launch per run instead of one
// per kernel (the packed kernels of small lattices take ~5 us, about as long
// as enqueuing one launch).
constexpr int64_t kGraphMinSteps = 16;

// Captures the run into a graph unless the last one had the same launch
// arguments, then launches it.  Returns false (nothing enqueued) if capture
// is not possible, so that the caller launches the kernels directly.
bool launch_group_graph(hlbm_group_s* g, int64_t n) {
  const uint64_t key[13] = {(uint64_t)g->stencil, (uint64_t)g->precision, (uint64_t)g->collision,
                            (uint64_t)(uintptr_t)g->tab_primal, (uint64_t)(uintptr_t)g->first_primal,
                            (uint64_t)g->n_primal, (uint64_t)g->blocks_primal,
                            (uint64_t)(uintptr_t)g->tab_adjoint, (uint64_t)(uintptr_t)g->first_adjoint,
                            (uint64_t)g->n_adjoint, (uint64_t)g->blocks_adjoint, (uint64_t)n,
                            (uint64_t)(g->steps_since_set & 1)};
  if (!g->gexec || std::memcmp(key, g->gkey, sizeof key) != 0) {
    if (g->gexec) {
      (void)hipGraphExecDestroy(g->gexec);
      g->gexec = nullptr;
    }
    if (hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    const hipError_t e = enqueue_group_steps(g, n);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(g->stream, &graph);
    hipGraphExec_t exec = nullptr;
    const bool ok = e == hipSuccess && e2 == hipSuccess && graph &&
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!ok) {
      (void)hipGetLastError();
      return false;
    }
    g->gexec = exec;
    std::memcpy(g->gkey, key, sizeof key);
  }
  return hipGraphLaunch(g->gexec, g->stream) == hipSuccess;
}
}  // namespace

extern "C" hlbm_status hlbm_group_step(hlbm_group g, int64_t n) {
  if (!g) return fail(HLBM_E_INVALID, "null group");
  if (n < 0) return fail(HLBM_E_INVALID, "negative step count");
  // the packed tables hold each member's AA parity (or adjoint buffer) as of
  // the set: a member advanced by any other call since then would be stepped
  // in the wrong layout
  for (int i = 0; i < g->count; ++i) {
    const hlbm_lattice_s* L = g->members[i];
    const int64_t now = g->modes[i] == HLBM_GROUP_ADJOINT ? L->adj_iters : L->steps;
    if (now != g->counts0[i] + g->steps_since_set)
      return fail(HLBM_E_STATE, "member %d was advanced outside the group since hlbm_group_set", i);
  }
  bool done = false;
  if (n >= kGraphMinSteps && g->stream != nullptr && g->graph_ok) {
    done = launch_group_graph(g, n);
    if (!done) g->graph_ok = false;  // from now on the plain launches below
  }
  if (!done) HIP_TRY(enqueue_group_steps(g, n));
  for (int i = 0; i < g->count; ++i) {
    hlbm_lattice_s* L = g->members[i];
    if (g->modes[i] == HLBM_GROUP_ADJOINT) {
      L->adj_iters += n;
      L->pvcur ^= (int)(n & 1);
    } else {
      L->parity ^= (int)(n & 1);
      L->steps += n;
      if (g->modes[i] == HLBM_GROUP_PRIMAL_WINDOW) L->nsamp += n;
      L->adj_ready = 0;
    }
  }
  g->steps_since_set += n;
  return HLBM_OK;
}

extern "C" hlbm_status hlbm_group_synchronize(hlbm_group g) {
  if (!g) return fail(HLBM_E_INVALID, "null group");
  HIP_TRY(hipStreamSynchronize(g->stream));
  return HLBM_OK;
}
