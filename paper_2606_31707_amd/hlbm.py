"""ctypes binding of libhlbm.so (the gfx950 HLBM mean-flow adjoint library).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Arrays may be numpy arrays (host memory) or torch tensors on the
GPU (device memory, passed by data_ptr()); all exchanged values are float64.
If the library is missing this module raises at import of the library, it
never falls back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhlbm.so")
# the same sources built with 64 x 4 tiles and no XCD tile remapping (tests)
CANARY_PATH = os.path.join(HERE, "libhlbm_canary.so")

D2Q9, D3Q19 = 0, 1
FP64, FP32, FP16S = 0, 1, 2
BC_PERIODIC, BC_WALLS, BC_INLET_OUTLET = 0, 1, 2
INLET_UNIFORM, INLET_PARABOLIC = 1, 2
OBJ_FFA, OBJ_DISS, OBJ_MOMENTUM, OBJ_MEA = 0, 1, 2, 3
TURB_FROZEN, TURB_DIFFERENTIATED = 0, 1
SOURCE_STEADY, SOURCE_MEAN = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
NOISE_NONE, NOISE_RIM, NOISE_BOX = 0, 1, 2
COLL_BGK, COLL_HRR = 0, 1
FIELD_RHO, FIELD_U, FIELD_MEAN_RHO, FIELD_MEAN_U, FIELD_POROSITY, FIELD_MEAN_TAU = range(6)

OK, W_NOT_CONVERGED = 0, 1
E_INVALID, E_OOM, E_STATE, E_DIVERGED, E_DEVICE = -1, -2, -3, -4, -5

EXPORTS = [
    "hlbm_create", "hlbm_destroy", "hlbm_footprint_bytes", "hlbm_set_porosity",
    "hlbm_build_cylinder", "hlbm_init_equilibrium", "hlbm_set_populations",
    "hlbm_get_populations", "hlbm_set_objective", "hlbm_run_primal", "hlbm_window_reset",
    "hlbm_window_count", "hlbm_get_objective", "hlbm_solve_adjoint", "hlbm_get_gradient",
    "hlbm_get_adjoint", "hlbm_get_field", "hlbm_synchronize", "hlbm_profile_enable",
    "hlbm_profile_get", "hlbm_bytes_per_update", "hlbm_status_string", "hlbm_last_error",
    "hlbm_set_probe", "hlbm_get_probe", "hlbm_reconfigure", "hlbm_group_create", "hlbm_group_destroy",
    "hlbm_group_set", "hlbm_group_step", "hlbm_group_synchronize", "hlbm_run_tangent",
    "hlbm_copy_probe", "hlbm_device_bytes", "hlbm_set_porosity_noalloc",
]

GROUP_PRIMAL, GROUP_PRIMAL_WINDOW, GROUP_ADJOINT = 0, 1, 2

PROFILE_PRIMAL, PROFILE_PRIMAL_WINDOW, PROFILE_ADJOINT = 0, 1, 2

CACHE_AUTO, CACHE_PLAIN, CACHE_STREAMING = 0, 1, 2


class Desc(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("stencil", C.c_int32),
        ("precision", C.c_int32),
        ("nx", C.c_int32),
        ("ny", C.c_int32),
        ("nz", C.c_int32),
        ("tau", C.c_double),
        ("smagorinsky_cs", C.c_double),
        ("bc_x", C.c_int32),
        ("bc_y", C.c_int32),
        ("bc_z", C.c_int32),
        ("inlet_profile", C.c_int32),
        ("u_in", C.c_double),
        ("force", C.c_double * 3),
        ("track_mean_populations", C.c_int32),
        ("collision", C.c_int32),
        ("cache_policy", C.c_int32),
        ("stream", C.c_void_p),
    ]


class AdjointOpts(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("source", C.c_int32),
        ("tau_adj", C.c_double),
        ("turb", C.c_int32),
        ("max_iters", C.c_int64),
        ("tol", C.c_double),
        ("check_every", C.c_int64),
        ("restart", C.c_int32),
    ]


class AdjointReport(C.Structure):
    _fields_ = [("iters", C.c_int64), ("residual", C.c_double)]


class HlbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libhlbm.so once per process (later calls return it); raises if it
    is not built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    _lib = open_library(path)
    return _lib


def open_library(path: str):
    """Loads a build of the library at `path` with the call signatures set
    (another build, e.g. the race-canary one, beside the default)."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() or "
                          "python paper_2606_31707_amd/build.py")
    # PyTorch ships its own HIP runtime; loading it first makes libhlbm.so bind
    # to that same runtime (same soname), so device pointers and streams are
    # shared with torch instead of two runtimes competing for the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "hlbm_create": (i32, [P(Desc), P(vp)]),
        "hlbm_destroy": (None, [vp]),
        "hlbm_footprint_bytes": (i32, [P(Desc), i32, i32, i64, i32, P(C.c_uint64)]),
        "hlbm_device_bytes": (i32, [vp, P(C.c_uint64)]),
        "hlbm_set_porosity": (i32, [vp, vp, i64, i32]),
        "hlbm_set_porosity_noalloc": (i32, [vp, vp, i64]),
        "hlbm_build_cylinder": (i32, [vp, dbl, dbl, dbl, vp, i64, i32, i32, dbl, dbl]),
        "hlbm_init_equilibrium": (i32, [vp, dbl, vp, i64, i32]),
        "hlbm_set_populations": (i32, [vp, vp, i64, i32]),
        "hlbm_get_populations": (i32, [vp, vp, i64, i32]),
        "hlbm_set_objective": (i32, [vp, i32, P(i32), P(i32), dbl, dbl]),
        "hlbm_run_primal": (i32, [vp, i64, i32, dbl, i64, P(i64)]),
        "hlbm_window_reset": (i32, [vp]),
        "hlbm_window_count": (i32, [vp, P(i64)]),
        "hlbm_get_objective": (i32, [vp, i32, P(dbl)]),
        "hlbm_solve_adjoint": (i32, [vp, P(AdjointOpts), P(AdjointReport)]),
        "hlbm_get_gradient": (i32, [vp, vp, i64, i32]),
        "hlbm_get_adjoint": (i32, [vp, vp, i64, i32]),
        "hlbm_get_field": (i32, [vp, i32, vp, i64, i32]),
        "hlbm_synchronize": (i32, [vp]),
        "hlbm_profile_enable": (i32, [vp, i32]),
        "hlbm_profile_get": (i32, [vp, i32, P(dbl), P(i64)]),
        "hlbm_set_probe": (i32, [vp, i32, i32, i32, i64]),
        "hlbm_reconfigure": (i32, [vp, dbl, dbl, dbl]),
        "hlbm_group_create": (i32, [vp, P(vp)]),
        "hlbm_group_destroy": (None, [vp]),
        "hlbm_group_set": (i32, [vp, P(vp), P(i32), i32]),
        "hlbm_group_step": (i32, [vp, i64]),
        "hlbm_group_synchronize": (i32, [vp]),
        "hlbm_get_probe": (i32, [vp, vp, i64, P(i64)]),
        "hlbm_run_tangent": (i32, [vp, vp, i64, i32, i64, i64, vp]),
        "hlbm_bytes_per_update": (i32, [vp, P(dbl), P(dbl), P(dbl)]),
        "hlbm_copy_probe": (i32, [vp, i32, i32, i64, P(dbl)]),
        "hlbm_status_string": (C.c_char_p, [i32]),
        "hlbm_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def _check(status: int, allow=(OK,)) -> int:
    if status in allow:
        return status
    lib = load_library()
    raise HlbmError(status, f"{lib.hlbm_status_string(status).decode()}: {lib.hlbm_last_error().decode()}")


def _arr_in(a, n):
    """(pointer, count, mem, keepalive) for an input array."""
    if a is None:
        return None, 0, MEM_HOST, None
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):  # torch tensor
        import torch
        t = a.detach()
        if t.dtype != torch.float64:
            t = t.to(torch.float64)
        t = t.contiguous()
        if t.is_cuda:
            return C.c_void_p(t.data_ptr()), t.numel(), MEM_DEVICE, t
        a = t.numpy()
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
    return arr.ctypes.data_as(C.c_void_p), arr.size, MEM_HOST, arr


def _out(out, n):
    """(pointer, mem, array) for an output buffer (numpy allocated if None)."""
    if out is None:
        arr = np.empty(n, dtype=np.float64)
        return arr.ctypes.data_as(C.c_void_p), MEM_HOST, arr
    if hasattr(out, "data_ptr") and getattr(out, "is_cuda", False):
        import torch
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == n
        return C.c_void_p(out.data_ptr()), MEM_DEVICE, out
    assert isinstance(out, np.ndarray) and out.dtype == np.float64 and out.flags.c_contiguous and out.size == n
    return out.ctypes.data_as(C.c_void_p), MEM_HOST, out


def make_desc(stencil=D2Q9, precision=FP64, nx=32, ny=16, nz=1, tau=0.8, cs=0.0,
              bc_x=BC_INLET_OUTLET, bc_y=BC_WALLS, bc_z=BC_PERIODIC,
              inlet_profile=INLET_PARABOLIC, u_in=0.03, force=(0.0, 0.0, 0.0),
              track_mean_populations=False, collision=0, cache_policy=0, stream=None) -> Desc:
    d = Desc()
    d.struct_size = C.sizeof(Desc)
    d.stencil, d.precision = stencil, precision
    d.nx, d.ny, d.nz = nx, ny, nz
    d.tau, d.smagorinsky_cs = tau, cs
    d.bc_x, d.bc_y, d.bc_z = bc_x, bc_y, bc_z
    d.inlet_profile, d.u_in = inlet_profile, u_in
    d.force = (C.c_double * 3)(*force)
    d.track_mean_populations = int(bool(track_mean_populations))
    d.collision = int(collision)
    d.cache_policy = int(cache_policy)
    d.stream = stream
    return d


def footprint_bytes(desc: Desc, with_window=True, with_adjoint=True, region_cells=0, objective=OBJ_FFA) -> int:
    """Device bytes one query on a lattice of this descriptor holds at most
    (objective region of region_cells cells of the given kind)."""
    lib = load_library()
    out = C.c_uint64()
    _check(lib.hlbm_footprint_bytes(C.byref(desc), int(with_window), int(with_adjoint), int(region_cells),
                                    int(objective), C.byref(out)))
    return int(out.value)


class Lattice:
    """One lattice on the GPU (owns an hlbm_lattice handle)."""

    def __init__(self, desc: Desc | None = None, lib=None, **kw):
        self._lib = lib if lib is not None else load_library()
        self.desc = desc if desc is not None else make_desc(**kw)
        h = C.c_void_p()
        _check(self._lib.hlbm_create(C.byref(self.desc), C.byref(h)))
        self._h = h
        self.q = 9 if self.desc.stencil == D2Q9 else 19
        self.n = self.desc.nx * self.desc.ny * self.desc.nz
        # bumped by every call that changes the porosity, the primal state,
        # the window or the objective (the adjoint of a forward pass is only
        # valid while it is unchanged)
        self.generation = 0

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.hlbm_destroy(h)
        self._h = None

    def __del__(self):
        self.close()

    # ---- geometry / state
    def set_porosity(self, d):
        self.generation += 1
        p, n, mem, _keep = _arr_in(d, self.n)
        _check(self._lib.hlbm_set_porosity(self._h, p, n, mem))

    def set_porosity_noalloc(self, d):
        """hlbm_set_porosity_noalloc: d must be a float64 CUDA tensor on the
        lattice's device (no staging, no allocation in the library)."""
        self.generation += 1
        if not (hasattr(d, "is_cuda") and d.is_cuda):
            raise ValueError("set_porosity_noalloc takes a CUDA tensor")
        import torch
        if d.dtype != torch.float64 or not d.is_contiguous():
            raise ValueError("set_porosity_noalloc takes a contiguous float64 tensor")
        _check(self._lib.hlbm_set_porosity_noalloc(self._h, C.c_void_p(d.data_ptr()), d.numel()))

    def build_cylinder(self, xc, yc, D, noise=None, noise_mode=NOISE_NONE, box_half=0.0, d_solid=0.0):
        self.generation += 1
        p, n, mem, _keep = _arr_in(noise, self.n)
        _check(self._lib.hlbm_build_cylinder(self._h, xc, yc, D, p, n if noise is not None else 0,
                                             mem, noise_mode, box_half, d_solid))

    def init_equilibrium(self, rho0=1.0, u=None):
        self.generation += 1
        p, n, mem, _keep = _arr_in(u, 3 * self.n)
        _check(self._lib.hlbm_init_equilibrium(self._h, rho0, p, n, mem))

    def set_populations(self, f):
        self.generation += 1
        p, n, mem, _keep = _arr_in(f, self.q * self.n)
        _check(self._lib.hlbm_set_populations(self._h, p, n, mem))

    def populations(self, out=None):
        p, mem, arr = _out(out, self.q * self.n)
        _check(self._lib.hlbm_get_populations(self._h, p, self.q * self.n, mem))
        return arr.reshape(self.q, self.n) if isinstance(arr, np.ndarray) else arr

    def porosity(self):
        return self.field(FIELD_POROSITY)

    def field(self, which, out=None):
        n = 3 * self.n if which in (FIELD_U, FIELD_MEAN_U) else self.n
        p, mem, arr = _out(out, n)
        _check(self._lib.hlbm_get_field(self._h, which, p, n, mem))
        if isinstance(arr, np.ndarray) and n == 3 * self.n:
            return arr.reshape(3, self.n)
        return arr

    def moments(self):
        return self.field(FIELD_RHO), self.field(FIELD_U)

    # ---- objective / primal / window
    def set_objective(self, kind, lo, hi, u0=0.0, p0=1.0 / 3.0):
        self.generation += 1
        lo3 = (C.c_int32 * 3)(*(list(lo) + [0] * (3 - len(lo))))
        hi3 = (C.c_int32 * 3)(*(list(hi) + [0] * (3 - len(hi))))
        _check(self._lib.hlbm_set_objective(self._h, kind, lo3, hi3, u0, p0))

    def run_primal(self, n_steps, accumulate=False, steady_tol=0.0, check_every=100):
        self.generation += 1
        done = C.c_int64()
        st = self._lib.hlbm_run_primal(self._h, int(n_steps), int(bool(accumulate)), steady_tol,
                                       int(check_every), C.byref(done))
        _check(st, allow=(OK, W_NOT_CONVERGED))
        return int(done.value)

    def step(self, n=1, accumulate=False):
        return self.run_primal(n, accumulate)

    def run_tangent(self, v, n_steps, record_every=1):
        """Forward tangent along v from the current state: returns an array
        [records, 2] of (J(t), dJ(t)/dd . v)."""
        self.generation += 1
        p, n, mem, _keep = _arr_in(v, self.n)
        nrec = int(n_steps) // int(record_every)
        out = np.zeros(2 * max(nrec, 1))
        _check(self._lib.hlbm_run_tangent(self._h, p, n, mem, int(n_steps), int(record_every),
                                          out.ctypes.data_as(C.c_void_p)))
        return out[: 2 * nrec].reshape(nrec, 2)

    def window_reset(self):
        self.generation += 1
        _check(self._lib.hlbm_window_reset(self._h))

    def window_count(self) -> int:
        c = C.c_int64()
        _check(self._lib.hlbm_window_count(self._h, C.byref(c)))
        return int(c.value)

    def objective(self, which=0) -> float:
        J = C.c_double()
        _check(self._lib.hlbm_get_objective(self._h, which, C.byref(J)))
        return J.value

    def window_objective(self) -> float:
        return self.objective(1)

    # ---- adjoint / gradient
    def solve_adjoint(self, source=SOURCE_STEADY, tau_adj=0.0, turb=TURB_DIFFERENTIATED,
                      max_iters=1000, tol=0.0, check_every=100, restart=True):
        o = AdjointOpts()
        o.struct_size = C.sizeof(AdjointOpts)
        o.source, o.tau_adj, o.turb = source, tau_adj, turb
        o.max_iters, o.tol, o.check_every, o.restart = int(max_iters), tol, int(check_every), int(bool(restart))
        rep = AdjointReport()
        st = self._lib.hlbm_solve_adjoint(self._h, C.byref(o), C.byref(rep))
        _check(st, allow=(OK, W_NOT_CONVERGED))
        return int(rep.iters), float(rep.residual), st

    def gradient(self, out=None):
        p, mem, arr = _out(out, self.n)
        _check(self._lib.hlbm_get_gradient(self._h, p, self.n, mem))
        return arr

    def adjoint(self, out=None):
        p, mem, arr = _out(out, self.q * self.n)
        _check(self._lib.hlbm_get_adjoint(self._h, p, self.q * self.n, mem))
        return arr.reshape(self.q, self.n) if isinstance(arr, np.ndarray) else arr

    # ---- timing
    def synchronize(self):
        _check(self._lib.hlbm_synchronize(self._h))

    def profile_enable(self, every=1):
        """Times the sweeps of each kind in blocks of up to `every` back-to-back launches with
        HIP events recorded on the stream (0: off); see profile()."""
        _check(self._lib.hlbm_profile_enable(self._h, int(every)))

    def profile(self):
        out = {}
        for kind, name in ((PROFILE_PRIMAL, "primal"), (PROFILE_PRIMAL_WINDOW, "primal_window"),
                           (PROFILE_ADJOINT, "adjoint")):
            us, n = C.c_double(), C.c_int64()
            _check(self._lib.hlbm_profile_get(self._h, kind, C.byref(us), C.byref(n)))
            out[name] = {"mean_us": us.value, "sampled": n.value}
        return out

    def set_probe(self, x, y, z=0, capacity=1 << 18):
        _check(self._lib.hlbm_set_probe(self._h, int(x), int(y), int(z), int(capacity)))
        self._probe_cap = int(capacity)

    def probe(self) -> np.ndarray:
        cap = getattr(self, "_probe_cap", 0)
        out = np.empty(max(cap, 1), dtype=np.float64)
        cnt = C.c_int64()
        _check(self._lib.hlbm_get_probe(self._h, out.ctypes.data_as(C.c_void_p), cap, C.byref(cnt)))
        return out[: cnt.value].copy()

    def reconfigure(self, tau, cs, u_in):
        self.generation += 1
        _check(self._lib.hlbm_reconfigure(self._h, tau, cs, u_in))
        self.desc.tau, self.desc.smagorinsky_cs, self.desc.u_in = tau, cs, u_in

    def device_bytes(self) -> int:
        """Device bytes this lattice holds now."""
        out = C.c_uint64()
        _check(self._lib.hlbm_device_bytes(self._h, C.byref(out)))
        return int(out.value)

    def copy_probe(self, pattern=0, streaming=False, n_launches=20) -> float:
        """Mean microseconds per launch of the bandwidth probe (a plain sweep's
        bytes without arithmetic; pattern 0 own slots, 1 odd-step neighbours,
        2 the two-array pull pattern)."""
        us = C.c_double()
        _check(self._lib.hlbm_copy_probe(self._h, int(pattern), int(bool(streaming)), int(n_launches),
                                         C.byref(us)))
        return us.value

    def bytes_per_update(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(self._lib.hlbm_bytes_per_update(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return {"primal": a.value, "primal_window": b.value, "adjoint": c.value}


class Group:
    """Packed launches over several lattices of one stencil and precision."""

    def __init__(self, stream=None):
        self._lib = load_library()
        h = C.c_void_p()
        _check(self._lib.hlbm_group_create(stream, C.byref(h)))
        self._h = h
        self.members = []

    def set(self, lattices, modes):
        n = len(lattices)
        arr = (C.c_void_p * max(n, 1))(*[L._h.value for L in lattices])
        md = (C.c_int32 * max(n, 1))(*modes)
        _check(self._lib.hlbm_group_set(self._h, arr, md, n))
        self.members = list(lattices)

    def step(self, n):
        _check(self._lib.hlbm_group_step(self._h, int(n)))

    def synchronize(self):
        _check(self._lib.hlbm_group_synchronize(self._h))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.hlbm_group_destroy(h)
        self._h = None

    def __del__(self):
        self.close()
