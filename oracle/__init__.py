"""Plain FP64 CPU oracle of the HLBM mean-flow adjoint path (ctypes binding).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package; the product library
never does.  The arithmetic lives in ``hlbm_oracle.c`` (plain loops, FP64,
built with ``-O2 -ffp-contract=off``); this module only marshals numpy arrays.

Array exchange layout: ``value[i, cell]`` with ``cell = x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from .build import LIB_PATH, build

D2Q9, D3Q19 = 0, 1
BC_PERIODIC, BC_WALLS, BC_INLET_OUTLET = 0, 1, 2
INLET_UNIFORM, INLET_PARABOLIC = 1, 2
OBJ_FFA, OBJ_DISS, OBJ_MOMENTUM, OBJ_MEA = 0, 1, 2, 3
TURB_FROZEN, TURB_DIFFERENTIATED = 0, 1
NOISE_NONE, NOISE_RIM, NOISE_BOX = 0, 1, 2
COLL_BGK, COLL_HRR = 0, 1


class _Params(C.Structure):
    _fields_ = [
        ("stencil", C.c_int),
        ("nx", C.c_int),
        ("ny", C.c_int),
        ("nz", C.c_int),
        ("tau", C.c_double),
        ("cs", C.c_double),
        ("bc_x", C.c_int),
        ("bc_y", C.c_int),
        ("bc_z", C.c_int),
        ("inlet_profile", C.c_int),
        ("u_in", C.c_double),
        ("force", C.c_double * 3),
        ("collision", C.c_int),
    ]


_lib = None
_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_IP = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # HLBM_ORACLE_LIB: another build of the same source (the sanitizer run)
    path = os.environ.get("HLBM_ORACLE_LIB") or LIB_PATH
    if not os.path.exists(path):
        build()
    lib = C.CDLL(path)
    vp = C.c_void_p
    sig = {
        "orc_create": (vp, [C.POINTER(_Params)]),
        "orc_destroy": (None, [vp]),
        "orc_q": (C.c_int, [vp]),
        "orc_n": (C.c_long, [vp]),
        "orc_set_porosity": (C.c_int, [vp, _DP]),
        "orc_get_porosity": (C.c_int, [vp, _DP]),
        "orc_build_cylinder": (C.c_int, [vp, C.c_double, C.c_double, C.c_double, vp, C.c_int, C.c_double,
                                         C.c_double]),
        "orc_init_equilibrium": (C.c_int, [vp, C.c_double, vp]),
        "orc_set_populations": (C.c_int, [vp, _DP]),
        "orc_get_populations": (C.c_int, [vp, _DP]),
        "orc_step": (C.c_int, [vp, C.c_long]),
        "orc_run_steady": (C.c_long, [vp, C.c_long, C.c_double, C.c_long]),
        "orc_moments": (C.c_int, [vp, _DP, _DP]),
        "orc_set_objective": (C.c_int, [vp, C.c_int, _IP, _IP, C.c_double, C.c_double]),
        "orc_objective": (C.c_double, [vp]),
        "orc_mea_surface": (C.c_int, [vp, vp]),
        "orc_tangent_seed": (C.c_int, [vp]),
        "orc_hrr_collide_cell": (None, [C.c_int, _DP, C.c_double, C.c_double, C.c_double, vp, _DP]),
        "orc_hrr_jacobian_cell": (None, [C.c_int, _DP, C.c_double, C.c_double, C.c_double, C.c_int, C.c_double,
                                         _DP]),
        "orc_hrr_dcdd_cell": (None, [C.c_int, _DP, C.c_double, C.c_double, C.c_double, C.c_int, C.c_double,
                                     _DP]),
        "orc_tangent_step": (C.c_int, [vp, _DP, C.c_long]),
        "orc_tangent_objective": (C.c_double, [vp, _DP]),
        "orc_get_tangent": (C.c_int, [vp, _DP]),
        "orc_mea_source": (C.c_int, [vp, _DP]),
        "orc_window_reset": (None, [vp]),
        "orc_window_sample": (None, [vp]),
        "orc_window_count": (C.c_long, [vp]),
        "orc_window_objective": (C.c_double, [vp]),
        "orc_window_mean_populations": (C.c_int, [vp, _DP]),
        "orc_adjoint_prepare": (C.c_int, [vp, C.c_int, C.c_double, C.c_int]),
        "orc_adjoint_reset": (None, [vp]),
        "orc_adjoint_iterate": (C.c_int, [vp, C.c_long]),
        "orc_adjoint_solve": (C.c_long, [vp, C.c_long, C.c_double, C.c_long, C.POINTER(C.c_double)]),
        "orc_get_adjoint": (C.c_int, [vp, _DP]),
        "orc_gradient": (C.c_int, [vp, _DP]),
        "orc_stencil": (None, [C.c_int, C.POINTER(C.c_int), _IP, _DP, _IP]),
        "orc_equilibrium": (None, [C.c_int, C.c_double, _DP, _DP]),
        "orc_tau_eff": (C.c_double, [C.c_int, _DP, C.c_double, C.c_double]),
        "orc_collide_cell": (None, [C.c_int, _DP, C.c_double, C.c_double, C.c_double, vp, _DP]),
        "orc_jacobian_cell": (None, [C.c_int, _DP, C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, _DP]),
        "orc_dcdd_cell": (None, [C.c_int, _DP, C.c_double, C.c_double, _DP]),
        "orc_objective_cell": (C.c_double, [C.c_int, C.c_int, _DP, C.c_double, C.c_double, C.c_double, C.c_double]),
        "orc_dJdf_cell": (None, [C.c_int, C.c_int, _DP, C.c_double, C.c_double, C.c_double, C.c_double, _DP]),
        "orc_dJdd_cell": (C.c_double, [C.c_int, C.c_int, _DP, C.c_double, C.c_double]),
        "orc_apply_stream": (C.c_int, [vp, _DP, _DP, _DP]),
        "orc_apply_stream_transpose": (C.c_int, [vp, _DP, _DP, _DP]),
        "orc_outlet_values_cell": (None, [C.c_int, _DP, _DP]),
        "orc_outlet_jacobian_cell": (None, [C.c_int, _DP, _DP]),
        "orc_get_adjoint_virtual": (C.c_int, [vp, _DP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# per-cell building blocks
# --------------------------------------------------------------------------

def stencil(kind: int):
    lib = _load()
    q = C.c_int()
    c = np.zeros(3 * 19, np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    lib.orc_stencil(kind, C.byref(q), c, w, opp)
    qq = q.value
    return c[: 3 * qq].reshape(qq, 3).copy(), w[:qq].copy(), opp[:qq].copy()


def equilibrium(kind: int, rho: float, v) -> np.ndarray:
    lib = _load()
    q = 9 if kind == D2Q9 else 19
    out = np.zeros(q)
    vv = np.zeros(3)
    vv[: len(v)] = v
    lib.orc_equilibrium(kind, rho, vv, out)
    return out


def tau_eff(kind, f, tau0, cs) -> float:
    return _load().orc_tau_eff(kind, _f64(f), tau0, cs)


def hrr_collide_cell(kind, f, d, tau0, cs=0.0, force=None) -> np.ndarray:
    f = _f64(f)
    out = np.zeros_like(f)
    fo = None if force is None else _f64(np.resize(np.asarray(force, float), 3))
    _load().orc_hrr_collide_cell(kind, f, d, tau0, cs, _ptr(fo), out)
    return out


def hrr_jacobian_cell(kind, f, d, tau_a, cs=0.0, turb=TURB_DIFFERENTIATED, tau_frozen=0.0) -> np.ndarray:
    f = _f64(f)
    q = len(f)
    A = np.zeros(q * q)
    _load().orc_hrr_jacobian_cell(kind, f, d, tau_a, cs, turb, tau_frozen, A)
    return A.reshape(q, q)


def hrr_dcdd_cell(kind, f, d, tau_a, cs=0.0, turb=TURB_DIFFERENTIATED, tau_frozen=0.0) -> np.ndarray:
    f = _f64(f)
    out = np.zeros(len(f))
    _load().orc_hrr_dcdd_cell(kind, f, d, tau_a, cs, turb, tau_frozen, out)
    return out


def collide_cell(kind, f, d, tau0, cs=0.0, force=None) -> np.ndarray:
    f = _f64(f)
    out = np.zeros_like(f)
    fo = None if force is None else _f64(np.resize(np.asarray(force, float), 3))
    _load().orc_collide_cell(kind, f, d, tau0, cs, _ptr(fo), out)
    return out


def jacobian_cell(kind, f, d, tau_a, cs=0.0, turb=TURB_DIFFERENTIATED, tau_frozen=0.0) -> np.ndarray:
    """A[j, i] = dC_j/df_i."""
    f = _f64(f)
    q = f.size
    A = np.zeros(q * q)
    _load().orc_jacobian_cell(kind, f, d, tau_a, cs, turb, tau_frozen, A)
    return A.reshape(q, q)


def dcdd_cell(kind, f, d, tau_used) -> np.ndarray:
    f = _f64(f)
    out = np.zeros_like(f)
    _load().orc_dcdd_cell(kind, f, d, tau_used, out)
    return out


def objective_cell(kind, obj, f, d, tau0, u0=0.0, p0=1.0 / 3.0) -> float:
    return _load().orc_objective_cell(kind, obj, _f64(f), d, tau0, u0, p0)


def dJdf_cell(kind, obj, f, d, tau0, u0=0.0, p0=1.0 / 3.0) -> np.ndarray:
    f = _f64(f)
    out = np.zeros_like(f)
    _load().orc_dJdf_cell(kind, obj, f, d, tau0, u0, p0, out)
    return out


def dJdd_cell(kind, obj, f, d, tau0) -> float:
    return _load().orc_dJdd_cell(kind, obj, _f64(f), d, tau0)


def outlet_values_cell(kind, f) -> np.ndarray:
    f = _f64(f)
    out = np.zeros_like(f)
    _load().orc_outlet_values_cell(kind, f, out)
    return out


def outlet_jacobian_cell(kind, f) -> np.ndarray:
    """B[j, i] = dV_j/df_i."""
    f = _f64(f)
    q = f.size
    B = np.zeros(q * q)
    _load().orc_outlet_jacobian_cell(kind, f, B)
    return B.reshape(q, q)


# --------------------------------------------------------------------------
# lattice
# --------------------------------------------------------------------------

@dataclass
class Params:
    stencil: int = D2Q9
    nx: int = 32
    ny: int = 16
    nz: int = 1
    tau: float = 0.8
    cs: float = 0.0
    bc_x: int = BC_INLET_OUTLET
    bc_y: int = BC_WALLS
    bc_z: int = BC_PERIODIC
    inlet_profile: int = INLET_PARABOLIC
    u_in: float = 0.03
    force: tuple = field(default_factory=lambda: (0.0, 0.0, 0.0))
    collision: int = 0   # COLL_BGK or COLL_HRR


class Lattice:
    """One oracle lattice (owns its C handle)."""

    def __init__(self, p: Params):
        lib = _load()
        cp = _Params(p.stencil, p.nx, p.ny, p.nz, p.tau, p.cs, p.bc_x, p.bc_y, p.bc_z,
                     p.inlet_profile, p.u_in, (C.c_double * 3)(*p.force), p.collision)
        h = lib.orc_create(C.byref(cp))
        if not h:
            raise ValueError(f"oracle rejected parameters {p}")
        self._h = h
        self._lib = lib
        self.p = p
        self.q = lib.orc_q(h)
        self.n = lib.orc_n(h)
        self.shape = (p.nz, p.ny, p.nx)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    # --- geometry / state
    def set_porosity(self, d):
        d = _f64(np.ravel(d))
        assert d.size == self.n
        if self._lib.orc_set_porosity(self._h, d) != 0:
            raise ValueError("porosity must lie in [0, 1]")

    def porosity(self) -> np.ndarray:
        d = np.zeros(self.n)
        self._lib.orc_get_porosity(self._h, d)
        return d

    def build_cylinder(self, xc, yc, D, noise=None, noise_mode=NOISE_NONE, box_half=0.0, d_solid=0.0):
        nz = None if noise is None else _f64(np.ravel(noise))
        self._lib.orc_build_cylinder(self._h, xc, yc, D, _ptr(nz), noise_mode, box_half, d_solid)

    def init_equilibrium(self, rho0=1.0, u=None):
        ua = None if u is None else _f64(np.reshape(u, (3, self.n)))
        self._lib.orc_init_equilibrium(self._h, rho0, _ptr(ua))

    def set_populations(self, f):
        f = _f64(np.reshape(f, (self.q, self.n)))
        self._lib.orc_set_populations(self._h, f)

    def populations(self) -> np.ndarray:
        f = np.zeros((self.q, self.n))
        self._lib.orc_get_populations(self._h, f)
        return f

    def step(self, n=1):
        self._lib.orc_step(self._h, int(n))

    def run_steady(self, max_steps, tol, check_every=100) -> int:
        return int(self._lib.orc_run_steady(self._h, int(max_steps), tol, int(check_every)))

    def moments(self):
        rho = np.zeros(self.n)
        u = np.zeros((3, self.n))
        self._lib.orc_moments(self._h, rho, u)
        return rho, u

    # --- objective / window
    def set_objective(self, kind, lo, hi, u0=0.0, p0=1.0 / 3.0):
        lo3 = np.zeros(3, np.int32)
        hi3 = np.zeros(3, np.int32)
        lo3[: len(lo)] = lo
        hi3[: len(hi)] = hi
        if self._lib.orc_set_objective(self._h, kind, lo3, hi3, u0, p0) != 0:
            raise ValueError("bad objective region")

    def objective(self) -> float:
        return self._lib.orc_objective(self._h)

    # --- forward tangent (App. C)
    def tangent_seed(self):
        self._lib.orc_tangent_seed(self._h)

    def tangent_step(self, v, n=1):
        self._v = _f64(np.ravel(v))
        if self._lib.orc_tangent_step(self._h, self._v, n) != 0:
            raise ValueError("tangent not seeded")

    def tangent_objective(self, v) -> float:
        return self._lib.orc_tangent_objective(self._h, _f64(np.ravel(v)))

    def tangent(self) -> np.ndarray:
        out = np.zeros(self.q * self.n)
        if self._lib.orc_get_tangent(self._h, out) != 0:
            raise ValueError("tangent not seeded")
        return out.reshape(self.q, self.n)

    def mea_surface(self) -> np.ndarray:
        """Surface flags of J_MEA (set_objective(OBJ_MEA, ...) first)."""
        out = np.zeros(self.n, np.uint8)
        if self._lib.orc_mea_surface(self._h, out.ctypes.data_as(C.c_void_p)) != 0:
            raise ValueError("no objective set")
        return out

    def mea_source(self) -> np.ndarray:
        """dJ_MEA/df as [q, n]."""
        out = np.zeros(self.q * self.n)
        if self._lib.orc_mea_source(self._h, out) != 0:
            raise ValueError("objective is not MEA")
        return out.reshape(self.q, self.n)

    def window_reset(self):
        self._lib.orc_window_reset(self._h)

    def window_sample(self):
        self._lib.orc_window_sample(self._h)

    def window_count(self) -> int:
        return int(self._lib.orc_window_count(self._h))

    def window_objective(self) -> float:
        return self._lib.orc_window_objective(self._h)

    def window_mean_populations(self) -> np.ndarray:
        f = np.zeros((self.q, self.n))
        if self._lib.orc_window_mean_populations(self._h, f) != 0:
            raise RuntimeError("empty window")
        return f

    # --- adjoint
    def adjoint_prepare(self, source=0, tau_adj=0.0, turb=TURB_DIFFERENTIATED):
        if self._lib.orc_adjoint_prepare(self._h, source, tau_adj, turb) != 0:
            raise RuntimeError("adjoint_prepare: objective or window missing")

    def adjoint_reset(self):
        self._lib.orc_adjoint_reset(self._h)

    def adjoint_iterate(self, iters):
        if self._lib.orc_adjoint_iterate(self._h, int(iters)) != 0:
            raise RuntimeError("adjoint not prepared")

    def adjoint_solve(self, max_iters, tol, check_every=100):
        r = C.c_double()
        k = self._lib.orc_adjoint_solve(self._h, int(max_iters), tol, int(check_every), C.byref(r))
        return int(k), r.value

    def adjoint(self) -> np.ndarray:
        phi = np.zeros((self.q, self.n))
        self._lib.orc_get_adjoint(self._h, phi)
        return phi

    def gradient(self) -> np.ndarray:
        g = np.zeros(self.n)
        if self._lib.orc_gradient(self._h, g) != 0:
            raise RuntimeError("adjoint not prepared")
        return g

    def adjoint_virtual(self) -> np.ndarray:
        phiv = np.zeros((self.q, self.n))
        self._lib.orc_get_adjoint_virtual(self._h, phiv)
        return phiv

    def apply_stream(self, x, xv) -> np.ndarray:
        """S: (post-collision values, outlet virtual values) -> state values."""
        x = _f64(np.reshape(x, (self.q, self.n)))
        xv = _f64(np.reshape(xv, (self.q, self.n)))
        out = np.zeros_like(x)
        self._lib.orc_apply_stream(self._h, x, xv, out)
        return out

    def apply_stream_transpose(self, y):
        """S^T: state values -> (post-collision values, outlet virtual values)."""
        y = _f64(np.reshape(y, (self.q, self.n)))
        out = np.zeros_like(y)
        vout = np.zeros_like(y)
        self._lib.orc_apply_stream_transpose(self._h, y, out, vout)
        return out, vout
