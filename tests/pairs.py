"""Builds matching oracle (CPU, FP64) and GPU (libhlbm.so) lattices from one
spec, for the parity tests.  The two share only the seeded inputs."""
from __future__ import annotations

import sys
from dataclasses import dataclass, field

import numpy as np

import oracle as O


@dataclass
class Spec:
    stencil: int = 0
    nx: int = 220
    ny: int = 41
    nz: int = 1
    tau: float = 0.53
    cs: float = 0.0
    bc_x: int = 2
    bc_y: int = 1
    bc_z: int = 0
    inlet_profile: int = 2
    u_in: float = 0.03
    force: tuple = (0.0, 0.0, 0.0)
    cyl: tuple | None = (40.0, 20.0, 10.0)   # xc, yc, D
    noise_mode: int = 0
    noise: np.ndarray | None = None
    box_half: float = 0.0
    porosity: np.ndarray | None = None        # overrides the cylinder
    init_u: np.ndarray | None = None
    init_f: np.ndarray | None = None
    obj: tuple | None = None                  # (kind, lo, hi, u0)
    track_mean: bool = False
    collision: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.nx * self.ny * self.nz


def make_oracle(s: Spec) -> O.Lattice:
    p = O.Params(stencil=s.stencil, nx=s.nx, ny=s.ny, nz=s.nz, tau=s.tau, cs=s.cs, bc_x=s.bc_x,
                 bc_y=s.bc_y, bc_z=s.bc_z, inlet_profile=s.inlet_profile, u_in=s.u_in,
                 force=tuple(s.force), collision=s.collision)
    L = O.Lattice(p)
    if s.porosity is not None:
        L.set_porosity(s.porosity)
    elif s.cyl is not None:
        L.build_cylinder(*s.cyl, noise=s.noise, noise_mode=s.noise_mode, box_half=s.box_half)
    if s.init_f is not None:
        L.set_populations(s.init_f)
    else:
        L.init_equilibrium(1.0, s.init_u)
    if s.obj is not None:
        kind, lo, hi, u0 = s.obj
        L.set_objective(kind, lo, hi, u0=u0)
    return L


def make_gpu(s: Spec, precision: int = 0):
    from paper_2606_31707_amd import hlbm as H
    G = H.Lattice(stencil=s.stencil, precision=precision, nx=s.nx, ny=s.ny, nz=s.nz, tau=s.tau, cs=s.cs,
                  bc_x=s.bc_x, bc_y=s.bc_y, bc_z=s.bc_z, inlet_profile=s.inlet_profile, u_in=s.u_in,
                  force=tuple(s.force), track_mean_populations=s.track_mean, collision=s.collision,
                  cache_policy=s.extra.get("cache_policy", 0))
    if s.porosity is not None:
        G.set_porosity(s.porosity)
    elif s.cyl is not None:
        G.build_cylinder(*s.cyl, noise=s.noise, noise_mode=s.noise_mode, box_half=s.box_half)
    if s.init_f is not None:
        G.set_populations(s.init_f)
    else:
        G.init_equilibrium(1.0, s.init_u)
    if s.obj is not None:
        kind, lo, hi, u0 = s.obj
        G.set_objective(kind, lo, hi, u0=u0)
    return G


def state_mask(s: Spec) -> np.ndarray:
    """Cells whose populations are state variables (all but the inlet column)."""
    col = np.arange(s.n) % s.nx
    return col > 0 if s.bc_x == 2 else np.ones(s.n, bool)


def rel_err(a, b, mask=None) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a = a[..., mask]
        b = b[..., mask]
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def objective_tol(L: O.Lattice, s: Spec, kind, lo, hi, u0, rel=1e-12) -> float:
    """Absolute tolerance for J: the first-order effect of population errors
    of rel * max|f| on J, i.e. rel * max|f| * sum over the region of
    sum_i |dJ_x/df_i| (J is often a small difference of O(u^2) terms)."""
    f = L.populations()
    d = L.porosity()
    fmax = np.abs(f).max()
    acc = 0.0
    for z in range(lo[2], hi[2] + 1):
        for y in range(lo[1], hi[1] + 1):
            for x in range(lo[0], hi[0] + 1):
                c = x + s.nx * (y + s.ny * z)
                acc += np.abs(O.dJdf_cell(s.stencil, kind, f[:, c], d[c], s.tau, u0)).sum()
    return rel * fmax * max(acc, 1e-300) + 1e-18


def say(*a):
    """Names the case on stdout before a GPU step (survives a crash)."""
    print(*a, flush=True)
    sys.stdout.flush()
