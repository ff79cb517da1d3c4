"""Seeded synthetic workloads (lattice units).  Holds no arithmetic of the
method: only sizes, parameters and the random numbers both the GPU path and
the test oracle take as inputs.

Workload recipes (stand-ins for the paper's cylinder cases, Sec. 5):
  channel_re20   2D channel 220 x 41, porous cylinder D = 10 at (40, 20),
                 parabolic inlet u_max = 0.03, Re = 20 on the mean inflow
                 (nu = u_mean D / Re), drag (FFA) plane at x_c + 5 D.
  vortex_re100   2D channel 1100 x 410, D = 40 at (160, 204.5), u_max = 0.04,
                 Re = 100, uniform +-0.02 porosity noise on the cylinder rim
                 (seed 2), dissipation box x in [1, 600], full height.
  les_re3900     3D 768 x 384 x 128 (D3Q19), D = 48 at (192, 191.5), uniform
                 inflow 0.04, Re = 3900, Smagorinsky Cs = 0.1, y/z periodic,
                 1% velocity noise (seed 3), drag plane x = 432, y in [48, 335].
  autograd_re40  2D 400 x 160, D = 40 at (160, 79.5), u_max = 0.03, Re = 40,
                 solid-fraction noise U[0, 0.05] in |x-x_c|, |y-y_c| <= 2D
                 (seeds 400..431), drag plane x = 360.
  porous3d_re40  the steady 3D validation case of Sec. 5.2 in lattice units:
                 3.6 x 0.8 x 0.4 m at N = 21 cells per diameter (dx = 0.1/21 m)
                 -> 756 x 168 x 84 D3Q19, D = 21 at (251.5, 83.5), tau = 0.55,
                 uniform inflow at Re = 40, y and z periodic, permeable
                 cylinder K = 1e-6 m^2 (core porosity 1 - tau nu / K in
                 lattice units = 0.792), drag plane x = 357 (1.7 m),
                 dissipation box x in [21, 482] (1.2 +- 1.1 m); T = 32 s =
                 42 336 steps.
  grid2d_8192x4096  the vortex-street geometry on a grid whose populations
                 exceed every cache (33.5 M cells, 2.4 GB FP64): D = 256 at
                 (1024, 2047.5), u_max = 0.04, Re = 100, drag plane x_c + 5 D;
                 the 2D roofline lattice of the sweep measurements.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

D2Q9, D3Q19 = 0, 1
BC_PERIODIC, BC_WALLS, BC_INLET_OUTLET = 0, 1, 2
INLET_UNIFORM, INLET_PARABOLIC = 1, 2
OBJ_FFA, OBJ_DISS = 0, 1
NOISE_NONE, NOISE_RIM, NOISE_BOX = 0, 1, 2


@dataclass
class Workload:
    name: str
    stencil: int
    nx: int
    ny: int
    nz: int
    u_max: float            # parabola maximum or uniform inflow speed
    inlet_profile: int
    Re: float
    D: float
    xc: float
    yc: float
    bc_y: int = BC_WALLS
    bc_z: int = BC_PERIODIC
    cs: float = 0.0
    objective: int = OBJ_FFA
    lo: tuple = (0, 0, 0)
    hi: tuple = (0, 0, 0)
    noise_mode: int = NOISE_NONE
    noise_amp: float = 0.0
    noise_seed: int = 0
    box_half: float = 0.0
    velocity_noise: float = 0.0   # amplitude of the initial velocity noise
    primal_steps: int = 4000
    d_solid: float = 0.0          # porosity inside a permeable cylinder
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def u_mean(self) -> float:
        return 2.0 / 3.0 * self.u_max if self.inlet_profile == INLET_PARABOLIC else self.u_max

    @property
    def nu(self) -> float:
        return self.u_mean * self.D / self.Re

    @property
    def tau(self) -> float:
        return 3.0 * self.nu + 0.5

    @property
    def u0(self) -> float:
        """FFA reference velocity: the inflow maximum."""
        return self.u_max


def channel_re20() -> Workload:
    D, xc = 10.0, 40.0
    x = int(xc + 5 * D)
    return Workload("channel_re20_220x41", D2Q9, 220, 41, 1, 0.03, INLET_PARABOLIC, 20.0, D, xc, 20.0,
                    objective=OBJ_FFA, lo=(x, 0, 0), hi=(x, 40, 0), primal_steps=4000)


def vortex_re100() -> Workload:
    return Workload("vortex_re100_1100x410", D2Q9, 1100, 410, 1, 0.04, INLET_PARABOLIC, 100.0, 40.0,
                    160.0, 204.5, objective=OBJ_DISS, lo=(1, 0, 0), hi=(600, 409, 0),
                    noise_mode=NOISE_RIM, noise_amp=0.02, noise_seed=2, primal_steps=200000,
                    extra={"window_periods": 10, "probe": (240, 204)})


def les_re3900() -> Workload:
    return Workload("les_re3900_768x384x128", D3Q19, 768, 384, 128, 0.04, INLET_UNIFORM, 3900.0, 48.0,
                    192.0, 191.5, bc_y=BC_PERIODIC, bc_z=BC_PERIODIC, cs=0.1, objective=OBJ_FFA,
                    lo=(432, 48, 0), hi=(432, 335, 127), velocity_noise=0.04 * 0.01, noise_seed=3,
                    primal_steps=100000)


def autograd_re40(seed: int = 400) -> Workload:
    return Workload(f"autograd_re40_400x160_s{seed}", D2Q9, 400, 160, 1, 0.03, INLET_PARABOLIC, 40.0,
                    40.0, 160.0, 79.5, objective=OBJ_FFA, lo=(360, 0, 0), hi=(360, 159, 0),
                    noise_mode=NOISE_BOX, noise_amp=0.05, noise_seed=seed, box_half=80.0)


def porous3d_re40() -> Workload:
    dx = 0.1 / 21.0                       # m per cell (N = 21 over D = 0.1 m)
    tau = 0.55
    nu_l = (tau - 0.5) / 3.0
    k_l = 1e-6 / (dx * dx)                # permeability in lattice units
    u = 40.0 * nu_l / 21.0                # Re = u D / nu
    return Workload("porous3d_re40_756x168x84", D3Q19, 756, 168, 84, u, INLET_UNIFORM, 40.0, 21.0, 251.5,
                    83.5, bc_y=BC_PERIODIC, bc_z=BC_PERIODIC, objective=OBJ_FFA, lo=(357, 0, 0),
                    hi=(357, 167, 83), primal_steps=42336, d_solid=1.0 - tau * nu_l / k_l,
                    extra={"dissipation_box": ((21, 0, 0), (482, 167, 83))})


def grid2d_8192x4096() -> Workload:
    D, xc = 256.0, 1024.0
    x = int(xc + 5 * D)
    return Workload("grid2d_8192x4096", D2Q9, 8192, 4096, 1, 0.04, INLET_PARABOLIC, 100.0, D, xc, 2047.5,
                    objective=OBJ_FFA, lo=(x, 0, 0), hi=(x, 4095, 0))


def scaled(w: Workload, factor: float, name: str | None = None) -> Workload:
    """Same geometry ratios on a grid scaled by `factor` (parity-test sizes)."""
    s = factor
    return replace(w, name=name or f"{w.name}_x{factor:g}", nx=max(3, int(round(w.nx * s))),
                   ny=max(1, int(round(w.ny * s))), nz=w.nz if w.stencil == D2Q9 else max(1, int(round(w.nz * s))),
                   D=w.D * s, xc=w.xc * s, yc=(max(1, int(round(w.ny * s))) - 1) / 2.0,
                   lo=tuple(int(v * s) for v in w.lo), hi=tuple(int(v * s) for v in w.hi),
                   box_half=w.box_half * s)


def porosity_noise(w: Workload) -> np.ndarray | None:
    """Per-cell noise values (one per cell, cell = x + nx*(y + ny*z))."""
    if w.noise_mode == NOISE_NONE:
        return None
    rng = np.random.default_rng(w.noise_seed)
    if w.noise_mode == NOISE_RIM:
        return rng.uniform(-w.noise_amp, w.noise_amp, w.n)
    return rng.uniform(0.0, w.noise_amp, w.n)


def initial_velocity(w: Workload) -> np.ndarray | None:
    """Uniform inflow plus seeded noise for the 3D case ([3, n]), else None
    (the inlet profile continued into the domain)."""
    if w.velocity_noise <= 0.0:
        return None
    rng = np.random.default_rng(w.noise_seed)
    u = w.velocity_noise * rng.uniform(-1.0, 1.0, (3, w.n))
    u[0] += w.u_max
    return u


def random_populations(q_weights: np.ndarray, n: int, amp: float, seed: int) -> np.ndarray:
    """f_i = w_i (1 + amp U(-1, 1)) for test states ([q, n])."""
    rng = np.random.default_rng(seed)
    return np.outer(q_weights, np.ones(n)) * (1.0 + amp * rng.uniform(-1, 1, (len(q_weights), n)))


def random_porosity(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)
