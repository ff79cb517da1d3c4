"""torch.autograd.Function over the HLBM objective: forward = primal sweep
(steady, or spin-up plus FP64 window) -> J; backward = adjoint sweep on the
frozen steady/mean flow -> dJ/dd (Sec. 3.2-3.3, Eqs. adjoint_steady /
adjoint_unsteady and gradients_steady / gradients_unsteady).

No primal trajectory is stored: the backward pass only needs the converged
or window-mean state the lattice keeps on the device.  All arithmetic runs in
libhlbm.so; this module passes device pointers and torch's current stream.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import hlbm as H


@dataclass
class Plan:
    """How one objective evaluation is run.

    window_steps = 0: steady objective J(f*) after at most primal_steps steps
    (stopping early once the steady criterion steady_tol is met; 0 runs all
    steps).  window_steps > 0: spin-up of primal_steps - window_steps steps,
    then the mean of J over window_steps steps (mean-flow adjoint).
    initial_populations: the state the primal starts from (q x n float64,
    canonical layout, host or device); None starts from the equilibrium
    f^eq(1, d u_in) of the lattice's inlet profile.
    """
    primal_steps: int = 20000
    window_steps: int = 0
    steady_tol: float = 0.0
    check_every: int = 500
    adjoint_iters: int = 20000
    adjoint_tol: float = 0.0
    tau_adj: float = 0.0
    turb: int = H.TURB_FROZEN
    initial_populations: object = None


def make_lattice(stencil=H.D2Q9, precision=H.FP64, **kw) -> H.Lattice:
    """A lattice whose kernels run on torch's current stream."""
    stream = torch.cuda.current_stream().cuda_stream
    return H.Lattice(stencil=stencil, precision=precision, stream=stream, **kw)


class HLBMObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d: torch.Tensor, lat: H.Lattice, plan: Plan):
        if not d.is_cuda:
            raise ValueError("porosity must be a CUDA tensor")
        dd = d.detach().to(torch.float64).contiguous().view(-1)
        lat.set_porosity(dd)
        if plan.initial_populations is not None:
            lat.set_populations(plan.initial_populations)
        else:
            lat.init_equilibrium()
        if plan.window_steps > 0:
            lat.run_primal(plan.primal_steps - plan.window_steps)
            lat.run_primal(plan.window_steps, accumulate=True)
            J = lat.objective(1)
        else:
            lat.run_primal(plan.primal_steps, steady_tol=plan.steady_tol, check_every=plan.check_every)
            J = lat.objective(0)
        ctx.lat, ctx.plan, ctx.shape = lat, plan, d.shape
        # the backward adjoint runs on the state the lattice holds then: it
        # must still be the one this forward produced
        ctx.generation = lat.generation
        return torch.tensor(J, dtype=torch.float64, device=d.device)

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        lat, plan = ctx.lat, ctx.plan
        if lat.generation != ctx.generation:
            raise RuntimeError("the lattice was changed (porosity, state or primal steps) after this objective's "
                               "forward pass; its backward would differentiate another state. Run backward first, "
                               "or give each objective evaluation its own lattice")
        source = H.SOURCE_MEAN if plan.window_steps > 0 else H.SOURCE_STEADY
        lat.solve_adjoint(source, tau_adj=plan.tau_adj, turb=plan.turb, max_iters=plan.adjoint_iters,
                          tol=plan.adjoint_tol, check_every=max(2, plan.check_every))
        g = torch.empty(lat.n, dtype=torch.float64, device=gJ.device)
        lat.gradient(out=g)
        return (gJ * g).view(ctx.shape), None, None


def objective(d: torch.Tensor, lat: H.Lattice, plan: Plan) -> torch.Tensor:
    """J(d) as a differentiable scalar (float64)."""
    return HLBMObjective.apply(d, lat, plan)


def objective_batch(d: torch.Tensor, lats: list, plan: Plan) -> torch.Tensor:
    """J for a batch of porosity fields d[B, ...] on B resident lattices."""
    if d.shape[0] != len(lats):
        raise ValueError("one lattice per field")
    return torch.stack([HLBMObjective.apply(d[b], lats[b], plan) for b in range(len(lats))])
