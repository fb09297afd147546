"""``torch.autograd.Function`` over the radiative-transfer subcycle.

``RTSubcycles.apply(log_lum, log_nH, problem)`` runs ``problem.n_subcycles``
FP64 subcycles through the C ABI and returns the final neutral fraction x_HI
(a float64 CUDA tensor).  Its backward calls ``rt_subcycle_adjoint``: the
gradients of a loss of x_HI with respect to the natural log of every
source's luminosity (all bins of a source scaled together) and the natural
log of the initial hydrogen density.  Torch supplies only device memory and
the stream; every step runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rt


class Problem:
    """Mesh, parameters and initial fields of a differentiable run.

    ``cfg`` is a workload dict (see rtgen); source rates are split over bins
    in the proportions of cfg["sources"]["rate"]: rate[b, k] = exp(log_lum[k])
    * split[b, k] with split = rate / rate.sum(0)."""

    def __init__(self, cfg: dict, n_subcycles: int | None = None, checkpoint_every: int = 10, device: int = 0,
                 dt: float = 0.0):
        self.cfg = cfg
        self.mesh = rt.Mesh(cfg["mesh"], device=device)
        self.params = rt.params_from_dict(cfg["params"])
        rate = np.asarray(cfg["sources"]["rate"], dtype=float).reshape(cfg["params"]["nb"], -1)
        tot = rate.sum(0)
        self.split = rate / np.where(tot > 0, tot, 1.0)[None, :]
        self.log_lum0 = np.log(np.where(tot > 0, tot, 1.0))
        self.n_subcycles = cfg["n_subcycles"] if n_subcycles is None else int(n_subcycles)
        self.checkpoint_every = int(checkpoint_every)
        self.dt = float(dt)          # subcycle length; <= 0: the CFL step

    def state(self, log_lum: np.ndarray, log_nH: np.ndarray) -> rt.State:
        st = self.cfg["state"]
        rate = np.ascontiguousarray(self.split * np.exp(log_lum)[None, :])
        return rt.State(self.mesh, self.params, rt.RT_FP64, st["N"], st["F"], np.exp(log_nH), st["species"], st["T"],
                        self.cfg["sources"]["cell"], rate)


class RTSubcycles(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_lum: torch.Tensor, log_nH: torch.Tensor, problem: Problem) -> torch.Tensor:
        s0 = problem.state(log_lum.detach().cpu().double().numpy(), log_nH.detach().cpu().double().numpy())
        run = s0.clone()
        run.subcycle(problem.n_subcycles, problem.dt, stream=torch.cuda.current_stream())
        out = torch.empty(problem.mesh.n_cells, dtype=torch.float64, device="cuda")
        x = torch.empty((5, problem.mesh.n_cells), dtype=torch.float64, device="cuda")
        rt.rt_state_get_field(run.h, rt.RT_FIELD_SPECIES, x)
        out.copy_(x[0])
        run.close()
        ctx.problem = problem
        ctx.s0 = s0          # released with the graph (State frees its handle when collected)
        ctx.n_src = log_lum.shape[0]
        return out

    @staticmethod
    def backward(ctx, grad_x: torch.Tensor):
        problem = ctx.problem
        g = grad_x.detach().to(device="cuda", dtype=torch.float64).contiguous()
        d_lum = torch.zeros(max(ctx.n_src, 1), dtype=torch.float64, device="cuda")
        d_nH = torch.zeros(problem.mesh.n_cells, dtype=torch.float64, device="cuda")
        torch.cuda.current_stream().synchronize()
        # The initial state is not modified by the adjoint, so a second
        # backward (retain_graph=True) can use it again.
        rt.rt_subcycle_adjoint(ctx.s0.h, problem.n_subcycles, problem.checkpoint_every, g,
                               d_lum if ctx.n_src else None, d_nH, torch.cuda.current_stream(), dt=problem.dt)
        return d_lum[:ctx.n_src], d_nH, None
