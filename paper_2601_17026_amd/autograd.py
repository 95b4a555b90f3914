"""Differentiable optimal-surface energy.

`SurfaceEnergy.apply(cost, delta, scale, alpha)` takes a float32 CUDA tensor
of shape (B, nx, ny, K), quantises it to int32 costs c_i = round(scale *
cost) (torch rounds half to even), solves the B volumes exactly as one batch
with the C-ABI library (smf_batch_solve) and returns (E, h):
E[b] = (sum_p c_i[b](p, h_b(p)) + a_i * sum |h_b(p) - h_b(q)|) / scale as
float32, with the soft smoothness weight a_i = round(scale * alpha) over
4-neighbour columns (alpha = 0: the hard bound only), and the
pointwise-lowest optimal surface h (int32, not differentiable).

E is a minimum of functions linear in the costs (Section 1.1, Eq. 1; the
smoothness term does not depend on them), so its gradient is the one-hot
indicator of the optimal height of each column (exact where the column's
optimal height is unique, a supergradient otherwise).  The backward pass
passes it straight through the quantisation and runs as the library's HIP
scatter kernel (smf_onehot_backward).
"""
from __future__ import annotations

import torch

from . import smf

_SOLVERS: dict = {}


def _solver(device: int, B: int, nx: int, ny: int, K: int, delta: int) -> smf.BatchSolver:
    """A cached batch handle on GPU `device` for B volumes of one shape."""
    key = (device, B, nx, ny, K, delta)
    s = _SOLVERS.get(key)
    if s is None:
        with torch.cuda.device(device):
            s = smf.BatchSolver([(nx, ny, K, delta)] * B)
        _SOLVERS[key] = s
    return s


def quantize(cost: torch.Tensor, scale: float = 16.0) -> torch.Tensor:
    """int32 costs round(scale * cost) (half to even)."""
    return torch.round(cost * scale).to(torch.int32).contiguous()


class SurfaceEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost: torch.Tensor, delta: int, scale: float = 16.0, alpha: float = 0.0):
        if cost.dim() != 4 or cost.device.type != "cuda":
            raise ValueError("cost must be a (B, nx, ny, K) CUDA tensor")
        B, nx, ny, K = cost.shape
        ci = quantize(cost.detach().float(), scale)
        solver = _solver(cost.device.index, B, nx, ny, K, int(delta))
        solver.set_param_per_volume("smooth_weight", [soft_weight(alpha, scale)] * B)
        h = torch.empty((B, nx, ny), dtype=torch.int32, device=cost.device)
        solver.solve(ci.view(-1))
        solver.surfaces(out=h.view(-1))
        E = torch.tensor([e / scale for e in solver.energies()], dtype=torch.float32,
                         device=cost.device)
        ctx.save_for_backward(h)
        ctx.K = K
        ctx.mark_non_differentiable(h)
        return E, h

    @staticmethod
    def backward(ctx, grad_E, grad_h):
        (h,) = ctx.saved_tensors
        g = grad_E.detach().float().contiguous()
        grad = smf.onehot_backward(h, g, ctx.K)
        return grad, None, None, None


def soft_weight(alpha: float, scale: float = 16.0) -> int:
    """The integer soft smoothness weight round(scale * alpha) (half to even)."""
    return int(torch.round(torch.tensor(float(alpha)) * scale).item())


def surface_energy(cost: torch.Tensor, delta: int, scale: float = 16.0, alpha: float = 0.0):
    return SurfaceEnergy.apply(cost, delta, scale, alpha)
