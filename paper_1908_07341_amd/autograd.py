"""torch.autograd.Function over the log-likelihood kernels.

Forward runs sd_loglik_fwd on the 12 exact counts, backward runs
sd_loglik_bwd; both are HIP kernels, this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import binding as B


class LogLik(torch.autograd.Function):
    """LL(J, q) of a set of trajectories given their counts (see sd_loglik_counts).

    Jq: float32 tensor [2] = (J, q) on the GPU; counts: int64 tensor [12].
    Returns a float32 scalar tensor; gradients flow to Jq only."""

    @staticmethod
    def forward(ctx, Jq: torch.Tensor, counts: torch.Tensor) -> torch.Tensor:
        if Jq.dtype != torch.float32 or Jq.numel() != 2 or not Jq.is_cuda:
            raise ValueError("Jq must be a float32 CUDA tensor of two elements")
        if counts.dtype != torch.int64 or counts.numel() != 12 or not counts.is_cuda:
            raise ValueError("counts must be an int64 CUDA tensor of 12 elements")
        Jq = Jq.detach().contiguous()
        counts = counts.contiguous()
        ll = torch.empty(1, dtype=torch.float32, device=Jq.device)
        B.sd_loglik_fwd(counts, Jq, ll)
        ctx.save_for_backward(counts, Jq)
        return ll.reshape(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        counts, Jq = ctx.saved_tensors
        g = grad_out.detach().reshape(1).to(torch.float32).contiguous()
        grad = torch.empty(2, dtype=torch.float32, device=Jq.device)
        B.sd_loglik_bwd(counts, Jq, g, grad)
        return grad, None


def loglik_counts(traj: torch.Tensor, n_traj: int, n_lat: int, L: int) -> torch.Tensor:
    """12 int64 counts of packed trajectories traj[n_traj][n_lat][L][L/64]."""
    counts = torch.empty(12, dtype=torch.int64, device=traj.device)
    B.sd_loglik_counts(traj, n_traj, n_lat, L, counts)
    return counts


def loglik(Jq: torch.Tensor, counts: torch.Tensor) -> torch.Tensor:
    return LogLik.apply(Jq, counts)
