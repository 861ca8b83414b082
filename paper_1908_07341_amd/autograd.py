"""torch.autograd.Function over the log-likelihood kernels.

Forward runs sd_loglik_fwd (12 exact counts) or sd_loglik_fwd_stats (6 paired
statistics), backward the matching sd_loglik_bwd / sd_loglik_bwd_stats; all
are HIP kernels, this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import binding as B

_FWD = {12: B.sd_loglik_fwd, 6: B.sd_loglik_fwd_stats}
_BWD = {12: B.sd_loglik_bwd, 6: B.sd_loglik_bwd_stats}


class LogLik(torch.autograd.Function):
    """LL(J, q) of a set of trajectories given their sufficient statistics:
    the 12 counts of sd_loglik_counts or the 6 paired statistics of
    sd_loglik_stats (told apart by their length).

    Jq: float32 tensor [2] = (J, q) on the GPU; stats: int64 tensor [12] or [6].
    Returns a float32 scalar tensor; gradients flow to Jq only."""

    @staticmethod
    def forward(ctx, Jq: torch.Tensor, stats: torch.Tensor) -> torch.Tensor:
        if Jq.dtype != torch.float32 or Jq.numel() != 2 or not Jq.is_cuda:
            raise ValueError("Jq must be a float32 CUDA tensor of two elements")
        if stats.dtype != torch.int64 or stats.numel() not in _FWD or not stats.is_cuda:
            raise ValueError("stats must be an int64 CUDA tensor of 12 counts or 6 paired statistics")
        Jq = Jq.detach().contiguous()
        stats = stats.contiguous()
        ll = torch.empty(1, dtype=torch.float32, device=Jq.device)
        _FWD[stats.numel()](stats, Jq, ll)
        ctx.save_for_backward(stats, Jq)
        return ll.reshape(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        stats, Jq = ctx.saved_tensors
        g = grad_out.detach().reshape(1).to(torch.float32).contiguous()
        grad = torch.empty(2, dtype=torch.float32, device=Jq.device)
        _BWD[stats.numel()](stats, Jq, g, grad)
        return grad, None


def loglik_counts(traj: torch.Tensor, n_traj: int, n_lat: int, L: int) -> torch.Tensor:
    """12 int64 counts of packed trajectories traj[n_traj][n_lat][L][L/64]."""
    counts = torch.empty(12, dtype=torch.int64, device=traj.device)
    B.sd_loglik_counts(traj, n_traj, n_lat, L, counts)
    return counts


def loglik_stats(traj: torch.Tensor, n_traj: int, n_lat: int, L: int) -> torch.Tensor:
    """6 int64 paired statistics (S_0..S_2, Z_0..Z_2) of the same trajectories."""
    stats = torch.empty(6, dtype=torch.int64, device=traj.device)
    B.sd_loglik_stats(traj, n_traj, n_lat, L, stats)
    return stats


def loglik(Jq: torch.Tensor, stats: torch.Tensor) -> torch.Tensor:
    return LogLik.apply(Jq, stats)
