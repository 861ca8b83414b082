"""Exact FP64 enumeration of the shaken dynamics on tiny tori.  TEST INFRASTRUCTURE ONLY.

Everything here is written from the definitions of section 2 of the paper,
with no reference to how the sampler is implemented:

* the pair Hamiltonian H(sigma, tau) = -sum_x [J sigma_x (tau_up + tau_right)
  + q sigma_x tau_x], eq. (5) (its second form is checked against the first);
* the Gibbs measure pi_2 ~ exp(-H), eq. (6);
* the half-step kernels P((sigma,tau),(sigma,tau')) = e^{-H(sigma,tau')}/Z_sigma
  and P((sigma,tau),(sigma',tau)) = e^{-H(sigma',tau)}/Z_tau, eqs. (15)-(16);
* the shaken marginal P_sq(sigma, sigma') = sum_tau K_A(sigma->tau) K_B(tau->sigma')
  (the displayed formula after eq. (16), with its first denominator read as
  Z_sigma) and its stationary law pi_s(sigma) = Z_sigma / Z;
* the honeycomb partition-function product form, eq. (8).

Only L <= 3 is practical (2^(L*L) states per sub-lattice).  L = 2 alone cannot
tell up from down (both are the same neighbour on a 2x2 torus), so the tests
use L = 3 for anything orientation-dependent.
"""
from __future__ import annotations

import itertools

import numpy as np


def configurations(L: int) -> np.ndarray:
    """All 2^(L*L) spin configurations, shape [2^N, L, L], entry +1/-1.
    Configuration index c has site s = j*L + i equal to +1 iff bit s of c is 1."""
    N = L * L
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1
    return (2 * bits - 1).astype(np.int64).reshape(-1, L, L)


def config_index(lattice: np.ndarray) -> int:
    flat = (np.asarray(lattice).reshape(-1) > 0).astype(np.int64)
    return int(np.sum(flat << np.arange(flat.size)))


def _up(x):     # value at (i, j+1) seen from (i, j); rows are j, columns i
    return np.roll(x, -1, axis=-2)


def _right(x):  # value at (i+1, j)
    return np.roll(x, -1, axis=-1)


def _down(x):   # value at (i, j-1)
    return np.roll(x, 1, axis=-2)


def _left(x):   # value at (i-1, j)
    return np.roll(x, 1, axis=-1)


def hamiltonian_matrix(L: int, J: float, q: float) -> np.ndarray:
    """H[a, b] = H(sigma_a, tau_b), first form of eq. (5)."""
    S = configurations(L).astype(np.float64)
    n = S.shape[0]
    # sum_x sigma_x (tau_up + tau_right): bilinear in (sigma, tau)
    Tn = (_up(S) + _right(S)).reshape(n, -1)
    Sf = S.reshape(n, -1)
    A = Sf @ Tn.T
    B = Sf @ Sf.T
    return -(J * A + q * B)


def hamiltonian_matrix_second_form(L: int, J: float, q: float) -> np.ndarray:
    """H[a, b] from the second form of eq. (5): -sum_x [J tau_x (sigma_down + sigma_left) + q tau_x sigma_x]."""
    S = configurations(L).astype(np.float64)
    n = S.shape[0]
    Sn = (_down(S) + _left(S)).reshape(n, -1)
    Sf = S.reshape(n, -1)
    A = Sn @ Sf.T          # [a, b] = sum_x (sigma_a down+left)_x tau_b,x
    B = Sf @ Sf.T
    return -(J * A + q * B)


class Enumeration:
    """All exact objects of the pair model at one (L, J, q)."""

    def __init__(self, L: int, J: float, q: float):
        self.L, self.J, self.q = L, J, q
        H = hamiltonian_matrix(L, J, q)
        self.H = H
        W = np.exp(-H)                       # W[sigma, tau]
        self.W = W
        self.Z_sigma = W.sum(axis=1)         # Z_sigma = sum_eta e^{-H(sigma, eta)}
        self.Z_tau = W.sum(axis=0)           # Z_tau   = sum_eta e^{-H(eta, tau)}
        self.Z = W.sum()
        self.K_A = W / self.Z_sigma[:, None]         # sigma -> tau
        self.K_B = (W / self.Z_tau[None, :]).T       # tau -> sigma'
        self.P_shaken = self.K_A @ self.K_B          # sigma -> sigma'
        self.pi_s = self.Z_sigma / self.Z
        self.pi_2 = W / self.Z                       # pi_2[sigma, tau]

    def pair_chain(self) -> np.ndarray:
        """Transition matrix of the alternate dynamics on pairs (sigma, tau) ->
        (sigma', tau'): tau' ~ K_A(sigma, .), then sigma' ~ K_B(tau', .).
        Pair index = a * n + b for (sigma_a, tau_b)."""
        n = self.W.shape[0]
        P = np.zeros((n * n, n * n))
        for a in range(n):
            # from (sigma_a, any tau): tau' = b', sigma' = a'
            row = (self.K_A[a][:, None] * self.K_B)          # [b', a']
            block = row.T.reshape(-1)                         # index a'*n + b'
            for b in range(n):
                P[a * n + b] = block
        return P


def honeycomb_partition_function(L: int, J: float, q: float) -> float:
    """Eq. (8): Z = sum over (sigma, tau) of prod_u cosh^2 J cosh q (1 + sigma tau_up tanh J)
    (1 + sigma tau_right tanh J)(1 + sigma tau tanh q)."""
    S = configurations(L).astype(np.float64)
    n = S.shape[0]
    tJ, tq = np.tanh(J), np.tanh(q)
    pref = (np.cosh(J) ** 2 * np.cosh(q)) ** (L * L)
    total = 0.0
    for a in range(n):
        s = S[a]
        f = (1 + s[None] * _up(S) * tJ) * (1 + s[None] * _right(S) * tJ) * (1 + s[None] * S * tq)
        total += np.prod(f.reshape(n, -1), axis=1).sum()
    return pref * total


def implemented_half_step_matrix(thresholds: np.ndarray) -> np.ndarray:
    """Transition matrix of one half-step drawn as dst_x = +1 iff r_x < T_x with
    r_x independent uniforms on [0, 2^32): thresholds[a] is the [L, L] array of
    per-site thresholds from source configuration a."""
    n = thresholds.shape[0]
    L = thresholds.shape[1]
    p_plus = thresholds.reshape(n, -1).astype(np.float64) / 2.0 ** 32   # [a, site]
    D = configurations(L).reshape(n, -1) > 0                            # [b, site]
    logp = np.log(p_plus)[:, None, :]
    logm = np.log1p(-p_plus)[:, None, :]
    return np.exp(np.where(D[None], logp, logm).sum(axis=2))


def all_sites(L: int):
    return list(itertools.product(range(L), range(L)))
