"""Statistical pins of the oracle chain.  Seeds are fixed, so each test is a
deterministic pass/fail; thresholds sit at roughly the 1e-4 tail."""
import math

import numpy as np

from oracle import enumerate as en

SEED = 77


def _visits(oracle, L, J, q, n_steps, thin, stream):
    sigma = oracle.init(L, 2, 0.5, 1, stream)
    counts = np.zeros(2 ** (L * L), dtype=np.int64)
    for n in range(n_steps):
        tau = oracle.half_step(sigma, J, q, 0, SEED, stream, 2 * n)
        sigma = oracle.half_step(tau, J, q, 1, SEED, stream, 2 * n + 1)
        if n % thin == 0:
            counts[en.config_index(sigma)] += 1
    return counts


def _chi2(counts, p):
    n = counts.sum()
    e = n * p
    return float(((counts - e) ** 2 / e).sum())


def test_visit_frequencies_match_pi_s_L2(oracle):
    ex = en.Enumeration(2, 0.4, 0.6)
    c = _visits(oracle, 2, 0.4, 0.6, 60000, 3, stream=1)
    chi2 = _chi2(c, ex.pi_s)
    assert chi2 < 45, chi2   # 15 dof


def test_visit_frequencies_match_pi_s_L3(oracle):
    ex = en.Enumeration(3, 0.3, 0.4)
    c = _visits(oracle, 3, 0.3, 0.4, 120000, 3, stream=2)
    chi2 = _chi2(c, ex.pi_s)
    assert chi2 < 511 + 4.5 * math.sqrt(2 * 511), chi2


def test_J_zero_magnetisation_decay(oracle):
    # J = 0: E[m_n] = tanh(q)^(2n) from the all-up start, and the recorded
    # pair has E[sigma_x tau_x] = tanh(q) at every step.
    L, q, n_chains, k = 32, 0.9, 40, 4
    m = np.zeros(k)
    b = np.zeros(k)
    for c in range(n_chains):
        _, _, obs = oracle.run(np.ones((L, L), np.int8), 0.0, q, SEED, 100 + c, 0, k, obs_every=1)
        m += obs[:, 0] / (L * L)
        b += obs[:, 2] / (L * L)
    m /= n_chains
    b /= n_chains
    N = L * L * n_chains
    for n in range(k):
        expect = math.tanh(q) ** (2 * (n + 1))
        assert abs(m[n] - expect) < 5 / math.sqrt(N), (n, m[n], expect)
        assert abs(b[n] - math.tanh(q)) < 5 / math.sqrt(N), (n, b[n])
