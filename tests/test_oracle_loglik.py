"""Pins of the trajectory log-likelihood machinery.

* The count-based LL equals the sum of log transition probabilities read off
  the exact half-step kernels of the enumeration (3x3 torus).
* The analytic gradient matches FP64 central differences.
* The LL is concave, and its maximiser on trajectories generated at a known
  (J, q) recovers that point within three standard errors (Fisher information
  from the closed-form Hessian).
"""
import math

import numpy as np
import pytest

from oracle import enumerate as en

SEED = 99


def test_counts_cover_every_transition(oracle):
    L, k = 8, 5
    traj = np.stack([oracle.trajectory(oracle.init(L, 2, 0.5, 1, a), 0.4, 0.6, SEED, a, 0, k) for a in range(3)])
    c = oracle.loglik_counts(traj)
    assert c.sum() == 3 * 2 * k * L * L
    assert np.all(c >= 0)


@pytest.mark.parametrize("J,q", [(0.4, 0.6), (1.1, 0.3), (0.0, 0.8)])
def test_loglik_equals_exact_transition_log_probabilities(oracle, J, q):
    L, k = 3, 6
    ex = en.Enumeration(L, J, q)
    traj = oracle.trajectory(oracle.init(L, 2, 0.5, 4, 1), J, q, SEED, 1, 0, k)
    exact = 0.0
    for m in range(2 * k):
        a, b = en.config_index(traj[m]), en.config_index(traj[m + 1])
        K = ex.K_A if m % 2 == 0 else ex.K_B
        exact += math.log(K[a, b])
    c = oracle.loglik_counts(traj[None])
    # evaluate at a second parameter point too: the counts are sufficient statistics
    assert math.isclose(oracle.loglik(c, J, q), exact, rel_tol=1e-12, abs_tol=1e-10)
    ex2 = en.Enumeration(L, J + 0.3, q + 0.1)
    exact2 = sum(math.log((ex2.K_A if m % 2 == 0 else ex2.K_B)[en.config_index(traj[m]), en.config_index(traj[m + 1])])
                 for m in range(2 * k))
    assert math.isclose(oracle.loglik(c, J + 0.3, q + 0.1), exact2, rel_tol=1e-12, abs_tol=1e-10)


def _counts_at(oracle, J, q, L, n_traj, k, stream0=0):
    traj = np.stack([oracle.trajectory(oracle.init(L, 2, 0.5, 1, stream0 + a), J, q, SEED, stream0 + a, 0, k)
                     for a in range(n_traj)])
    return oracle.loglik_counts(traj)


def test_gradient_matches_central_differences(oracle):
    c = _counts_at(oracle, 0.45, 0.7, 16, 2, 10)
    for J, q in [(0.2, 0.2), (0.45, 0.7), (1.0, 1.5), (0.0, 0.0)]:
        g = oracle.loglik_grad(c, J, q)
        eps = 1e-5
        fdJ = (oracle.loglik(c, J + eps, q) - oracle.loglik(c, J - eps, q)) / (2 * eps)
        fdq = (oracle.loglik(c, J, q + eps) - oracle.loglik(c, J, q - eps)) / (2 * eps)
        scale = np.abs(c).sum() * 2.0
        assert abs(g[0] - fdJ) <= 1e-7 * scale, (J, q, g[0], fdJ)
        assert abs(g[1] - fdq) <= 1e-7 * scale, (J, q, g[1], fdq)


def _hessian(c, J, q):
    H = np.zeros((2, 2))
    for k in range(3):
        for cp in range(2):
            a, b = 2 * k - 2, 2 * cp - 1
            h = J * a + q * b
            n = c[2 * (2 * k + cp)] + c[2 * (2 * k + cp) + 1]
            w = n / math.cosh(h) ** 2
            H -= w * np.array([[a * a, a * b], [a * b, b * b]])
    return H


def test_loglik_concave(oracle):
    c = _counts_at(oracle, 0.45, 0.7, 16, 2, 10)
    for J, q in [(0.2, 0.2), (0.45, 0.7), (2.0, 0.1)]:
        ev = np.linalg.eigvalsh(_hessian(c, J, q))
        assert ev.max() < 0
    # and the closed-form Hessian matches differences of the analytic gradient
    eps = 1e-5
    H = _hessian(c, 0.45, 0.7)
    gJp, gJm = oracle.loglik_grad(c, 0.45 + eps, 0.7), oracle.loglik_grad(c, 0.45 - eps, 0.7)
    assert np.allclose((gJp - gJm) / (2 * eps), H[:, 0], rtol=1e-5)


@pytest.mark.slow
def test_mle_recovers_generating_parameters(oracle):
    J0, q0 = 0.45, 0.7
    c = _counts_at(oracle, J0, q0, 32, 4, 150, stream0=10)
    theta = np.array([0.2, 0.2])
    for _ in range(30):   # Newton ascent on a concave objective
        g = oracle.loglik_grad(c, *theta)
        theta = theta - np.linalg.solve(_hessian(c, *theta), g)
    cov = np.linalg.inv(-_hessian(c, *theta))
    se = np.sqrt(np.diag(cov))
    assert np.linalg.norm(oracle.loglik_grad(c, *theta)) < 1e-6 * c.sum()
    assert abs(theta[0] - J0) < 3 * se[0], (theta, se)
    assert abs(theta[1] - q0) < 3 * se[1], (theta, se)


def _pair_map(c):
    """Linear map from the 12 transition counts (class 2k + [c = +1], drawn
    spin) to the paired statistics: the pair is (j, 5 - j), j = 0, 1, 2."""
    S = [c[2 * j] + c[2 * j + 1] + c[2 * (5 - j)] + c[2 * (5 - j) + 1] for j in range(3)]
    Z = [c[2 * j + 1] + c[2 * (5 - j)] for j in range(3)]
    return np.array(S + Z, dtype=np.int64)


@pytest.mark.parametrize("L,k", [(3, 6), (8, 5), (10, 3)])
def test_paired_stats_are_the_pair_map_of_the_counts(oracle, L, k):
    traj = np.stack([oracle.trajectory(oracle.init(L, 2, 0.5, 1, a), 0.4, 0.6, SEED, a, 0, k) for a in range(3)])
    s = oracle.loglik_stats(traj)
    assert np.array_equal(s, _pair_map(oracle.loglik_counts(traj)))
    assert s[:3].sum() == 3 * 2 * k * L * L
    assert np.all(s[3:] <= s[:3]) and np.all(s[3:] >= 0)


@pytest.mark.parametrize("J,q", [(0.4, 0.6), (1.1, -0.3), (0.0, 0.8)])
def test_paired_loglik_equals_exact_transition_log_probabilities(oracle, J, q):
    L, k = 3, 6
    traj = oracle.trajectory(oracle.init(L, 2, 0.5, 4, 1), J, q, SEED, 1, 0, k)
    s = oracle.loglik_stats(traj[None])
    for Je, qe in [(J, q), (J - 0.2, q + 0.5)]:
        ex = en.Enumeration(L, Je, qe)
        exact = sum(math.log((ex.K_A if m % 2 == 0 else ex.K_B)[en.config_index(traj[m]), en.config_index(traj[m + 1])])
                    for m in range(2 * k))
        ll, _ = oracle.loglik_from_stats(s, Je, qe)
        assert math.isclose(ll, exact, rel_tol=1e-12, abs_tol=1e-10)


def test_paired_gradient_matches_central_differences(oracle):
    traj = np.stack([oracle.trajectory(oracle.init(16, 2, 0.5, 1, a), 0.45, 0.7, SEED, a, 0, 10) for a in range(2)])
    s = oracle.loglik_stats(traj)
    scale = 2.0 * s[:3].sum()
    for J, q in [(0.2, 0.2), (0.45, 0.7), (1.0, -1.5), (0.0, 0.0)]:
        _, g = oracle.loglik_from_stats(s, J, q)
        eps = 1e-5
        fdJ = (oracle.loglik_from_stats(s, J + eps, q)[0] - oracle.loglik_from_stats(s, J - eps, q)[0]) / (2 * eps)
        fdq = (oracle.loglik_from_stats(s, J, q + eps)[0] - oracle.loglik_from_stats(s, J, q - eps)[0]) / (2 * eps)
        assert abs(g[0] - fdJ) <= 1e-7 * scale, (J, q, g[0], fdJ)
        assert abs(g[1] - fdq) <= 1e-7 * scale, (J, q, g[1], fdq)
