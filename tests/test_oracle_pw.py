"""Pins of the oracle's coupling-from-the-past sampler (Propp-Wilson, the
exact sampler section 3.2 builds on the monotone coupling).

* Exactness: on the 2x2 and 3x3 tori the samples follow the stationary law
  pi_s of the shaken chain, computed by exact enumeration (chi-square over
  the number of +1 spins and over the states).
* The defining property: every chain started at time -T (the returned T)
  reaches the sample at time 0, and so does the pair started at -2T.
* Sandwiching before coalescence, the T_max cut-off and the argument checks.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import enumerate as en

STEP_END = 1 << 20


def _chi2_p(counts, expected):
    keep = expected >= 5.0
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(expected[keep], expected[~keep].sum())
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    return stats.chi2.sf(((obs - exp) ** 2 / exp).sum(), len(obs) - 1)


@pytest.mark.parametrize("L,J,q", [(2, 0.7, 0.5), (3, 0.5, 0.4)])
def test_samples_follow_the_stationary_law(oracle, L, J, q):
    N = 20000
    ex = en.Enumeration(L, J, q)
    n_states = 2 ** (L * L)
    confs = en.configurations(L).reshape(n_states, -1)
    n_plus = (confs > 0).sum(axis=1)
    counts = np.zeros(n_states)
    for s in range(N):
        x, T = oracle.propp_wilson(L, J, q, 5, s, STEP_END, 1, STEP_END)
        assert T > 0
        counts[en.config_index(x)] += 1
    expected = ex.pi_s * N
    by_plus = np.array([counts[n_plus == k].sum() for k in range(L * L + 1)])
    exp_plus = np.array([expected[n_plus == k].sum() for k in range(L * L + 1)])
    assert _chi2_p(by_plus, exp_plus) > 1e-3
    assert _chi2_p(counts, expected) > 1e-3


def test_every_chain_started_at_minus_T_reaches_the_sample(oracle):
    L, J, q = 8, 0.4, 0.5
    rng = np.random.default_rng(3)
    for stream in range(4):
        x, T = oracle.propp_wilson(L, J, q, 9, stream, STEP_END, 2, 1 << 12)
        assert T > 0
        for _ in range(3):
            start = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L))
            end, _, _ = oracle.run(start, J, q, 9, stream, STEP_END - T, T)
            assert np.array_equal(end, x)
        for kind in (0, 1):   # the extreme pair from -2T agrees too
            end, _, _ = oracle.run(oracle.init(L, kind), J, q, 9, stream, STEP_END - 2 * T, 2 * T)
            assert np.array_equal(end, x)


def test_sandwich_before_coalescence(oracle):
    L, J, q, T = 8, 0.6, 0.6, 3
    rng = np.random.default_rng(4)
    top, _, _ = oracle.run(oracle.init(L, 0), J, q, 1, 0, STEP_END - T, T)
    bot, _, _ = oracle.run(oracle.init(L, 1), J, q, 1, 0, STEP_END - T, T)
    assert not np.array_equal(top, bot)
    for _ in range(5):
        start = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L))
        mid, _, _ = oracle.run(start, J, q, 1, 0, STEP_END - T, T)
        assert np.all(bot <= mid) and np.all(mid <= top)


def test_uncoupled_sites_coalesce_in_one_step(oracle):
    # J = q = 0: every spin is +1 iff the top bit of its uniform is 0, whatever
    # the lattice, so the pair from -T0 agrees at once and the sample is the
    # last half-step of step step_end - 1
    L = 8
    x, T = oracle.propp_wilson(L, 0.0, 0.0, 2, 6, STEP_END, 4, 64)
    assert T == 4
    t = 2 * (STEP_END - 1) + 1
    expect = np.array([[1 if oracle.site_uniform(2, 6, t, 0, j * L + i) < 2 ** 31 else -1 for i in range(L)]
                       for j in range(L)], dtype=np.int8)
    assert np.array_equal(x, expect)


def test_cut_off_and_bad_arguments(oracle):
    L, J, q = 8, 1.5, 1.0
    x, T = oracle.propp_wilson(L, J, q, 1, 0, STEP_END, 1, 4)
    assert T == 0
    top, _, _ = oracle.run(oracle.init(L, 0), J, q, 1, 0, STEP_END - 4, 4)
    assert np.array_equal(x, top)
    for args in [(L, -0.1, q, 1, 0, STEP_END, 1, 4), (L, J, q, 1, 0, 3, 1, 4), (L, J, q, 1, 0, STEP_END, 0, 4),
                 (L, J, q, 1, 0, STEP_END, 8, 4), (L, J, float("nan"), 1, 0, STEP_END, 1, 4)]:
        with pytest.raises(ValueError):
            oracle.propp_wilson(*args)
