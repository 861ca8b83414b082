"""Exact-enumeration pins (FP64) on 2x2 and 3x3 tori.

The enumeration module is checked against facts of section 2 that do not
depend on how it is written (second form of the Hamiltonian, product form of
the partition function, stationarity and reversibility of the shaken marginal,
equality of pi_s and the sigma-marginal of pi_2).  The oracle's half-step
thresholds are then turned into transition matrices and compared with the
exact half-step kernels: they must agree to within N * 2^-33 per entry, N the
number of sites, since each per-site probability is rounded by at most 2^-33.
"""
import numpy as np
import pytest

from oracle import enumerate as en

PARAMS = [(2, 0.4, 0.6), (3, 0.4, 0.6), (3, 0.9, 0.2), (3, 0.0, 0.7), (3, 0.7, 0.0), (3, 1.3, 2.1)]


@pytest.fixture(scope="module", params=PARAMS, ids=lambda p: "L%d-J%g-q%g" % p)
def ex(request):
    return en.Enumeration(*request.param)


def test_hamiltonian_two_forms_agree(ex):
    H2 = en.hamiltonian_matrix_second_form(ex.L, ex.J, ex.q)
    assert np.allclose(ex.H, H2, atol=1e-12, rtol=0)


def test_partition_function_product_form(ex):
    if ex.L == 3 and ex.J > 1.0:
        pytest.skip("product form only evaluated on the small parameter set")
    Zp = en.honeycomb_partition_function(ex.L, ex.J, ex.q)
    assert np.isclose(Zp, ex.Z, rtol=1e-11)


def test_half_step_kernels_are_stochastic(ex):
    assert np.allclose(ex.K_A.sum(1), 1, atol=1e-13)
    assert np.allclose(ex.K_B.sum(1), 1, atol=1e-13)


def test_shaken_marginal_stationary_and_reversible(ex):
    P, pi = ex.P_shaken, ex.pi_s
    assert np.allclose(pi @ P, pi, atol=1e-14, rtol=1e-11)
    F = pi[:, None] * P
    assert np.allclose(F, F.T, atol=1e-16, rtol=1e-10)
    ev = np.linalg.eigvals(P)
    assert np.max(np.abs(ev.imag)) < 1e-9
    assert ev.real.min() > -1e-9 and ev.real.max() < 1 + 1e-9


def test_pi_s_is_sigma_marginal_of_pi_2(ex):
    assert np.allclose(ex.pi_2.sum(axis=1), ex.pi_s, atol=1e-15, rtol=1e-12)


def test_Z_sigma_is_product_of_2cosh(ex):
    S = en.configurations(ex.L).astype(float)
    h = ex.J * (np.roll(S, 1, axis=-2) + np.roll(S, 1, axis=-1)) + ex.q * S
    prod = np.prod(2 * np.cosh(h).reshape(S.shape[0], -1), axis=1)
    assert np.allclose(prod, ex.Z_sigma, rtol=1e-12)


def test_pair_chain_stationary_not_reversible():
    ex = en.Enumeration(2, 0.4, 0.6)
    P = ex.pair_chain()
    pi2 = ex.pi_2.reshape(-1)
    assert np.allclose(pi2 @ P, pi2, atol=1e-15, rtol=1e-11)
    F = pi2[:, None] * P
    assert np.max(np.abs(F - F.T)) > 1e-4


def _oracle_matrix(oracle, ex, which):
    S = en.configurations(ex.L).astype(np.int8)
    T = np.stack([oracle.row_thresholds(s, ex.J, ex.q, which) for s in S])
    return en.implemented_half_step_matrix(T)


def test_oracle_half_steps_match_exact_kernels(oracle, ex):
    N = ex.L * ex.L
    bound = N * 2.0 ** -33 + 1e-13
    KA = _oracle_matrix(oracle, ex, 0)
    KB = _oracle_matrix(oracle, ex, 1)
    assert np.max(np.abs(KA - ex.K_A)) <= bound
    assert np.max(np.abs(KB - ex.K_B)) <= bound


def test_direction_bug_would_be_caught(oracle):
    # On 3x3 the exact A kernel (down/left field) differs from the mirrored
    # (up/right) one, so swapping the half-step stencils cannot pass the test above.
    ex = en.Enumeration(3, 0.4, 0.6)
    KB_as_A = _oracle_matrix(oracle, ex, 1)
    assert np.max(np.abs(KB_as_A - ex.K_A)) > 1e-3
