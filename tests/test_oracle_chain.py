"""Pathwise pins of the oracle chain: exact identities that any correct
implementation of the two half-steps must satisfy draw by draw."""
import numpy as np
import pytest

SEED = 0x5EED


def _planes0(oracle, seed, stream, t, n_sites):
    """Bit 31 of every r_s(t): bit b of the plane-0 word of group g."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    out = np.zeros(n_sites, dtype=np.int64)
    for g in range((n_sites + 63) // 64):
        x = oracle.philox4x32_10([stream, t, 0, g], key)
        word = int(x[0]) | (int(x[1]) << 32)
        for b in range(64):
            s = 64 * g + b
            if s < n_sites:
                out[s] = (word >> b) & 1
    return out


@pytest.mark.parametrize("L", [3, 8, 64])
def test_J_q_zero_is_complemented_msb_plane(oracle, L):
    # With J = q = 0 every threshold is 2^31: a new spin is +1 exactly when the
    # top bit of its uniform is 0, whatever the source lattice.
    rng = np.random.default_rng(L)
    src = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L))
    for which, t in ((0, 6), (1, 7)):
        dst = oracle.half_step(src, 0.0, 0.0, which, SEED, 5, t)
        msb = _planes0(oracle, SEED, 5, t, L * L).reshape(L, L)
        assert np.array_equal(dst, np.where(msb == 0, 1, -1).astype(np.int8))


def test_J_zero_sites_decouple(oracle):
    # With J = 0 the new spin at x depends only on the old spin at x and r_x.
    L = 16
    rng = np.random.default_rng(3)
    src = rng.choice(np.array([-1, 1], dtype=np.int8), size=(L, L))
    for which in (0, 1):
        up = oracle.half_step(np.ones((L, L), np.int8), 0.0, 0.8, which, SEED, 2, 11)
        dn = oracle.half_step(-np.ones((L, L), np.int8), 0.0, 0.8, which, SEED, 2, 11)
        mixed = oracle.half_step(src, 0.0, 0.8, which, SEED, 2, 11)
        assert np.array_equal(mixed, np.where(src > 0, up, dn))


def test_monotone_coupling(oracle):
    # Sandwiching (section 3.2): with J, q >= 0 and shared randomness the
    # partial order between configurations survives every half-step.
    L, J, q = 16, 0.55, 0.4
    top = np.ones((L, L), np.int8)
    bot = -np.ones((L, L), np.int8)
    mid = oracle.init(L, 2, 0.5, 9, 9)
    for n in range(150):
        for which, t in ((0, 2 * n), (1, 2 * n + 1)):
            top, mid, bot = (oracle.half_step(x, J, q, which, SEED, 4, t) for x in (top, mid, bot))
            assert np.all(top >= mid) and np.all(mid >= bot)


def test_global_spin_flip_with_complemented_randoms(oracle):
    # T(-h) = 2^32 - T(h): flipping every spin and replacing r by 2^32-1-r
    # flips every later spin exactly.
    L, J, q = 12, 0.5, 0.3
    s0 = oracle.init(L, 2, 0.5, 1, 1)
    a, b = s0.copy(), (-s0).astype(np.int8)
    for n in range(40):
        for which, t in ((0, 2 * n), (1, 2 * n + 1)):
            a = oracle.half_step(a, J, q, which, SEED, 8, t)
            with oracle.complement_randoms():
                b = oracle.half_step(b, J, q, which, SEED, 8, t)
            assert np.array_equal(a, -b)


def test_resume_identity(oracle):
    L, J, q = 24, 0.4, 0.6
    s0 = oracle.init(L, 2, 0.5, 2, 3)
    s_all, t_all, o_all = oracle.run(s0, J, q, SEED, 3, 0, 30, obs_every=1)
    s1, t1, o1 = oracle.run(s0, J, q, SEED, 3, 0, 12, obs_every=1)
    s2, t2, o2 = oracle.run(s1, J, q, SEED, 3, 12, 18, obs_every=1)
    assert np.array_equal(s_all, s2) and np.array_equal(t_all, t2)
    assert np.array_equal(o_all, np.concatenate([o1, o2]))


def test_run_equals_half_step_sequence(oracle):
    L, J, q = 10, 0.7, 0.9
    s = oracle.init(L, 0)
    ref_s, ref_t, obs = oracle.run(s, J, q, SEED, 6, 4, 5, obs_every=1)
    x = s
    for n in range(4, 9):
        tau = oracle.half_step(x, J, q, 0, SEED, 6, 2 * n)
        x = oracle.half_step(tau, J, q, 1, SEED, 6, 2 * n + 1)
        assert np.array_equal(obs[n - 4], oracle.observe(x, tau))
    assert np.array_equal(x, ref_s) and np.array_equal(tau, ref_t)


def test_observables_brute_force(oracle):
    # A from the second form of the pair Hamiltonian: sum_x tau_x (sigma_down + sigma_left).
    rng = np.random.default_rng(11)
    for L in (2, 3, 7, 16):
        s = rng.choice(np.array([-1, 1], np.int8), size=(L, L))
        t = rng.choice(np.array([-1, 1], np.int8), size=(L, L))
        S, T = s.astype(np.int64), t.astype(np.int64)
        M = S.sum()
        A = (T * (np.roll(S, 1, axis=0) + np.roll(S, 1, axis=1))).sum()
        B = (S * T).sum()
        assert list(oracle.observe(s, t)) == [M, A, B]


def test_row_correlation_brute_force(oracle):
    rng = np.random.default_rng(12)
    for L in (2, 5, 16):
        s = rng.choice(np.array([-1, 1], np.int8), size=(L, L))
        D = oracle.corr_row(s, L - 1)
        S = s.astype(np.int64)
        for r in range(L):
            assert D[r] == (S * np.roll(S, -r, axis=1)).sum()
        assert D[0] == L * L
        assert all(D[r] == D[L - r] for r in range(1, L))
    with pytest.raises(ValueError):
        oracle.corr_row(s, L)


def test_diagonal_correlation_brute_force(oracle):
    # section 3.3 / Table 1: SW-NE pairs x, x + (l, l); NW-SE pairs x, x + (l, -l)
    # (i = column = axis 1, j = row = axis 0 of the array)
    rng = np.random.default_rng(13)
    for L in (2, 3, 7, 16):
        s = rng.choice(np.array([-1, 1], np.int8), size=(L, L))
        D = oracle.corr_diag(s, L - 1)
        S = s.astype(np.int64)
        for l in range(L):
            assert D[0, l] == (S * np.roll(S, (-l, -l), axis=(0, 1))).sum()
            assert D[1, l] == (S * np.roll(S, (l, -l), axis=(0, 1))).sum()
        assert D[0, 0] == D[1, 0] == L * L
        assert all(D[d, l] == D[d, L - l] for d in range(2) for l in range(1, L))
    # a lattice constant along the NW-SE diagonals (a function of i + j) has
    # NW-SE sums L^2 at every l; along SW-NE the same lattice decorrelates
    L = 6
    i, j = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
    s = np.where((i + j) % 3 == 0, 1, -1).astype(np.int8)
    D = oracle.corr_diag(s, L - 1)
    assert np.all(D[1] == L * L)
    assert D[0, 1] == (s.astype(np.int64) * np.roll(s, (-1, -1), axis=(0, 1))).sum() < L * L
    with pytest.raises(ValueError):
        oracle.corr_diag(s, L)


def test_init_kinds(oracle):
    L = 64
    assert np.all(oracle.init(L, 0) == 1)
    assert np.all(oracle.init(L, 1) == -1)
    assert np.all(oracle.init(L, 2, 0.0) == -1)
    assert np.all(oracle.init(L, 2, 1.0) == 1)
    frac = (oracle.init(L, 2, 0.3, 5, 1) == 1).mean()
    assert abs(frac - 0.3) < 5 * np.sqrt(0.3 * 0.7 / (L * L))
    a, b = oracle.init(L, 2, 0.5, 5, 1), oracle.init(L, 2, 0.5, 5, 2)
    assert not np.array_equal(a, b)


def _q_with_threshold(oracle, target):
    """A field value h > 0 whose threshold is exactly `target` (> 2^31), by
    bisection on the monotone threshold function."""
    lo, hi = 0.0, 12.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        T = oracle.threshold(mid)
        if T == target:
            return mid
        if T < target:
            lo = mid
        else:
            hi = mid
    return None


def test_strict_comparison_at_exact_tie(oracle):
    # Algorithm 3 draws +1 only when the uniform is strictly below p: a site
    # whose uniform equals its threshold exactly must come out -1.
    L, t, stream = 8, 4, 3
    s = next(s for s in range(L * L) if oracle.site_uniform(SEED, stream, t, 0, s) > 2 ** 31 + 2 ** 20)
    r = oracle.site_uniform(SEED, stream, t, 0, s)
    q = _q_with_threshold(oracle, r)
    assert q is not None and oracle.threshold(q) == r
    src = np.ones((L, L), np.int8)               # J = 0: field q at every site
    dst = oracle.half_step(src, 0.0, q, 0, SEED, stream, t)
    assert dst.reshape(-1)[s] == -1
    # one step above the tie it flips to +1
    q_up = _q_with_threshold(oracle, r + 1)
    if q_up is not None:
        assert oracle.half_step(src, 0.0, q_up, 0, SEED, stream, t).reshape(-1)[s] == 1
