"""GPU parity of trajectories, log-likelihood counts, the FP32 forward and
backward kernels and the autograd wrapper, against the oracle's integer
counts and FP64 closed forms."""
import math

import numpy as np
import pytest
import torch

import paper_1908_07341_amd as sd
from paper_1908_07341_amd import autograd as AG
from paper_1908_07341_amd import inputs

pytestmark = pytest.mark.gpu

SEED = 4242


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.lib()


def _traj_gpu(L, J, q, n_traj, k, stream0=0):
    nb = sd.sd_lattice_bytes(L, sd.SD_P64)
    traj = torch.empty((n_traj, 2 * k + 1, nb // 8), dtype=torch.int64, device="cuda")
    for a in range(n_traj):
        s0 = sd.new_lattice(L, sd.SD_P64)
        sd.sd_init(s0, L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, SEED, stream0 + a)
        sd.sd_trajectory(s0, traj[a], L, sd.SD_P64, J, q, SEED, stream0 + a, 0, k)
    return traj


@pytest.mark.parametrize("L,n_traj,k", [(64, 3, 12), (64, 2, 130), (128, 2, 5), (192, 2, 71), (256, 1, 9),
                                        (320, 2, 4), (512, 1, 3), (576, 1, 2)])
def test_trajectory_and_counts_match_oracle(oracle, L, n_traj, k):
    # L <= 512 take the LDS-staged count kernel: one wave per lattice (64),
    # one word per lane (128), four words per lane with idle lanes (192, and
    # 320 on 1024 lanes) and without (256, and 512 on 1024 lanes); k = 130
    # spans two transition chunks with a ragged second one, k = 71 and 9 end
    # in a partial ring group.  L = 576 takes the generic kernel.
    J, q = 0.45, 0.7
    print(f"trajectories L={L} n={n_traj} k={k}", flush=True)
    traj = _traj_gpu(L, J, q, n_traj, k)
    torch.cuda.synchronize()
    host = traj.cpu().numpy()
    ref = []
    for a in range(n_traj):
        s0 = oracle.init(L, oracle.INIT_RANDOM, 0.5, SEED, a)
        X = oracle.trajectory(s0, J, q, SEED, a, 0, k)
        for m in range(2 * k + 1):
            assert np.array_equal(inputs.unpack_bits(host[a, m], L), X[m]), (a, m)
        ref.append(X)
    counts = AG.loglik_counts(traj, n_traj, 2 * k + 1, L)
    assert np.array_equal(counts.cpu().numpy(), oracle.loglik_counts(np.stack(ref)))
    stats = AG.loglik_stats(traj, n_traj, 2 * k + 1, L)
    assert np.array_equal(stats.cpu().numpy(), oracle.loglik_stats(np.stack(ref)))
    # a single lattice has no transitions
    one = AG.loglik_counts(traj[:1, :1].contiguous(), 1, 1, L)
    assert not one.any()
    one = AG.loglik_stats(traj[:1, :1].contiguous(), 1, 1, L)
    assert not one.any()


@pytest.mark.parametrize("L,layout,n_traj,k", [(64, sd.SD_P64, 5, 17), (256, sd.SD_P64, 3, 6),
                                               (512, sd.SD_P32, 2, 3), (96, sd.SD_P32, 2, 4)])
def test_trajectories_batched_match_single(oracle, L, layout, n_traj, k):
    # one launch for all trajectories (LDS-resident lattices when L % 64 == 0),
    # one sd_trajectory call per trajectory otherwise; both equal the
    # one-by-one recording, and trajectory 0 equals the oracle's
    J, q, stream0 = 0.6, 0.3, 7
    print(f"batched trajectories L={L} layout={layout} n={n_traj} k={k}", flush=True)
    nb = sd.sd_lattice_bytes(L, layout)
    starts = torch.empty((n_traj, nb), dtype=torch.uint8, device="cuda")
    for a in range(n_traj):
        sd.sd_init(starts[a], L, layout, sd.SD_INIT_RANDOM, 0.5, SEED, stream0 + a)
    got = torch.full((n_traj, 2 * k + 1, nb), 0x5A, dtype=torch.uint8, device="cuda")
    sd.sd_trajectories(starts, got, n_traj, L, layout, J, q, SEED, stream0, 3, k)
    ref = torch.empty_like(got)
    for a in range(n_traj):
        sd.sd_trajectory(starts[a], ref[a], L, layout, J, q, SEED, stream0 + a, 3, k)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    s0 = oracle.init(L, oracle.INIT_RANDOM, 0.5, SEED, stream0)
    X = oracle.trajectory(s0, J, q, SEED, stream0, 3, k)
    host = got[0].cpu().numpy()
    for m in range(2 * k + 1):
        assert np.array_equal(inputs.unpack_bits(host[m].view(np.uint64), L), X[m]), m


def _fp64(oracle, counts, J, q):
    return oracle.loglik(counts, J, q), oracle.loglik_grad(counts, J, q)


def _fd5(oracle, counts, J, q, eps=1e-3):
    def d(f):
        return (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * eps)
    gJ = d(lambda s: oracle.loglik(counts, J + s * eps, q))
    gq = d(lambda s: oracle.loglik(counts, J, q + s * eps))
    return np.array([gJ, gq])


@pytest.fixture(scope="module")
def c5_small():
    # the differentiation workload at reduced size: 16 trajectories of 128^2,
    # 300 steps, generated at (J, q) = (0.45, 0.7) from random starts
    L, J, q, n_traj, k = 128, 0.45, 0.7, 16, 300
    traj = _traj_gpu(L, J, q, n_traj, k, stream0=100)
    counts = AG.loglik_counts(traj, n_traj, 2 * k + 1, L)
    stats = AG.loglik_stats(traj, n_traj, 2 * k + 1, L)
    del traj
    return counts, stats


def test_paired_stats_are_the_pair_map_of_the_counts(c5_small):
    c, s = (t.cpu().numpy() for t in c5_small)
    S = [c[2 * j] + c[2 * j + 1] + c[2 * (5 - j)] + c[2 * (5 - j) + 1] for j in range(3)]
    Z = [c[2 * j + 1] + c[2 * (5 - j)] for j in range(3)]
    assert np.array_equal(s, np.array(S + Z))


def test_forward_and_backward_against_fp64(oracle, c5_small):
    c5_small, _ = c5_small
    ch = c5_small.cpu().numpy()
    N = int(ch.sum())
    for J, q in [(0.2, 0.2), (0.45, 0.7), (1.0, 1.5), (0.0, 0.0), (0.6, 0.3)]:
        J32, q32 = float(np.float32(J)), float(np.float32(q))
        Jq = torch.tensor([J32, q32], dtype=torch.float32, device="cuda")
        ll = torch.empty(1, dtype=torch.float32, device="cuda")
        grad = torch.empty(2, dtype=torch.float32, device="cuda")
        sd.sd_loglik_fwd(c5_small, Jq, ll)
        sd.sd_loglik_bwd(c5_small, Jq, None, grad)
        ll64, g64 = _fp64(oracle, ch, J32, q32)
        got_ll = float(ll.cpu()[0])
        got_g = grad.cpu().numpy().astype(np.float64)
        print(f"J={J} q={q} N={N} ll={got_ll} ll64={ll64} g={got_g} g64={g64}", flush=True)
        assert abs(got_ll - ll64) <= 1e-6 * abs(ll64)
        # plain relative tolerance on each component; at the MLE the gradient
        # is small, so also bound it by the scale of the summed terms
        scale = 2.0 * N
        for i in range(2):
            assert abs(got_g[i] - g64[i]) <= 1e-5 * abs(g64[i]) + 1e-9 * scale, (i, got_g[i], g64[i])
        fd = _fd5(oracle, ch, J32, q32)
        for i in range(2):
            assert abs(got_g[i] - fd[i]) <= 1e-5 * abs(fd[i]) + 1e-7 * scale, (i, got_g[i], fd[i])


def test_paired_forward_and_backward_against_fp64(oracle, c5_small):
    _, st = c5_small
    sh = st.cpu().numpy()
    scale = 2.0 * float(sh[:3].sum())
    for J, q in [(0.2, 0.2), (0.45, 0.7), (1.0, 1.5), (0.0, 0.0), (0.6, -0.3)]:
        J32, q32 = float(np.float32(J)), float(np.float32(q))
        Jq = torch.tensor([J32, q32], dtype=torch.float32, device="cuda")
        ll = torch.empty(1, dtype=torch.float32, device="cuda")
        grad = torch.empty(2, dtype=torch.float32, device="cuda")
        g_out = torch.tensor([-2.0], dtype=torch.float32, device="cuda")
        sd.sd_loglik_fwd_stats(st, Jq, ll)
        sd.sd_loglik_bwd_stats(st, Jq, g_out, grad)
        ll64, g64 = oracle.loglik_from_stats(sh, J32, q32)
        got_ll = float(ll.cpu()[0])
        got_g = grad.cpu().numpy().astype(np.float64) / -2.0
        print(f"paired J={J} q={q} ll={got_ll} ll64={ll64} g={got_g} g64={g64}", flush=True)
        assert abs(got_ll - ll64) <= 1e-6 * abs(ll64)
        for i in range(2):
            assert abs(got_g[i] - g64[i]) <= 1e-5 * abs(g64[i]) + 1e-9 * scale, (i, got_g[i], g64[i])


def test_autograd_function(oracle, c5_small):
    c5_small, st = c5_small
    Jq2 = torch.tensor([0.3, 0.5], dtype=torch.float32, device="cuda", requires_grad=True)
    (g2,) = torch.autograd.grad(3.0 * AG.loglik(Jq2, st), Jq2)
    _, g64s = oracle.loglik_from_stats(st.cpu().numpy(), float(np.float32(0.3)), float(np.float32(0.5)))
    assert np.allclose(g2.cpu().numpy(), 3.0 * g64s, rtol=1e-5)
    Jq = torch.tensor([0.3, 0.5], dtype=torch.float32, device="cuda", requires_grad=True)
    ll = AG.loglik(Jq, c5_small)
    (g,) = torch.autograd.grad(3.0 * ll, Jq)
    ch = c5_small.cpu().numpy()
    g64 = oracle.loglik_grad(ch, float(np.float32(0.3)), float(np.float32(0.5)))
    assert np.allclose(g.cpu().numpy(), 3.0 * g64, rtol=1e-5)


def test_gradient_ascent_recovers_parameters(oracle, c5_small):
    c5_small, _ = c5_small
    ch = c5_small.cpu().numpy()
    N = float(ch.sum())
    # plain gradient ascent on LL / N (a concave objective with curvature of
    # order one), the gradient coming from the hand-written backward kernel
    Jq = torch.tensor([0.2, 0.2], dtype=torch.float32, device="cuda", requires_grad=True)
    for it in range(400):
        (g,) = torch.autograd.grad(AG.loglik(Jq, c5_small) / N, Jq)
        with torch.no_grad():
            Jq += 0.5 * g
    est = Jq.detach().cpu().numpy().astype(np.float64)
    # standard errors from the FP64 Fisher information at the estimate
    H = np.zeros((2, 2))
    for k in range(3):
        for cp in range(2):
            a, b = 2 * k - 2, 2 * cp - 1
            h = est[0] * a + est[1] * b
            n = ch[2 * (2 * k + cp)] + ch[2 * (2 * k + cp) + 1]
            H -= n / math.cosh(h) ** 2 * np.array([[a * a, a * b], [a * b, b * b]])
    se = np.sqrt(np.diag(np.linalg.inv(-H)))
    print("estimate", est, "se", se, flush=True)
    assert abs(est[0] - 0.45) < 3 * se[0] and abs(est[1] - 0.7) < 3 * se[1]
