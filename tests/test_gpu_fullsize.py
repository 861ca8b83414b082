"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times, on outputs the oracle can compute one by one:

* the headline chain (16384^2 packed, J = q = 0.5, seed 1, stream 0) in the
  launch configuration the benchmark tunes: every site of sigma and tau after
  steps 0 and 1, and the two fused records, against the oracle;
* the 4096-chain (q, J) scan (L from {128, 256, 512}, 5000 steps, records
  every step): one chain of every size in full against the oracle, one chain
  of every size against its own sd_run, and for every chain the last record
  against a recount of the returned lattice pair;
* one point of the 1024^2 int8 sweep for its full 10^4 steps: records,
  D(r) and sampled sites of a further step against the oracle;
* the sweep's own path (the five chains through sd_run_many in calls of 100
  steps, their D(r) through sd_corr_row_many): one chain's lattices, records
  and D(r) over the first 200 steps against the oracle;
* the differentiation workload (256 trajectories of 256^2, 2000 steps):
  trajectory 0 lattice by lattice and its counts and paired statistics
  against the oracle; for the whole set, the site total, the pair map of
  the counts, the FP32 LL and gradient against FP64 from the counts, FP64
  finite differences, and the gradient ascent recovering (0.45, 0.7) within
  three Fisher-information standard errors."""
import os

import numpy as np
import pytest
import torch

import paper_1908_07341_amd as sd
from paper_1908_07341_amd import autograd as AG
from paper_1908_07341_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.lib()


def _unpack_many(raw: np.ndarray, L: int) -> np.ndarray:
    bits = np.unpackbits(np.ascontiguousarray(raw).view(np.uint8).reshape(raw.shape[0], -1), axis=1,
                         bitorder="little")[:, : L * L]
    return (2 * bits.astype(np.int8) - 1).reshape(-1, L, L)


def test_C3_full_lattice_matches_oracle(oracle):
    # the benchmark's chain and launch choice (its tune cache), two steps with
    # a record each, compared as packed bytes: all 2^28 sites of both lattices
    L, J, q, seed, stream = 16384, 0.5, 0.5, 1, 0
    cache = os.path.join(ROOT, "paper_1908_07341_amd", "tune_cache.json")
    sd.sd_tune(L, sd.SD_P64, cache)
    print(f"C3 full lattice, run choice {sd.sd_tuned_choice(L, sd.SD_P64)}", flush=True)
    sigma = sd.new_lattice(L, sd.SD_P64)
    tau = sd.new_lattice(L, sd.SD_P64)
    sd.sd_init(sigma, L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, seed, stream)
    ref_s = oracle.init(L, oracle.INIT_RANDOM, 0.5, seed, stream)

    def packed(t):
        torch.cuda.synchronize()
        return t.view(torch.uint8).view(-1).cpu().numpy()

    assert np.array_equal(packed(sigma), inputs.pack_bits(ref_s))
    for n in (0, 1):
        obs = torch.full((1, 3), -7, dtype=torch.int64, device="cuda")
        sd.sd_run(sigma, tau, L, sd.SD_P64, J, q, seed, stream, n, 1, obs, 1)
        print(f"C3 full lattice: oracle step {n}", flush=True)
        ref_s, ref_t, ref_o = oracle.run(ref_s, J, q, seed, stream, n, 1, obs_every=1)
        assert np.array_equal(packed(tau), inputs.pack_bits(ref_t)), f"tau after step {n}"
        assert np.array_equal(packed(sigma), inputs.pack_bits(ref_s)), f"sigma after step {n}"
        assert np.array_equal(obs.cpu().numpy(), ref_o), f"record of step {n}"
        del ref_t


def test_C4_full_scan_sampled(oracle, tmp_path):
    qv, Jv, Lv = inputs.scan_table()
    n, K = len(qv), 5000
    streams = np.arange(n, dtype=np.uint32)
    print("C4 plan", flush=True)
    plan = sd.sd_batch_plan_create(Jv, qv, Lv, streams, layout=sd.SD_P64, seed=1, k_steps=K, obs_every=1,
                                   tune_cache_path=str(tmp_path / "tune.json"))
    lat = torch.empty(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
    traces = torch.empty(sd.sd_batch_trace_len(plan), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan, lat, sd.SD_INIT_RANDOM, 0.5)
    start = lat.clone()
    print("C4 run", flush=True)
    sd.sd_batch_run(plan, lat, traces, 0)
    torch.cuda.synchronize()
    tr = traces.view(n, K, 3)

    def pair(c):
        Lc = int(Lv[c])
        nb = sd.sd_lattice_bytes(Lc, sd.SD_P64)
        so, to = sd.sd_batch_chain_offset(plan, c, 0), sd.sd_batch_chain_offset(plan, c, 1)
        return Lc, nb, so, to

    # every chain: the last record is (M, A, B) of the returned pair
    out = torch.empty((n, 3), dtype=torch.int64, device="cuda")
    for c in range(n):
        Lc, nb, so, to = pair(c)
        sd.sd_observe(lat[so:so + nb], lat[to:to + nb], Lc, sd.SD_P64, out[c])
    torch.cuda.synchronize()
    assert torch.equal(out, tr[:, K - 1, :])

    rng = np.random.default_rng(11)
    # one chain of every size against its own sd_run from the same start
    for size in (128, 256, 512):
        c = int(rng.choice(np.flatnonzero(Lv == size)))
        Lc, nb, so, to = pair(c)
        sig = start[so:so + nb].clone()
        tau = torch.empty_like(sig)
        obs = torch.empty((K, 3), dtype=torch.int64, device="cuda")
        print(f"C4 chain {c} L={Lc} against sd_run", flush=True)
        sd.sd_run(sig, tau, Lc, sd.SD_P64, float(Jv[c]), float(qv[c]), 1, c, 0, K, obs, 1)
        torch.cuda.synchronize()
        assert torch.equal(sig, lat[so:so + nb]) and torch.equal(tau, lat[to:to + nb]), c
        assert torch.equal(obs, tr[c]), c
    # one chain of every size (128^2, 256^2, 512^2) in full against the oracle:
    # both lattices after 5000 steps and all 5000 records
    for size in (128, 256, 512):
        c = int(rng.choice(np.flatnonzero(Lv == size)))
        Lc, nb, so, to = pair(c)
        print(f"C4 chain {c} L={Lc} against the oracle", flush=True)
        s0 = oracle.init(Lc, oracle.INIT_RANDOM, 0.5, 1, c)
        assert np.array_equal(inputs.unpack_bits(start[so:so + nb].cpu().numpy(), Lc), s0)
        rs, rt, ro = oracle.run(s0, float(Jv[c]), float(qv[c]), 1, c, 0, K, obs_every=1)
        assert np.array_equal(inputs.unpack_bits(lat[so:so + nb].cpu().numpy(), Lc), rs), c
        assert np.array_equal(inputs.unpack_bits(lat[to:to + nb].cpu().numpy(), Lc), rt), c
        assert np.array_equal(tr[c].cpu().numpy(), ro), c
    plan.close()


def test_C5_full_loglik_sampled(oracle):
    n_traj, L, k, J, q = 256, 256, 2000, 0.45, 0.7
    nb = sd.sd_lattice_bytes(L, sd.SD_P64)
    n_lat = 2 * k + 1
    print("C5 trajectories", flush=True)
    starts = torch.empty((n_traj, nb // 8), dtype=torch.int64, device="cuda")
    for a in range(n_traj):
        sd.sd_init(starts[a], L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, 1, a)
    traj = torch.empty((n_traj, n_lat, nb // 8), dtype=torch.int64, device="cuda")
    sd.sd_trajectories(starts, traj, n_traj, L, sd.SD_P64, J, q, 1, 0, 0, k)
    counts = AG.loglik_counts(traj, n_traj, n_lat, L)
    stats = AG.loglik_stats(traj, n_traj, n_lat, L)
    c0 = AG.loglik_counts(traj[:1], 1, n_lat, L)
    s0_ = AG.loglik_stats(traj[:1], 1, n_lat, L)
    torch.cuda.synchronize()
    # trajectory 0 lattice by lattice
    print("C5 trajectory 0 against the oracle", flush=True)
    X = oracle.trajectory(oracle.init(L, oracle.INIT_RANDOM, 0.5, 1, 0), J, q, 1, 0, 0, k)
    assert np.array_equal(_unpack_many(traj[0].cpu().numpy(), L), X)
    assert np.array_equal(c0.cpu().numpy(), oracle.loglik_counts(X[None]))
    assert np.array_equal(s0_.cpu().numpy(), oracle.loglik_stats(X[None]))
    del X
    # the whole set
    ch, sh = counts.cpu().numpy(), stats.cpu().numpy()
    assert ch.sum() == n_traj * 2 * k * L * L
    S = [ch[2 * j] + ch[2 * j + 1] + ch[2 * (5 - j)] + ch[2 * (5 - j) + 1] for j in range(3)]
    Z = [ch[2 * j + 1] + ch[2 * (5 - j)] for j in range(3)]
    assert np.array_equal(sh, np.array(S + Z))
    for Jp, qp in ((0.2, 0.2), (0.45, 0.7)):
        Jt = torch.tensor([Jp, qp], dtype=torch.float32, device="cuda", requires_grad=True)
        J32, q32 = (float(x) for x in Jt.detach().cpu().numpy())
        for vec in (counts, stats):
            ll = AG.loglik(Jt, vec)
            (g,) = torch.autograd.grad(ll, Jt)
            ll64, g64 = oracle.loglik(ch, J32, q32), oracle.loglik_grad(ch, J32, q32)
            assert abs(float(ll.detach()) - ll64) <= 1e-6 * abs(ll64)
            scale = 2.0 * float(ch.sum())
            gg = g.cpu().numpy().astype(np.float64)
            for i in range(2):
                assert abs(gg[i] - g64[i]) <= 1e-5 * abs(g64[i]) + 1e-9 * scale, (Jp, qp, i, gg[i], g64[i])
    # FP64 finite differences of the LL of the full counts (5-point stencil,
    # step 1e-4) against the FP64 analytic gradient, at the ascent start and
    # at the generating point
    eps = 1e-4
    for Jp, qp in ((0.2, 0.2), (0.45, 0.7)):
        g64 = oracle.loglik_grad(ch, Jp, qp)

        def fd(dJ, dq):
            f = [oracle.loglik(ch, Jp + m * dJ, qp + m * dq) for m in (-2, -1, 1, 2)]
            return (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / 12.0

        scale = 2.0 * float(ch.sum())
        assert abs(fd(eps, 0) / eps - g64[0]) <= 1e-7 * scale, (Jp, qp)
        assert abs(fd(0, eps) / eps - g64[1]) <= 1e-7 * scale, (Jp, qp)
    # the generating (J, q) recovered within three standard errors: FP32
    # gradient ascent on LL / N through the backward kernel, against the FP64
    # Newton maximum of the same counts and its Fisher-information errors
    N = float(ch.sum())
    x = torch.tensor([0.2, 0.2], dtype=torch.float32, device="cuda", requires_grad=True)
    for _ in range(300):
        (gg,) = torch.autograd.grad(AG.loglik(x, stats) / N, x)
        with torch.no_grad():
            x += 0.5 * gg
    est = x.detach().cpu().numpy().astype(np.float64)
    mle, se = _newton_mle(oracle, ch)
    print(f"C5 ascent {est}, FP64 MLE {mle}, standard errors {se}", flush=True)
    assert np.all(np.abs(mle - np.array([J, q])) < 3 * se), (mle, se)
    assert np.all(np.abs(est - np.array([J, q])) < 3 * se), (est, se)
    assert np.all(np.abs(est - mle) < 0.5 * se), (est, mle, se)


def _hessian(c, J, q):
    """FP64 Hessian of the LL of the 12 counts: -sum n sech^2 h (a, b)(a, b)^T
    with a = 2k - 2, b = 2c - 1 the coefficients of J and q in h."""
    H = np.zeros((2, 2))
    for k in range(3):
        for cp in range(2):
            a, b = 2 * k - 2, 2 * cp - 1
            h = J * a + q * b
            n = float(c[2 * (2 * k + cp)] + c[2 * (2 * k + cp) + 1])
            H -= n / np.cosh(h) ** 2 * np.array([[a * a, a * b], [a * b, b * b]])
    return H


def _newton_mle(oracle, c):
    theta = np.array([0.2, 0.2])
    for _ in range(30):
        theta = theta - np.linalg.solve(_hessian(c, *theta), oracle.loglik_grad(c, *theta))
    return theta, np.sqrt(np.diag(np.linalg.inv(-_hessian(c, *theta))))


def test_C2_full_length_point(oracle):
    # 1024^2 int8 from a random start at J = q = 0.6 (the middle of the sweep,
    # stream 2), 10^4 steps with (M, A, B) every step and D(r <= 512) every 100
    # steps: D(0) = L^2 at every measurement, the final D(r) against the
    # oracle's sum over the returned lattice, the last record against a recount
    # of the returned pair, and one more step's sampled sites against the
    # oracle's thresholds and uniforms
    L, J, q, stream = 1024, 0.6, 0.6, 2
    sigma = sd.new_lattice(L, sd.SD_I8)
    tau = sd.new_lattice(L, sd.SD_I8)
    sd.sd_init(sigma, L, sd.SD_I8, sd.SD_INIT_RANDOM, 0.5, 1, stream)
    obs = torch.empty((10000, 3), dtype=torch.int64, device="cuda")
    D = torch.empty((100, 513), dtype=torch.int64, device="cuda")
    print("C2 full-length run", flush=True)
    for blk in range(100):
        sd.sd_run(sigma, tau, L, sd.SD_I8, J, q, 1, stream, 100 * blk, 100, obs[100 * blk:100 * (blk + 1)], 1)
        sd.sd_corr_row(sigma, L, sd.SD_I8, 512, D[blk])
    torch.cuda.synchronize()
    assert bool((D[:, 0] == L * L).all())
    s_fin = to_host_i8(sigma, L)
    assert np.array_equal(D[-1].cpu().numpy(), oracle.corr_row(s_fin, 512))
    out3 = torch.empty(3, dtype=torch.int64, device="cuda")
    sd.sd_observe(sigma, tau, L, sd.SD_I8, out3)
    assert torch.equal(out3, obs[-1])
    sd.sd_run(sigma, tau, L, sd.SD_I8, J, q, 1, stream, 10000, 1, None, 0)
    t_new, s_new = to_host_i8(tau, L), to_host_i8(sigma, L)
    rng = np.random.default_rng(2)
    for j in [0, L - 1] + [int(x) for x in rng.integers(0, L, 6)]:
        rowA = oracle.row_thresholds_of(s_fin, J, q, 0, j)
        rowB = oracle.row_thresholds_of(t_new, J, q, 1, j)
        for i in [0, L - 1] + [int(x) for x in rng.integers(0, L, 40)]:
            s = j * L + i
            assert t_new[j, i] == (1 if oracle.site_uniform(1, stream, 20000, 0, s) < rowA[i] else -1), (j, i)
            assert s_new[j, i] == (1 if oracle.site_uniform(1, stream, 20001, 0, s) < rowB[i] else -1), (j, i)


def to_host_i8(t: torch.Tensor, L: int) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.int8).reshape(L, L)


def test_C2_sweep_path_against_oracle(oracle):
    # the five 1024^2 int8 chains of the sweep (q = J in {0.2, ..., 1.0},
    # stream = point index) as the benchmark runs them: sd_run_many calls of
    # 100 steps with (M, A, B) every step, then D(r <= 512) of all five in one
    # sd_corr_row_many call; chain 4 (J = q = 1) over 200 steps against the
    # oracle (the middle point's full length is checked above)
    L, per_call, n_calls, rmax = 1024, 100, 2, 512
    points = [0.2, 0.4, 0.6, 0.8, 1.0]
    sigmas = [sd.new_lattice(L, sd.SD_I8) for _ in points]
    taus = [sd.new_lattice(L, sd.SD_I8) for _ in points]
    for a, sigma in enumerate(sigmas):
        sd.sd_init(sigma, L, sd.SD_I8, sd.SD_INIT_RANDOM, 0.5, 1, a)
    obs = torch.empty((n_calls, len(points), per_call, 3), dtype=torch.int64, device="cuda")
    D = torch.empty((n_calls, len(points), rmax + 1), dtype=torch.int64, device="cuda")
    for c in range(n_calls):
        print(f"C2 sweep path call {c}", flush=True)
        sd.sd_run_many(sigmas, taus, L, sd.SD_I8, points, points, 1, list(range(len(points))), per_call * c,
                       per_call, obs[c], 1)
        sd.sd_corr_row_many(sigmas, L, sd.SD_I8, rmax, D[c])
    torch.cuda.synchronize()
    for a in (4,):
        print(f"C2 sweep path chain {a} against the oracle", flush=True)
        s = oracle.init(L, oracle.INIT_RANDOM, 0.5, 1, a)
        for c in range(n_calls):
            s, t, o = oracle.run(s, points[a], points[a], 1, a, per_call * c, per_call, obs_every=1)
            assert np.array_equal(obs[c, a].cpu().numpy(), o), (a, c)
            assert np.array_equal(D[c, a].cpu().numpy(), oracle.corr_row(s, rmax)), (a, c)
        assert np.array_equal(sigmas[a].cpu().numpy().reshape(L, L), s), a
        assert np.array_equal(taus[a].cpu().numpy().reshape(L, L), t), a
