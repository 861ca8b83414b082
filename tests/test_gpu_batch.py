"""GPU parity of the batched persistent scan and of the single-workgroup LDS
path of sd_run: every chain bit-identical to the oracle and to sd_run."""
import numpy as np
import pytest
import torch

import paper_1908_07341_amd as sd
from paper_1908_07341_amd import inputs

pytestmark = pytest.mark.gpu

SEED = 77


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.lib()
    p = torch.cuda.get_device_properties(0)
    print(f"device {p.name} CUs={p.multi_processor_count}", flush=True)


def _unpack(buf, off, L, layout):
    n = sd.sd_lattice_bytes(L, layout)
    raw = buf[off:off + n].cpu().numpy()
    if layout == sd.SD_I8:
        return raw.view(np.int8).reshape(L, L)
    return inputs.unpack_bits(raw, L)


def _chains(n, sizes, seed=3):
    rng = np.random.default_rng(seed)
    J = rng.uniform(0.0, 1.5, n)
    q = rng.uniform(0.0, 2.0, n)
    # two chains whose tables contain 2^31 exactly (h = 0 for some class):
    # they take the general threshold form inside the batched kernel
    J[0], q[0] = 0.25, 0.5
    J[1], q[1] = 0.0, 0.0
    L = rng.choice(np.asarray(sizes), n)
    streams = rng.permutation(1000)[:n]
    return J, q, L, streams


@pytest.mark.parametrize("sizes", [[64, 128, 192], [8, 40, 72, 200]])
@pytest.mark.parametrize("layout", [sd.SD_P64, sd.SD_I8])
def test_batch_matches_oracle(oracle, layout, sizes):
    # the second set of sizes has rows off 64-bit word boundaries (bit-string
    # neighbours in the batched kernel)
    J, q, L, st = _chains(12, sizes)
    k, every = 30, 3
    plan = sd.sd_batch_plan_create(J, q, L, st, layout=layout, seed=SEED, k_steps=k, obs_every=every)
    lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
    tr = torch.full((sd.sd_batch_trace_len(plan),), -5, dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan, lat, sd.SD_INIT_RANDOM, 0.5)
    print("batch run", layout, flush=True)
    sd.sd_batch_run(plan, lat, tr, 5)
    torch.cuda.synchronize()
    trh = tr.cpu().numpy().reshape(len(J), k // every, 3)
    for c in range(len(J)):
        s0 = oracle.init(int(L[c]), oracle.INIT_RANDOM, 0.5, SEED, int(st[c]))
        rs, rt, ro = oracle.run(s0, J[c], q[c], SEED, int(st[c]), 5, k, obs_every=every)
        assert np.array_equal(_unpack(lat, sd.sd_batch_chain_offset(plan, c, 0), int(L[c]), layout), rs), c
        assert np.array_equal(_unpack(lat, sd.sd_batch_chain_offset(plan, c, 1), int(L[c]), layout), rt), c
        assert np.array_equal(trh[c], ro), c
    plan.close()


def test_batch_general_compare_flag_identical():
    # scan-like (J, q) including rows with h = 0 classes (J = 0, q = 0, q = 2J)
    J = np.array([0.0, 0.3, 0.5, 0.7, 0.0, 0.45, 1.2, 0.25])
    q = np.array([0.0, 0.0, 1.0, 0.4, 0.9, 0.9, 0.3, 0.5])
    L = np.array([64, 128, 40, 200, 72, 64, 8, 128])
    st = np.arange(8) + 70
    res = []
    for flags in (0, sd.SD_FLAG_GENERAL_COMPARE):
        plan = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=20, obs_every=2, flags=flags)
        lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
        tr = torch.zeros(sd.sd_batch_trace_len(plan), dtype=torch.int64, device="cuda")
        sd.sd_batch_init(plan, lat, sd.SD_INIT_RANDOM, 0.5)
        sd.sd_batch_run(plan, lat, tr, 0)
        torch.cuda.synchronize()
        res.append(([_unpack(lat, sd.sd_batch_chain_offset(plan, c, w), int(L[c]), sd.SD_P64)
                     for c in range(len(J)) for w in (0, 1)], tr.cpu().numpy()))
        plan.close()
    assert all(np.array_equal(a, b) for a, b in zip(res[0][0], res[1][0]))
    assert np.array_equal(res[0][1], res[1][1])


def test_batch_equals_plain_runs_and_graph_reuse():
    J, q, L, st = _chains(40, [128, 256, 512], seed=9)
    k = 25
    plan = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=k, obs_every=1)
    for b in range(3):
        print("bucket", b, sd.sd_batch_launch_shape(plan, b), flush=True)
    lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
    tr = torch.zeros(sd.sd_batch_trace_len(plan), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan, lat, sd.SD_INIT_RANDOM, 0.5)
    plain = lat.clone()
    plain_tr = torch.zeros_like(tr).view(len(J), k, 3)
    # two graph launches with different step0, then the same again (graph reuse)
    sd.sd_batch_run(plan, lat, tr, 0)
    tr0 = tr.clone()
    sd.sd_batch_run(plan, lat, tr, k)
    tr1 = tr.clone()
    torch.cuda.synchronize()
    for c in range(len(J)):
        Lc = int(L[c])
        nb = sd.sd_lattice_bytes(Lc, sd.SD_P64)
        so, to = sd.sd_batch_chain_offset(plan, c, 0), sd.sd_batch_chain_offset(plan, c, 1)
        sig = plain[so:so + nb].view(torch.int64)
        tau = plain[to:to + nb].view(torch.int64)
        obs_a = torch.zeros((k, 3), dtype=torch.int64, device="cuda")
        obs_b = torch.zeros((k, 3), dtype=torch.int64, device="cuda")
        sd.sd_run(sig, tau, Lc, sd.SD_P64, J[c], q[c], SEED, int(st[c]), 0, k, obs_a, 1)
        sd.sd_run(sig, tau, Lc, sd.SD_P64, J[c], q[c], SEED, int(st[c]), k, k, obs_b, 1)
        assert torch.equal(obs_a, tr0.view(len(J), k, 3)[c]), c
        assert torch.equal(obs_b, tr1.view(len(J), k, 3)[c]), c
    torch.cuda.synchronize()
    assert torch.equal(plain, lat)
    # direct (non-graph) enqueue gives the same
    lat2 = lat.clone()
    sd.sd_batch_run_direct(plan, lat2, tr, 2 * k)
    sd.sd_batch_run(plan, lat, tr1, 2 * k)
    torch.cuda.synchronize()
    assert torch.equal(lat2, lat) and torch.equal(tr, tr1)
    plan.close()


def test_batch_autotune_cache(tmp_path):
    J, q, L, st = _chains(64, [128, 256], seed=4)
    path = str(tmp_path / "tune.json")
    plan = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=4, obs_every=1, tune_cache_path=path)
    shapes = [sd.sd_batch_launch_shape(plan, b) for b in range(2)]
    print("tuned", shapes, open(path).read(), flush=True)
    plan.close()
    plan2 = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=4, obs_every=1, tune_cache_path=path)
    assert [sd.sd_batch_launch_shape(plan2, b) for b in range(2)] == shapes
    plan2.close()


def test_bucket_times_of_graph_and_direct_runs():
    # each bucket's launch stamps its first start and last end on the device:
    # the earliest start is 0, every end follows its start, and both kinds of
    # run leave times (the graph run first)
    J, q, L, st = _chains(48, [64, 128, 256], seed=6)
    plan = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=20, obs_every=1)
    lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
    tr = torch.zeros(sd.sd_batch_trace_len(plan), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan, lat, sd.SD_INIT_RANDOM, 0.5)
    with pytest.raises(sd.ShakenError):   # no run yet
        sd.sd_batch_bucket_times(plan, 0)
    n_buckets = 0
    while True:
        try:
            sd.sd_batch_launch_shape(plan, n_buckets)
        except sd.ShakenError:
            break
        n_buckets += 1
    for run in (sd.sd_batch_run, sd.sd_batch_run_direct):
        run(plan, lat, tr, 0)
        times = [sd.sd_batch_bucket_times(plan, b) for b in range(n_buckets)]
        print(run.__name__, times, flush=True)
        assert min(s_ for s_, _ in times) == 0.0
        assert all(0.0 <= s_ <= e for s_, e in times)
    with pytest.raises(sd.ShakenError):
        sd.sd_batch_bucket_times(plan, n_buckets)
    plan.close()


@pytest.mark.parametrize("threads", [64, 640, 128])
def test_batch_forced_block_sizes_agree(tmp_path, threads):
    # the same plan with its block size pinned through the tuner's cache:
    # lattices and records identical whatever the block size (640, the
    # paired kernel's largest workgroup, has ten wavefronts adding records)
    import json
    J, q, L, st = _chains(24, [64, 128, 256], seed=9)
    k, every = 12, 1
    path = str(tmp_path / "tune.json")

    def run(plan):
        lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
        tr = torch.full((sd.sd_batch_trace_len(plan),), -5, dtype=torch.int64, device="cuda")
        sd.sd_batch_init(plan, lat, sd.SD_INIT_RANDOM, 0.5)
        sd.sd_batch_run(plan, lat, tr, 3)
        torch.cuda.synchronize()
        return lat, tr

    plan = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=k, obs_every=every, tune_cache_path=path)
    lat0, tr0 = run(plan)
    plan.close()
    with open(path) as f:
        cache = json.load(f)
    forced = {key: (min(threads, 640 if ":p=1" in key else 512) if key.startswith("batch:") else v)
              for key, v in cache.items()}
    with open(path, "w") as f:
        json.dump(forced, f)
    plan = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=k, obs_every=every, tune_cache_path=path)
    shapes = []
    for b in range(8):
        try:
            shapes.append(sd.sd_batch_launch_shape(plan, b))
        except sd.ShakenError:
            break
    print("forced", threads, shapes, flush=True)
    # a cached size is taken up to 64 threads per 64-word tile of the lattice
    # (above that the plan tunes again within that bound)
    for Lb, _, thr, _ in shapes:
        cap = max(64, 64 * ((Lb * Lb // 64 + 63) // 64))
        assert thr == min(threads, 640) if min(threads, 640) <= cap else thr <= cap, (Lb, thr)
    lat1, tr1 = run(plan)
    plan.close()
    assert torch.equal(lat1, lat0) and torch.equal(tr1, tr0)


@pytest.mark.parametrize("L", [40, 64, 128, 200, 256])
def test_lds_and_global_paths_agree(L):
    J, q, k = 0.55, 0.45, 60
    s0 = inputs.random_lattice(L, L)
    outs = []
    for flags in (0, sd.SD_FLAG_GLOBAL_KERNELS):
        for layout in (sd.SD_P64, sd.SD_I8):
            sig = sd.new_lattice(L, layout)
            if layout == sd.SD_I8:
                sig.copy_(torch.from_numpy(s0))
            else:
                sig.view(torch.uint8).view(-1).copy_(torch.from_numpy(inputs.pack_bits(s0)))
            tau = sd.new_lattice(L, layout)
            obs = torch.zeros((k, 3), dtype=torch.int64, device="cuda")
            sd.sd_run(sig, tau, L, layout, J, q, SEED, 3, 11, k, obs, 1, flags)
            torch.cuda.synchronize()
            if layout == sd.SD_I8:
                got = (sig.cpu().numpy(), tau.cpu().numpy())
            else:
                got = (inputs.unpack_bits(sig.cpu().numpy(), L), inputs.unpack_bits(tau.cpu().numpy(), L))
            outs.append((got[0], got[1], obs.cpu().numpy()))
    for o in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(outs[0], o))


@pytest.mark.parametrize("L,layout", [(128, sd.SD_P64), (256, sd.SD_I8), (1024, sd.SD_P64), (96, sd.SD_P32)])
def test_sd_tune_keeps_results_and_caches(tmp_path, L, layout):
    path = str(tmp_path / "run_tune.json")
    J, q, k = 0.6, 0.4, 12
    s0 = inputs.random_lattice(L, 7 * L)

    def run():
        sig = sd.new_lattice(L, layout)
        if layout == sd.SD_I8:
            sig.copy_(torch.from_numpy(s0))
        else:
            sig.view(torch.uint8).view(-1).copy_(torch.from_numpy(inputs.pack_bits(s0)))
        tau = sd.new_lattice(L, layout)
        obs = torch.zeros((k, 3), dtype=torch.int64, device="cuda")
        sd.sd_run(sig, tau, L, layout, J, q, SEED, 1, 0, k, obs, 1)
        torch.cuda.synchronize()
        return sig.cpu().numpy().tobytes(), tau.cpu().numpy().tobytes(), obs.cpu().numpy()

    before = run()
    sd.sd_tune(L, layout, path)
    choice = sd.sd_tuned_choice(L, layout)
    print("tuned", L, layout, choice, flush=True)
    assert choice[0] in (1, 2)
    after = run()
    assert before[0] == after[0] and before[1] == after[1] and np.array_equal(before[2], after[2])
    text = open(path).read()
    assert f"L={L}:layout={layout}" in text
    sd.sd_tune(L, layout, path)          # from the cache
    assert sd.sd_tuned_choice(L, layout) == choice


def test_batch_moments_equal_sums_of_traces():
    # SD_FLAG_MOMENTS keeps, per chain, sum M, sum M^2, sum |M|, sum A, sum B
    # over the recorded steps: exactly the sums of the records of a trace plan
    J, q, L, st = _chains(10, [40, 64, 200], seed=21)
    k, every = 40, 2
    plans = {}
    for flags in (0, sd.SD_FLAG_MOMENTS):
        plan = sd.sd_batch_plan_create(J, q, L, st, seed=SEED, k_steps=k, obs_every=every, flags=flags)
        lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
        tr = torch.full((sd.sd_batch_trace_len(plan),), -3, dtype=torch.int64, device="cuda")
        sd.sd_batch_init(plan, lat, sd.SD_INIT_DOWN)
        sd.sd_batch_run(plan, lat, tr, 11)
        torch.cuda.synchronize()
        plans[flags] = (lat.cpu(), tr.cpu().numpy())
        plan.close()
    assert torch.equal(plans[0][0], plans[sd.SD_FLAG_MOMENTS][0])
    rec = plans[0][1].reshape(len(J), k // every, 3).astype(np.int64)
    M, A, B = rec[..., 0], rec[..., 1], rec[..., 2]
    want = np.stack([M.sum(1), (M * M).sum(1), np.abs(M).sum(1), A.sum(1), B.sum(1)], axis=1)
    assert np.array_equal(plans[sd.SD_FLAG_MOMENTS][1].reshape(len(J), 5), want)


def test_critical_scan_moments_small(oracle):
    # the section 3.1 pipeline at small scale, against the oracle: from all -1
    # on a 64 x 64 torus at q = 0.6585 (J_c(q) = 0.6585 by eq. (12)), a warm-up
    # plan then a moments plan; the sums equal those of the oracle's records,
    # and m relaxes to 0 below the curve, stays near -1 above it and
    # fluctuates most near J_c
    q, L, warm, rec = 0.6585, 64, 4000, 4000
    Js = np.array([0.3, 0.6585, 1.0])
    qs = np.full(3, q)
    Ls = np.full(3, L)
    st = np.arange(3, dtype=np.uint32)
    pw = sd.sd_batch_plan_create(Js, qs, Ls, st, seed=5, k_steps=warm, obs_every=0)
    pr = sd.sd_batch_plan_create(Js, qs, Ls, st, seed=5, k_steps=rec, obs_every=1, flags=sd.SD_FLAG_MOMENTS)
    lat = torch.zeros(sd.sd_batch_lattice_bytes(pr), dtype=torch.uint8, device="cuda")
    mom = torch.zeros(sd.sd_batch_trace_len(pr), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(pw, lat, sd.SD_INIT_DOWN)
    sd.sd_batch_run(pw, lat, None, 0)
    sd.sd_batch_run(pr, lat, mom, warm)
    torch.cuda.synchronize()
    got = mom.cpu().numpy().reshape(3, 5)
    pw.close()
    pr.close()
    for c in range(3):
        s0 = np.full((L, L), -1, np.int8)
        s1, _, _ = oracle.run(s0, Js[c], q, 5, c, 0, warm)
        _, _, obs = oracle.run(s1, Js[c], q, 5, c, warm, rec, obs_every=1)
        M, A, B = (obs[:, i].astype(np.int64) for i in range(3))
        assert np.array_equal(got[c], [M.sum(), (M * M).sum(), np.abs(M).sum(), A.sum(), B.sum()]), c
    S = got.astype(np.float64)
    N = float(L * L)
    mean = S[:, 0] / (rec * N)
    var = S[:, 1] / (rec * N * N) - mean ** 2
    absm = S[:, 2] / (rec * N)
    assert absm[0] < 0.05 and mean[2] < -0.95
    assert var[1] > 3 * var[0] and var[1] > 3 * var[2]


def test_coalescence_times_match_oracle(oracle):
    # section 3.2: chains from all +1 and all -1 sharing a stream stay ordered
    # site by site, so they have met exactly when their magnetisations agree;
    # the first such step from the batched records equals the first step at
    # which the oracle's two lattices are identical
    L, J, q, n_pairs, chunk, cap = 16, 0.45, 0.45, 8, 25, 1000
    n = 2 * n_pairs
    streams = np.repeat(np.arange(300, 300 + n_pairs, dtype=np.uint32), 2)
    plan = sd.sd_batch_plan_create(np.full(n, J), np.full(n, q), np.full(n, L), streams, seed=SEED,
                                   k_steps=chunk, obs_every=1)
    lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
    tr = torch.zeros(sd.sd_batch_trace_len(plan), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan, lat, sd.SD_INIT_DOWN)
    nb = sd.sd_lattice_bytes(L, sd.SD_P64)
    for p_ in range(n_pairs):
        off = sd.sd_batch_chain_offset(plan, 2 * p_, 0)
        lat[off:off + nb].fill_(0xFF)
    M = []
    for step in range(0, cap, chunk):
        sd.sd_batch_run_direct(plan, lat, tr, step)
        torch.cuda.synchronize()
        M.append(tr.view(n, chunk, 3)[:, :, 0].cpu().numpy().copy())
    plan.close()
    M = np.concatenate(M, axis=1)
    for p_ in range(n_pairs):
        eq = np.flatnonzero(M[2 * p_] == M[2 * p_ + 1])
        t_gpu = int(eq[0]) + 1 if len(eq) else -1
        top = np.ones((L, L), np.int8)
        bot = -np.ones((L, L), np.int8)
        t_ref = -1
        for step in range(cap):
            top, _, _ = oracle.run(top, J, q, SEED, 300 + p_, step, 1)
            bot, _, _ = oracle.run(bot, J, q, SEED, 300 + p_, step, 1)
            assert np.all(top >= bot)
            if np.array_equal(top, bot):
                t_ref = step + 1
                break
        assert t_gpu == t_ref, (p_, t_gpu, t_ref)
        assert t_ref > 0
