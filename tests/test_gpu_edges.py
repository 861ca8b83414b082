"""GPU edge cases through the C ABI: calls with zero steps leave every buffer
as it was, zero-length requests do no device work, and a run shorter than its
record interval advances the chain without writing a record."""
import pytest
import torch

import paper_1908_07341_amd as sd

pytestmark = pytest.mark.gpu

SEED = 0x1234ABCD


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.lib()


def _pair(L, layout):
    sigma, tau = sd.new_lattice(L, layout), sd.new_lattice(L, layout)
    sd.sd_init(sigma, L, layout, sd.SD_INIT_RANDOM, 0.5, SEED, 1)
    sd.sd_init(tau, L, layout, sd.SD_INIT_RANDOM, 0.5, SEED, 2)
    return sigma, tau


# L = 64 and 96 take the single-workgroup kernel, 1024 int8 and 2048 packed
# the grid kernels
@pytest.mark.parametrize("L,layout", [(64, sd.SD_P64), (96, sd.SD_P64), (1024, sd.SD_I8), (2048, sd.SD_P64)])
def test_run_zero_steps_is_a_no_op(L, layout):
    print(f"zero-step run L={L} layout={layout}", flush=True)
    sigma, tau = _pair(L, layout)
    s0, t0 = sigma.clone(), tau.clone()
    obs = torch.full((4, 3), -7, dtype=torch.int64, device="cuda")
    sd.sd_run(sigma, tau, L, layout, 0.5, 0.5, SEED, 0, 0, 0, obs, 1)
    sd.sd_run(sigma, tau, L, layout, 0.5, 0.5, SEED, 0, 5, 0, None, 0)
    torch.cuda.synchronize()
    assert torch.equal(sigma, s0) and torch.equal(tau, t0)
    assert bool((obs == -7).all())


@pytest.mark.parametrize("L,layout", [(64, sd.SD_P64), (1024, sd.SD_I8), (2048, sd.SD_P64)])
def test_run_shorter_than_record_interval(L, layout):
    # 3 steps with a record every 5: the chain moves as without records and
    # the record buffer is not touched
    print(f"short run L={L} layout={layout}", flush=True)
    sigma, tau = _pair(L, layout)
    ref_s, ref_t = sigma.clone(), tau.clone()
    obs = torch.full((2, 3), -7, dtype=torch.int64, device="cuda")
    sd.sd_run(sigma, tau, L, layout, 0.4, 0.6, SEED, 3, 11, 3, obs, 5)
    sd.sd_run(ref_s, ref_t, L, layout, 0.4, 0.6, SEED, 3, 11, 3, None, 0)
    torch.cuda.synchronize()
    assert torch.equal(sigma, ref_s) and torch.equal(tau, ref_t)
    assert bool((obs == -7).all())
    assert not torch.equal(sigma, _pair(L, layout)[0])


@pytest.mark.parametrize("L", [64, 2048])
def test_trajectories_of_zero_steps_hold_the_start(L):
    # L = 64: one launch with LDS-resident lattices; 2048: one trajectory at a
    # time, whose first lattice is a copy of the start
    print(f"zero-step trajectories L={L}", flush=True)
    n = 3
    words = sd.sd_lattice_bytes(L, sd.SD_P64) // 8
    starts = torch.empty((n, words), dtype=torch.int64, device="cuda")
    for a in range(n):
        sd.sd_init(starts[a], L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, SEED, a)
    traj = torch.zeros((n, 1, words), dtype=torch.int64, device="cuda")
    sd.sd_trajectories(starts, traj, n, L, sd.SD_P64, 0.45, 0.7, SEED, 0, 0, 0)
    one = torch.zeros((1, words), dtype=torch.int64, device="cuda")
    sd.sd_trajectory(starts[1], one, L, sd.SD_P64, 0.45, 0.7, SEED, 1, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(traj[:, 0], starts)
    assert torch.equal(one[0], starts[1])


def test_zero_length_requests():
    print("zero-length requests", flush=True)
    L = 64
    words = sd.sd_lattice_bytes(L, sd.SD_P64) // 8
    starts = torch.zeros((1, words), dtype=torch.int64, device="cuda")
    traj = torch.full((1, 3, words), 5, dtype=torch.int64, device="cuda")
    sd.sd_trajectories(starts, traj, 0, L, sd.SD_P64, 0.45, 0.7, SEED, 0, 0, 1)
    torch.cuda.synchronize()
    assert bool((traj == 5).all())
    # no transitions: every count and statistic is zero
    counts = torch.full((12,), -1, dtype=torch.int64, device="cuda")
    stats = torch.full((6,), -1, dtype=torch.int64, device="cuda")
    sd.sd_loglik_counts(traj, 1, 1, L, counts)
    sd.sd_loglik_stats(traj, 1, 1, L, stats)
    torch.cuda.synchronize()
    assert bool((counts == 0).all()) and bool((stats == 0).all())


def test_replica_zero_steps_is_a_no_op():
    print("zero-step replica run", flush=True)
    L = 64
    nb = sd.sd_replica_lattice_bytes(L)
    sig = torch.empty(nb // 8, dtype=torch.int64, device="cuda")
    sig.random_()
    tau = torch.zeros_like(sig)
    s0 = sig.clone()
    J = [0.1 * (r % 10) for r in range(64)]
    q = [0.05 * (r % 20) for r in range(64)]
    sd.sd_replica_run(sig, tau, L, J, q, SEED, 1, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(sig, s0) and bool((tau == 0).all())
