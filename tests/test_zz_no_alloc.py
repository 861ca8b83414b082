"""The allocation-free chain entry point (sd_run_noalloc) through the C ABI:
two calls in a row, the second on a smaller lattice, each bit-identical to
sd_run on the same inputs (lattices and every record).  Both calls take the
grid kernels with records, so that the partial sums go through the library's
static scratch array; the first spans several chunks of records (several
finishing launches), the second starts from a later step index with a record
every third step."""
import pytest
import torch

import paper_1908_07341_amd as sd

pytestmark = pytest.mark.gpu

SEED = 0x5EED0001


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sd.lib()


def _start(L, layout, stream):
    sigma = sd.new_lattice(L, layout)
    sd.sd_init(sigma, L, layout, sd.SD_INIT_RANDOM, 0.5, SEED, stream)
    return sigma


# (L, layout, J, q, stream, step0, k_steps, obs_every, flags): 4096^2 packed
# runs 256 workgroups, so 64 records fill the scratch array and 150 records
# take three finishing launches; 1024^2 int8 is the smaller second call
CALLS = [
    (4096, sd.SD_P64, 0.5, 0.5, 3, 0, 150, 1, 0),
    (1024, sd.SD_I8, 0.8, 0.3, 7, 11, 31, 3, 0),
]


def _one(fn, L, layout, J, q, stream, step0, k, every, flags, start):
    sigma = start.clone()
    tau = torch.empty_like(sigma)
    obs = torch.full((k // every, 3), -7, dtype=torch.int64, device="cuda")
    fn(sigma, tau, L, layout, J, q, SEED, stream, step0, k, obs, every, flags)
    torch.cuda.synchronize()
    return sigma, tau, obs


def test_noalloc_matches_sd_run_on_two_calls():
    results = []
    for L, layout, J, q, stream, step0, k, every, flags in CALLS:
        print(f"sd_run_noalloc L={L} layout={layout} J={J} q={q} k={k} every={every}", flush=True)
        start = _start(L, layout, stream)
        got = _one(sd.sd_run_noalloc, L, layout, J, q, stream, step0, k, every, flags, start)
        ref = _one(sd.sd_run, L, layout, J, q, stream, step0, k, every, flags, start)
        assert torch.equal(got[0], ref[0]), f"sigma differs at L={L}"
        assert torch.equal(got[1], ref[1]), f"tau differs at L={L}"
        assert torch.equal(got[2], ref[2]), f"records differ at L={L}"
        assert bool((got[2][:, 0].abs() <= L * L).all())
        results.append(got)
    # the first call's records are not what the second call left in the array
    assert not torch.equal(results[0][2][:1], results[1][2][:1])


def test_noalloc_rejects_bad_arguments():
    L = 1024
    sigma = _start(L, sd.SD_P64, 0)
    tau = torch.empty_like(sigma)
    obs = torch.zeros((4, 3), dtype=torch.int64, device="cuda")
    with pytest.raises(sd.ShakenError):
        sd.sd_run_noalloc(sigma, tau, L, sd.SD_P64, 0.5, 0.5, SEED, 0, 0, 4, obs, 0)   # obs without obs_every
    with pytest.raises(sd.ShakenError):
        sd.sd_run_noalloc(sigma, sigma, L, sd.SD_P64, 0.5, 0.5, SEED, 0, 0, 4)          # overlapping lattices
    with pytest.raises(sd.ShakenError):
        sd.sd_run_noalloc(sigma, tau, L, sd.SD_P64, float("nan"), 0.5, SEED, 0, 0, 4)
