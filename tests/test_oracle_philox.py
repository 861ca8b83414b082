"""Pins of the oracle's random stream.

* The Philox4x32-10 bijection against rocRAND's independently written engine
  (a second implementation of the SC'11 generator, called through its public
  header), on random and on extreme counters and keys.
* The per-site uniform against the stream contract, rebuilt here from raw
  Philox outputs, and a coarse uniformity check.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_bijection(tmp_path_factory):
    gxx = shutil.which("g++")
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if gxx is None or not os.path.exists(hdr):
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("xcheck") / "philox_xcheck")
    subprocess.run([gxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "helpers", "rocrand_philox_xcheck.cpp"), "-o", exe], check=True)

    def apply(rows):
        text = "\n".join(" ".join("%08x" % x for x in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]

    return apply


def test_philox_matches_rocrand(oracle, rocrand_bijection):
    rng = np.random.default_rng(20190819)
    rows = rng.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64).astype(np.uint32)
    # include counters shaped like the stream contract's (small words, top bits set)
    rows[:8, 0] = np.arange(8)
    rows[:8, 1] = (np.arange(8) % 4) << 30
    rows[8] = 0                    # all-zero counter and key
    rows[9] = 0xFFFFFFFF           # all-one counter and key
    rows[10, 4:6] = 0              # zero key, random counter
    ref = rocrand_bijection(rows.tolist())
    for r, expected in zip(rows, ref):
        got = oracle.philox4x32_10(r[:4], r[4:6])
        assert list(got) == expected


def _contract_uniform(oracle, seed, stream, t, tag, s):
    """r_s rebuilt from raw Philox words following the stream contract."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    g, b = s >> 6, s & 63
    planes = []
    for p in range(4):
        x = [int(v) for v in oracle.philox4x32_10([stream, t | (p << 30), 2 * tag, g], key)]
        planes.append(x[0] | (x[1] << 32))
        planes.append(x[2] | (x[3] << 32))
    top = 0
    for m in range(8):
        top = (top << 1) | ((planes[m] >> b) & 1)
    y = oracle.philox4x32_10([stream, t, 2 * tag + 1, s >> 2], key)
    return (top << 24) | (int(y[s & 3]) >> 8)


def test_site_uniform_follows_contract(oracle):
    rng = np.random.default_rng(7)
    for _ in range(300):
        seed = int(rng.integers(0, 2 ** 63))
        stream = int(rng.integers(0, 2 ** 32))
        t = int(rng.integers(0, 2 ** 30))
        tag = int(rng.integers(0, 2))
        s = int(rng.integers(0, 2 ** 32))
        assert oracle.site_uniform(seed, stream, t, tag, s) == _contract_uniform(oracle, seed, stream, t, tag, s)


def test_site_uniform_is_uniform(oracle):
    # 16384 consecutive sites of one half-step: every one of the 256 top-byte
    # values and of 256 low-byte values appears with chi-square-plausible counts.
    r = np.array([oracle.site_uniform(1, 3, 10, 0, s) for s in range(16384)], dtype=np.uint64)
    for byte in (r >> 24, (r >> 8) & 0xFF):
        counts = np.bincount(byte.astype(np.int64), minlength=256)
        chi2 = float(((counts - 64.0) ** 2 / 64.0).sum())
        assert 150 < chi2 < 380, chi2   # 255 dof, roughly the 1e-6 tails
    assert len(np.unique(r)) > 16384 - 5


def test_site_uniform_depends_on_every_counter_input(oracle):
    # The uniform of site s at half-step t must change with t, with the
    # site's 64-site group, its position inside the group, the half-step
    # tag and the stream: each pair below compares 16384 sites of one
    # half-step with a second set that differs in one of these inputs.
    # Independent 24-bit tails coincide with probability 2^-24 and top bytes
    # with probability 1/256; a counter that dropped the input would make
    # every tail (or every top byte) coincide.  The Pearson correlation of
    # the tails must also be that of independent draws (|r| < 5/sqrt(n)).
    n = 16384
    sites = np.arange(n)

    def draw(stream, t, tag, offset):
        return np.array([oracle.site_uniform(1, stream, t, tag, int(s) + offset) for s in sites], dtype=np.uint64)

    base = draw(3, 10, 0, 0)
    for other in (draw(3, 11, 0, 0),      # next half-step index
                  draw(3, 10, 1, 0),      # the other half-step tag
                  draw(4, 10, 0, 0),      # next stream
                  draw(3, 10, 0, 64),     # same bit of the next 64-site group
                  draw(3, 10, 0, 4),      # same Philox output word, next counter
                  draw(3, 10, 0, 1)):     # next output word of the same call
        tail_a, tail_b = base & 0xFFFFFF, other & 0xFFFFFF
        assert int((tail_a == tail_b).sum()) <= 3
        top_same = int(((base >> 24) == (other >> 24)).sum())
        assert 20 < top_same < 120, top_same   # 64 expected
        r = np.corrcoef(tail_a.astype(np.float64), tail_b.astype(np.float64))[0, 1]
        assert abs(r) < 5 / np.sqrt(n), r
    # within one site: the tail is not a function of the top byte
    r = np.corrcoef((base >> 24).astype(np.float64), (base & 0xFFFFFF).astype(np.float64))[0, 1]
    assert abs(r) < 5 / np.sqrt(n), r
