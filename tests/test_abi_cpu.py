"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/shaken.h declares, computes the same threshold table as
the oracle, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1908_07341_amd as sd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^SD_API\s+[\w\s\*]+?\b(sd_\w+)\s*\(", text, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = sd.lib()
    declared = _declared_symbols()
    assert {"sd_run", "sd_init", "sd_half_step", "sd_observe", "sd_corr_row", "sd_threshold_table"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(sd.binding.SIGNATURES) == declared
    assert sd.sd_abi_version() == 1


def test_threshold_table_matches_oracle(oracle):
    rng = np.random.default_rng(5)
    pts = [(0.4, 0.6), (0.0, 0.0), (0.5, 0.5), (1.5, 2.0), (-0.7, 0.3), (0.6585, 0.6585), (5.0, 3.0)]
    pts += [tuple(x) for x in rng.uniform(-3, 3, size=(300, 2))]
    for J, q in pts:
        assert sd.sd_threshold_table(J, q) == [int(x) for x in oracle.threshold_table(J, q)], (J, q)


def test_lattice_bytes():
    assert sd.sd_lattice_bytes(64, sd.SD_I8) == 4096
    assert sd.sd_lattice_bytes(64, sd.SD_P64) == 512
    assert sd.sd_lattice_bytes(96, sd.SD_P32) == 96 * 96 // 8
    # P64 is the bit string of the lattice: any L % 8 == 0 (L * L fills whole words)
    assert sd.sd_lattice_bytes(96, sd.SD_P64) == 96 * 96 // 8
    assert sd.sd_lattice_bytes(200, sd.SD_P64) == 200 * 200 // 8
    assert sd.sd_lattice_bytes(8, sd.SD_P64) == 8
    assert sd.sd_lattice_bytes(100, sd.SD_P64) == 0
    assert sd.sd_lattice_bytes(4, sd.SD_P64) == 0
    assert sd.sd_lattice_bytes(40, sd.SD_P32) == 0
    assert sd.sd_lattice_bytes(3, sd.SD_I8) == 9
    assert sd.sd_lattice_bytes(1, sd.SD_I8) == 0
    assert sd.sd_lattice_bytes(65536, sd.SD_I8) == 0
    assert sd.sd_lattice_bytes(16384, sd.SD_P64) == 16384 * 16384 // 8


def test_fastdiv_exact():
    rng = np.random.default_rng(0)
    ds = list(range(1, 300)) + [1023, 1024, 1025, 16384, 65535, 65536, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1]
    ds += [int(x) for x in rng.integers(1, 2 ** 32, 200)]
    for d in ds:
        ns = [0, 1, d - 1, d, d + 1, 2 ** 32 - 1, 2 ** 32 - 2] + [int(x) for x in rng.integers(0, 2 ** 32, 50)]
        for n in ns:
            n &= 0xFFFFFFFF
            assert sd.sd_debug_fastdiv(n, d) == n // d, (n, d)


def test_bad_arguments_rejected_without_device_work():
    lib = sd.lib()
    st = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x10000)
    assert lib.sd_init(None, 64, sd.SD_I8, 0, 0.5, 1, 0, st) == sd.SD_EINVAL
    assert lib.sd_init(fake, 1, sd.SD_I8, 0, 0.5, 1, 0, st) == sd.SD_EINVAL
    assert lib.sd_init(fake, 100, sd.SD_P64, 0, 0.5, 1, 0, st) == sd.SD_EINVAL
    assert lib.sd_init(fake, 64, sd.SD_I8, 2, 1.5, 1, 0, st) == sd.SD_EINVAL
    assert lib.sd_init(fake, 64, sd.SD_I8, 7, 0.5, 1, 0, st) == sd.SD_EINVAL
    assert b"kind" in lib.sd_last_error()
    fake2 = ctypes.c_void_p(0x20000)
    assert lib.sd_half_step(fake, fake2, 64, sd.SD_I8, 2, 0.4, 0.6, 1, 0, 0, 0, st) == sd.SD_EINVAL
    assert lib.sd_half_step(fake, fake2, 64, sd.SD_I8, 0, float("nan"), 0.6, 1, 0, 0, 0, st) == sd.SD_EINVAL
    assert lib.sd_half_step(fake, fake2, 64, sd.SD_I8, 0, 0.4, 0.6, 1, 0, 2 ** 30, 0, st) == sd.SD_EINVAL
    assert lib.sd_half_step(fake, ctypes.c_void_p(0x10100), 64, sd.SD_I8, 0, 0.4, 0.6, 1, 0, 0, 0, st) == sd.SD_EINVAL
    assert b"overlap" in lib.sd_last_error()
    assert lib.sd_half_step(fake, fake2, 64, sd.SD_I8, 0, 0.4, 0.6, 1, 0, 0, 16, st) == sd.SD_EINVAL
    assert lib.sd_half_step(ctypes.c_void_p(0x10004), fake2, 64, sd.SD_P64, 0, 0.4, 0.6, 1, 0, 0, 0, st) == sd.SD_EINVAL
    assert lib.sd_run(fake, fake2, 64, sd.SD_I8, 0.4, 0.6, 1, 0, 0, 10, fake, 0, 0, st) == sd.SD_EINVAL
    assert lib.sd_run(fake, fake2, 64, sd.SD_I8, 0.4, 0.6, 1, 0, 2 ** 29, 1, None, 0, 0, st) == sd.SD_EINVAL
    assert lib.sd_observe(fake, fake2, 64, sd.SD_I8, None, st) == sd.SD_EINVAL
    assert lib.sd_corr_row(fake, 64, sd.SD_I8, 64, fake2, st) == sd.SD_EINVAL
    assert lib.sd_corr_row(fake, 64, sd.SD_I8, -1, fake2, st) == sd.SD_EINVAL
    lats = (ctypes.c_void_p * 17)(*([0x10000 + 0x10000 * a for a in range(17)]))
    assert lib.sd_corr_row_many(lats, 0, 64, sd.SD_I8, 3, fake2, st) == sd.SD_EINVAL
    assert lib.sd_corr_row_many(lats, 17, 64, sd.SD_I8, 3, fake2, st) == sd.SD_EINVAL
    assert lib.sd_corr_row_many(None, 2, 64, sd.SD_I8, 3, fake2, st) == sd.SD_EINVAL
    assert lib.sd_corr_row_many(lats, 2, 64, sd.SD_I8, 64, fake2, st) == sd.SD_EINVAL
    assert lib.sd_corr_row_many(lats, 2, 64, sd.SD_I8, 3, None, st) == sd.SD_EINVAL
    lats[1] = 0x10004
    assert lib.sd_corr_row_many(lats, 2, 64, sd.SD_P64, 3, fake2, st) == sd.SD_EINVAL
    assert b"aligned" in lib.sd_last_error()
    lats[1] = None
    assert lib.sd_corr_row_many(lats, 2, 64, sd.SD_I8, 3, fake2, st) == sd.SD_EINVAL
    assert lib.sd_corr_diag(fake, 64, sd.SD_I8, 64, fake2, st) == sd.SD_EINVAL
    assert lib.sd_corr_diag(fake, 64, sd.SD_I8, 3, None, st) == sd.SD_EINVAL
    assert lib.sd_trajectories(fake, fake2, -1, 64, sd.SD_P64, 0.4, 0.6, 1, 0, 0, 2, st) == sd.SD_EINVAL
    assert lib.sd_trajectories(fake, fake2, 2, 64, sd.SD_I8, 0.4, 0.6, 1, 0, 0, 2, st) == sd.SD_EUNSUPPORTED
    assert lib.sd_loglik_stats(fake, 1, 3, 96, fake2, st) == sd.SD_EINVAL
    assert b"sd_loglik_stats" in lib.sd_last_error()
    assert lib.sd_loglik_stats(ctypes.c_void_p(0x10004), 1, 3, 64, fake2, st) == sd.SD_EINVAL
    assert lib.sd_loglik_stats(fake, 1, 0, 64, fake2, st) == sd.SD_EINVAL
    assert lib.sd_loglik_stats(fake, 1, 3, 64, None, st) == sd.SD_EINVAL
    assert lib.sd_loglik_fwd_stats(None, fake, fake2, st) == sd.SD_EINVAL
    assert lib.sd_loglik_bwd_stats(fake, fake, None, None, st) == sd.SD_EINVAL
    Jr = (ctypes.c_double * 64)(*([0.4] * 64))
    far = ctypes.c_void_p(0x100000)
    assert lib.sd_replica_run(fake, far, 12, Jr, Jr, 1, 0, 0, 2, st) == sd.SD_EINVAL
    assert lib.sd_replica_run(fake, ctypes.c_void_p(0x10040), 16, Jr, Jr, 1, 0, 0, 2, st) == sd.SD_EINVAL
    assert b"overlap" in lib.sd_last_error()
    assert lib.sd_replica_run(fake, far, 16, None, Jr, 1, 0, 0, 2, st) == sd.SD_EINVAL
    Jr[63] = float("inf")
    assert lib.sd_replica_run(fake, far, 16, Jr, Jr, 1, 0, 0, 2, st) == sd.SD_EINVAL
    assert lib.sd_replica_observe(fake, far, 16, None, st) == sd.SD_EINVAL
    assert sd.sd_replica_lattice_bytes(16) == 16 * 16 * 8 and sd.sd_replica_lattice_bytes(12) == 0
    tu = (ctypes.c_int64 * 4)()
    assert lib.sd_propp_wilson(fake, far, 4, 12, 0.4, 0.5, 1, 0, 100, 1, 10, tu, st) == sd.SD_EINVAL
    assert lib.sd_propp_wilson(fake, far, 4, 16, -0.4, 0.5, 1, 0, 100, 1, 10, tu, st) == sd.SD_EINVAL
    assert b"monotone" in lib.sd_last_error()
    assert lib.sd_propp_wilson(fake, far, 4, 16, 0.4, 0.5, 1, 0, 100, 1, 200, tu, st) == sd.SD_EINVAL
    assert lib.sd_propp_wilson(fake, far, 4, 16, 0.4, 0.5, 1, 0, 2 ** 30, 1, 200, tu, st) == sd.SD_EINVAL
    assert lib.sd_propp_wilson(fake, far, 4, 16, 0.4, 0.5, 1, 0, 100, 0, 10, tu, st) == sd.SD_EINVAL
    assert lib.sd_propp_wilson(fake, ctypes.c_void_p(0x10010), 4, 16, 0.4, 0.5, 1, 0, 100, 1, 10, tu, st) == sd.SD_EINVAL
    assert b"overlap" in lib.sd_last_error()
    assert lib.sd_propp_wilson(fake, far, 4, 16, 0.4, 0.5, 1, 0, 100, 1, 10, None, st) == sd.SD_EINVAL
    out = (ctypes.c_uint32 * 6)()
    assert lib.sd_threshold_table(float("inf"), 0.1, out) == sd.SD_EINVAL
    assert lib.sd_threshold_table(0.1, 0.1, None) == sd.SD_EINVAL


def test_product_path_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_1908_07341_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in text.replace("no oracle", ""), os.path.join(dirpath, fn)
