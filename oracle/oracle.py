"""Python access to the shaken-dynamics CPU oracle.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product library never loads it.

Thin ctypes marshalling over ``shaken_oracle.c`` (built into
``oracle/libshaken_oracle.so`` by :func:`build`); every array is a host numpy
array, int8 lattices hold +1 / -1 in row-major order (site s = j*L + i).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shaken_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libshaken_oracle.so")

INIT_UP, INIT_DOWN, INIT_RANDOM = 0, 1, 2
TAG_DYNAMICS, TAG_INIT = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", _SRC, "-lm", "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i8p = ctypes.POINTER(ctypes.c_int8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        c = ctypes
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_philox4x32_10.restype = None
        L.or_site_uniform.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32, c.c_uint32, c.c_uint64]
        L.or_site_uniform.restype = c.c_uint32
        L.or_set_complement.argtypes = [c.c_int]
        L.or_set_complement.restype = None
        L.or_threshold.argtypes = [c.c_double]
        L.or_threshold.restype = c.c_uint32
        L.or_threshold_table.argtypes = [c.c_double, c.c_double, u32p]
        L.or_threshold_table.restype = None
        L.or_init.argtypes = [i8p, c.c_int, c.c_int, c.c_double, c.c_uint64, c.c_uint32]
        L.or_init.restype = c.c_int
        L.or_row_thresholds.argtypes = [i8p, c.c_int, c.c_double, c.c_double, c.c_int, c.c_int, u32p]
        L.or_row_thresholds.restype = None
        for name in ("or_half_step_A", "or_half_step_B"):
            f = getattr(L, name)
            f.argtypes = [i8p, i8p, c.c_int, c.c_double, c.c_double, c.c_uint64, c.c_uint32, c.c_uint32]
            f.restype = None
        L.or_observe.argtypes = [i8p, i8p, c.c_int, i64p]
        L.or_observe.restype = None
        L.or_corr_row.argtypes = [i8p, c.c_int, c.c_int, i64p]
        L.or_corr_row.restype = c.c_int
        L.or_corr_diag.argtypes = [i8p, c.c_int, c.c_int, i64p]
        L.or_corr_diag.restype = c.c_int
        L.or_run.argtypes = [i8p, i8p, c.c_int, c.c_double, c.c_double, c.c_uint64, c.c_uint32,
                             c.c_uint64, c.c_uint32, i64p, c.c_uint32]
        L.or_run.restype = c.c_int
        L.or_loglik_counts.argtypes = [i8p, c.c_int, c.c_int, c.c_int, i64p]
        L.or_loglik_counts.restype = c.c_int
        L.or_propp_wilson.argtypes = [i8p, c.c_int, c.c_double, c.c_double, c.c_uint64, c.c_uint32, c.c_uint64,
                                      c.c_uint32, c.c_uint32]
        L.or_propp_wilson.restype = c.c_int64
        L.or_loglik_stats.argtypes = [i8p, c.c_int, c.c_int, c.c_int, i64p]
        L.or_loglik_stats.restype = c.c_int
        L.or_loglik_from_stats.argtypes = [i64p, c.c_double, c.c_double, ctypes.POINTER(c.c_double)]
        L.or_loglik_from_stats.restype = c.c_double
        L.or_loglik.argtypes = [i64p, c.c_double, c.c_double]
        L.or_loglik.restype = c.c_double
        L.or_loglik_grad.argtypes = [i64p, c.c_double, c.c_double, ctypes.POINTER(c.c_double)]
        L.or_loglik_grad.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _lat(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int8)
    return a


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def site_uniform(seed: int, stream: int, t: int, tag: int, s: int) -> int:
    return int(lib().or_site_uniform(seed, stream, t, tag, s))


class complement_randoms:
    """Context manager: replace every oracle uniform r by 2^32 - 1 - r."""

    def __enter__(self):
        lib().or_set_complement(1)
        return self

    def __exit__(self, *exc):
        lib().or_set_complement(0)
        return False


def threshold(h: float) -> int:
    return int(lib().or_threshold(float(h)))


def threshold_table(J: float, q: float) -> np.ndarray:
    T = np.zeros(6, dtype=np.uint32)
    lib().or_threshold_table(float(J), float(q), _p(T, ctypes.c_uint32))
    return T


def init(L: int, kind: int, p_up: float = 0.5, seed: int = 1, stream: int = 0) -> np.ndarray:
    sigma = np.zeros(L * L, dtype=np.int8)
    rc = lib().or_init(_p(sigma, ctypes.c_int8), L, kind, float(p_up), seed, stream)
    if rc != 0:
        raise ValueError("oracle init rejected its arguments")
    return sigma.reshape(L, L)


def row_thresholds(src: np.ndarray, J: float, q: float, which: int) -> np.ndarray:
    """Per-site thresholds used by half-step A (which=0) or B (which=1)."""
    src = _lat(src)
    L = src.shape[0]
    out = np.zeros((L, L), dtype=np.uint32)
    row = np.zeros(L, dtype=np.uint32)
    for j in range(L):
        lib().or_row_thresholds(_p(src, ctypes.c_int8), L, float(J), float(q), which, j,
                                _p(row, ctypes.c_uint32))
        out[j] = row
    return out


def row_thresholds_of(src: np.ndarray, J: float, q: float, which: int, j: int) -> np.ndarray:
    """Thresholds of the sites of row j only (src is the whole L x L lattice)."""
    src = _lat(src)
    L = src.shape[0]
    row = np.zeros(L, dtype=np.uint32)
    lib().or_row_thresholds(_p(src, ctypes.c_int8), L, float(J), float(q), which, j, _p(row, ctypes.c_uint32))
    return row


def half_step(src: np.ndarray, J: float, q: float, which: int, seed: int, stream: int, t: int) -> np.ndarray:
    src = _lat(src)
    L = src.shape[0]
    dst = np.zeros_like(src)
    f = lib().or_half_step_A if which == 0 else lib().or_half_step_B
    f(_p(src, ctypes.c_int8), _p(dst, ctypes.c_int8), L, float(J), float(q), seed, stream, t)
    return dst


def observe(sigma: np.ndarray, tau: np.ndarray) -> np.ndarray:
    sigma, tau = _lat(sigma), _lat(tau)
    out = np.zeros(3, dtype=np.int64)
    lib().or_observe(_p(sigma, ctypes.c_int8), _p(tau, ctypes.c_int8), sigma.shape[0], _p(out, ctypes.c_int64))
    return out


def corr_row(sigma: np.ndarray, rmax: int) -> np.ndarray:
    sigma = _lat(sigma)
    out = np.zeros(rmax + 1, dtype=np.int64)
    rc = lib().or_corr_row(_p(sigma, ctypes.c_int8), sigma.shape[0], rmax, _p(out, ctypes.c_int64))
    if rc != 0:
        raise ValueError("rmax out of range")
    return out


def corr_diag(sigma: np.ndarray, lmax: int) -> np.ndarray:
    """[2, lmax+1] int64: row 0 the SW-NE sums sum_x s(i,j) s(i+l,j+l), row 1 the
    NW-SE sums sum_x s(i,j) s(i+l,j-l) (section 3.3, Table 1)."""
    sigma = _lat(sigma)
    out = np.zeros(2 * (lmax + 1), dtype=np.int64)
    rc = lib().or_corr_diag(_p(sigma, ctypes.c_int8), sigma.shape[0], lmax, _p(out, ctypes.c_int64))
    if rc != 0:
        raise ValueError("lmax out of range")
    return out.reshape(2, lmax + 1)


def run(sigma: np.ndarray, J: float, q: float, seed: int, stream: int, step0: int, k: int,
        obs_every: int = 0, tau: np.ndarray | None = None):
    """k full steps from step index step0.  Returns (sigma, tau, obs[n_rec, 3])."""
    sigma = _lat(sigma).copy()
    L = sigma.shape[0]
    tau = np.zeros_like(sigma) if tau is None else _lat(tau).copy()
    n_rec = (k // obs_every) if obs_every else 0
    obs = np.zeros((max(n_rec, 1), 3), dtype=np.int64)
    rc = lib().or_run(_p(sigma, ctypes.c_int8), _p(tau, ctypes.c_int8), L, float(J), float(q), seed,
                      stream, step0, k, _p(obs, ctypes.c_int64) if obs_every else None, obs_every)
    if rc != 0:
        raise ValueError("oracle run rejected its arguments")
    return sigma, tau, obs[:n_rec]


def trajectory(sigma0: np.ndarray, J: float, q: float, seed: int, stream: int, step0: int, k: int) -> np.ndarray:
    """Lattices X_0 = sigma_0, X_1 = tau_1, X_2 = sigma_1, ... (2k + 1 of them)."""
    X = [_lat(sigma0).copy()]
    for m in range(k):
        n = step0 + m
        X.append(half_step(X[-1], J, q, 0, seed, stream, 2 * n))
        X.append(half_step(X[-1], J, q, 1, seed, stream, 2 * n + 1))
    return np.stack(X)


def propp_wilson(L: int, J: float, q: float, seed: int, stream: int, step_end: int, T0: int, T_max: int):
    """Coupling from the past: (sample [L, L] int8, T that coalesced or 0)."""
    out = np.zeros((L, L), dtype=np.int8)
    T = int(lib().or_propp_wilson(_p(out, ctypes.c_int8), L, float(J), float(q), seed, stream, step_end, T0, T_max))
    if T < 0:
        raise ValueError("oracle Propp-Wilson rejected its arguments")
    return out, T


def loglik_counts(traj: np.ndarray) -> np.ndarray:
    """traj: [n_traj, n_lat, L, L] int8 -> 12 int64 counts."""
    traj = np.ascontiguousarray(traj, dtype=np.int8)
    n_traj, n_lat, L, _ = traj.shape
    out = np.zeros(12, dtype=np.int64)
    rc = lib().or_loglik_counts(_p(traj, ctypes.c_int8), n_traj, n_lat, L, _p(out, ctypes.c_int64))
    if rc != 0:
        raise ValueError("bad trajectory shape")
    return out


def loglik_stats(traj: np.ndarray) -> np.ndarray:
    """traj: [n_traj, n_lat, L, L] int8 -> 6 int64 paired statistics
    (S_0, S_1, S_2, Z_0, Z_1, Z_2) of the class pairs (0,5), (1,4), (2,3)."""
    traj = np.ascontiguousarray(traj, dtype=np.int8)
    n_traj, n_lat, L, _ = traj.shape
    out = np.zeros(6, dtype=np.int64)
    rc = lib().or_loglik_stats(_p(traj, ctypes.c_int8), n_traj, n_lat, L, _p(out, ctypes.c_int64))
    if rc != 0:
        raise ValueError("bad trajectory shape")
    return out


def loglik_from_stats(stats: np.ndarray, J: float, q: float):
    """(LL, gradient) in FP64 from the 6 paired statistics."""
    st = np.ascontiguousarray(stats, dtype=np.int64)
    g = np.zeros(2, dtype=np.float64)
    ll = float(lib().or_loglik_from_stats(_p(st, ctypes.c_int64), float(J), float(q), _p(g, ctypes.c_double)))
    return ll, g


def loglik(counts: np.ndarray, J: float, q: float) -> float:
    c = np.ascontiguousarray(counts, dtype=np.int64)
    return float(lib().or_loglik(_p(c, ctypes.c_int64), float(J), float(q)))


def loglik_grad(counts: np.ndarray, J: float, q: float) -> np.ndarray:
    c = np.ascontiguousarray(counts, dtype=np.int64)
    g = np.zeros(2, dtype=np.float64)
    lib().or_loglik_grad(_p(c, ctypes.c_int64), float(J), float(q), _p(g, ctypes.c_double))
    return g
