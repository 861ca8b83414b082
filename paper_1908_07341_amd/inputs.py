"""Seeded synthetic inputs shared by the tests and the benchmark.

Nothing here computes any part of the shaken dynamics: it produces random
+-1 lattices, converts between the int8 and bit-packed byte layouts, and lays
out the (q, J, L) table of the batched scan.
"""
from __future__ import annotations

import numpy as np


def random_lattice(L: int, seed: int, p_up: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L, L)) < p_up, 1, -1).astype(np.int8)


def pack_bits(lattice: np.ndarray) -> np.ndarray:
    """int8 +-1 lattice -> packed bytes, bit s of the lattice = bit s % 8 of byte s / 8."""
    flat = (np.asarray(lattice).reshape(-1) > 0).astype(np.uint8)
    return np.packbits(flat, bitorder="little")


def unpack_bits(packed: np.ndarray, L: int) -> np.ndarray:
    """Packed bytes (any integer dtype view) -> int8 +-1 lattice [L, L]."""
    raw = np.ascontiguousarray(packed).view(np.uint8).reshape(-1)
    bits = np.unpackbits(raw, bitorder="little")[: L * L]
    return (2 * bits.astype(np.int8) - 1).reshape(L, L)


def scan_table(n_q: int = 64, n_J: int = 64, q_max: float = 2.0, J_max: float = 1.5,
               sizes=(128, 256, 512), seed: int = 1):
    """The batched (q, J) scan: chain c = a * n_J + b has q = q_max * a / (n_q - 1),
    J = J_max * b / (n_J - 1) and a lattice size drawn uniformly from `sizes`
    with numpy's default_rng(seed).  Returns (q, J, L) arrays."""
    a, b = np.meshgrid(np.arange(n_q), np.arange(n_J), indexing="ij")
    q = q_max * a.reshape(-1) / (n_q - 1)
    J = J_max * b.reshape(-1) / (n_J - 1)
    rng = np.random.default_rng(seed)
    L = rng.choice(np.asarray(sizes), size=q.size)
    return q.astype(np.float64), J.astype(np.float64), L.astype(np.int32)


def pack_replicas(lattices: np.ndarray) -> np.ndarray:
    """int8 +-1 lattices [64, L, L] -> replica words [L * L] uint64, bit r of
    word s = site s of replica r (1 = +1)."""
    lat = np.asarray(lattices)
    bits = (lat.reshape(lat.shape[0], -1) > 0).astype(np.uint64)
    shifts = np.arange(lat.shape[0], dtype=np.uint64)[:, None]
    return np.bitwise_or.reduce(bits << shifts, axis=0)


def unpack_replicas(words: np.ndarray, L: int, n: int = 64) -> np.ndarray:
    """Replica words [L * L] (any 8-byte dtype view) -> int8 +-1 lattices [n, L, L]."""
    w = np.ascontiguousarray(words).view(np.uint64).reshape(-1)
    bits = (w[None, :] >> np.arange(n, dtype=np.uint64)[:, None]) & np.uint64(1)
    return (2 * bits.astype(np.int8) - 1).reshape(n, L, L)
