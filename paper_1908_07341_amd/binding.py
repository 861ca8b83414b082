"""ctypes binding of libshaken with the names of include/shaken.h.

Argument marshalling only: tensors become device pointers, the current torch
stream becomes the hipStream_t, and a non-OK status becomes ShakenError.  All
work runs in the library's HIP kernels; there is no fallback: if libshaken.so
has not been built, loading fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libshaken.so")

SD_OK, SD_EINVAL, SD_EUNSUPPORTED, SD_EHIP, SD_ENOSPACE = 0, -1, -2, -3, -4
SD_I8, SD_P32, SD_P64 = 0, 1, 2
SD_INIT_UP, SD_INIT_DOWN, SD_INIT_RANDOM = 0, 1, 2
SD_FLAG_COMPLEMENT_RNG = 1
SD_FLAG_GLOBAL_KERNELS = 2
SD_FLAG_MOMENTS = 4
SD_FLAG_GENERAL_COMPARE = 8


class sd_chain_desc(ctypes.Structure):
    _fields_ = [("J", ctypes.c_double), ("q", ctypes.c_double), ("L", ctypes.c_int32), ("stream", ctypes.c_uint32)]

# Every function the header declares, with its ctypes signature.
_VP, _I32, _U32, _U64, _F64, _F32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_float)
SIGNATURES = {
    "sd_abi_version": (_I32, []),
    "sd_last_error": (ctypes.c_char_p, []),
    "sd_lattice_bytes": (ctypes.c_size_t, [_I32, _I32]),
    "sd_threshold_table": (_I32, [_F64, _F64, ctypes.POINTER(_U32)]),
    "sd_init": (_I32, [_VP, _I32, _I32, _I32, _F64, _U64, _U32, _VP]),
    "sd_half_step": (_I32, [_VP, _VP, _I32, _I32, _I32, _F64, _F64, _U64, _U32, _U32, _U32, _VP]),
    "sd_run": (_I32, [_VP, _VP, _I32, _I32, _F64, _F64, _U64, _U32, _U64, _U32, _VP, _U32, _U32, _VP]),
    "sd_run_noalloc": (_I32, [_VP, _VP, _I32, _I32, _F64, _F64, _U64, _U32, _U64, _U32, _VP, _U32, _U32, _VP]),
    "sd_run_many": (_I32, [_VP, _VP, _I32, _I32, _I32, _VP, _VP, _U64, _VP, _U64, _U32, _VP, _U32, _U32, _VP]),
    "sd_observe": (_I32, [_VP, _VP, _I32, _I32, _VP, _VP]),
    "sd_corr_row": (_I32, [_VP, _I32, _I32, _I32, _VP, _VP]),
    "sd_corr_row_many": (_I32, [_VP, _I32, _I32, _I32, _I32, _VP, _VP]),
    "sd_corr_diag": (_I32, [_VP, _I32, _I32, _I32, _VP, _VP]),
    "sd_batch_plan_create": (_I32, [ctypes.POINTER(_VP), ctypes.POINTER(sd_chain_desc), _I32, _I32, _U64, _U32,
                                     _U32, _U32, ctypes.c_char_p]),
    "sd_batch_lattice_bytes": (ctypes.c_size_t, [_VP]),
    "sd_batch_trace_len": (ctypes.c_size_t, [_VP]),
    "sd_batch_chain_offset": (ctypes.c_int64, [_VP, _I32, _I32]),
    "sd_batch_launch_shape": (_I32, [_VP, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                      ctypes.POINTER(_I32)]),
    "sd_batch_init": (_I32, [_VP, _VP, _I32, _F64, _VP]),
    "sd_batch_run": (_I32, [_VP, _VP, _VP, _U64, _VP]),
    "sd_batch_run_direct": (_I32, [_VP, _VP, _VP, _U64, _VP]),
    "sd_batch_plan_destroy": (None, [_VP]),
    "sd_batch_bucket_times": (_I32, [_VP, _I32, ctypes.POINTER(_F32), ctypes.POINTER(_F32)]),
    "sd_trajectory": (_I32, [_VP, _VP, _I32, _I32, _F64, _F64, _U64, _U32, _U64, _U32, _VP]),
    "sd_trajectories": (_I32, [_VP, _VP, _I32, _I32, _I32, _F64, _F64, _U64, _U32, _U64, _U32, _VP]),
    "sd_loglik_counts": (_I32, [_VP, _I32, _I32, _I32, _VP, _VP]),
    "sd_loglik_fwd": (_I32, [_VP, _VP, _VP, _VP]),
    "sd_loglik_bwd": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "sd_loglik_stats": (_I32, [_VP, _I32, _I32, _I32, _VP, _VP]),
    "sd_replica_lattice_bytes": (ctypes.c_size_t, [_I32]),
    "sd_replica_run": (_I32, [_VP, _VP, _I32, _VP, _VP, _U64, _U32, _U64, _U32, _VP]),
    "sd_replica_observe": (_I32, [_VP, _VP, _I32, _VP, _VP]),
    "sd_propp_wilson": (_I32, [_VP, _VP, _I32, _I32, _F64, _F64, _U64, _U32, _U64, _U32, _U32, _VP, _VP]),
    "sd_loglik_fwd_stats": (_I32, [_VP, _VP, _VP, _VP]),
    "sd_loglik_bwd_stats": (_I32, [_VP, _VP, _VP, _VP, _VP]),
    "sd_tune": (_I32, [_I32, _I32, ctypes.c_char_p, _VP]),
    "sd_tuned_choice": (_I32, [_I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                               ctypes.POINTER(_I32)]),
    "sd_debug_fastdiv": (_U32, [_U32, _U32]),
}


class ShakenError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libshaken status {status}: {message}")
        self.status = status


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(or python paper_1908_07341_amd/build.py)")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != SD_OK:
        raise ShakenError(status, lib().sd_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    if not t.is_cuda:
        raise ValueError("libshaken works on device tensors")
    if not t.is_contiguous():
        raise ValueError("libshaken needs contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, nbytes: int, what: str) -> None:
    """Raise ValueError if tensor t holds fewer than nbytes bytes.  The ABI
    takes raw pointers and cannot check lengths, so every wrapper checks the
    tensors it passes against what the library will read or write.  (A raw
    integer address is passed through unchecked.)"""
    if t is None or isinstance(t, int):
        return
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{what}: tensor holds {have} bytes, the call needs {nbytes}")


def _lattice(t, L: int, layout: int, what: str) -> None:
    nb = sd_lattice_bytes(L, layout)
    if nb:   # an unsupported (L, layout) is reported by the library itself
        _need(t, nb, what)


def _stream(hip_stream):
    if hip_stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(hip_stream, torch.cuda.Stream):
        return ctypes.c_void_p(hip_stream.cuda_stream)
    return ctypes.c_void_p(hip_stream)


def sd_abi_version() -> int:
    return int(lib().sd_abi_version())


def sd_lattice_bytes(L: int, layout: int) -> int:
    return int(lib().sd_lattice_bytes(L, layout))


def sd_threshold_table(J: float, q: float) -> list:
    out = (ctypes.c_uint32 * 6)()
    _check(lib().sd_threshold_table(float(J), float(q), out))
    return [int(x) for x in out]


def sd_init(lattice, L, layout, kind, p_up=0.5, seed=1, stream=0, hip_stream=None) -> None:
    _lattice(lattice, L, layout, "sd_init")
    _check(lib().sd_init(_ptr(lattice), L, layout, kind, float(p_up), seed, stream, _stream(hip_stream)))


def sd_half_step(src, dst, L, layout, which, J, q, seed, stream, t, flags=0, hip_stream=None) -> None:
    _lattice(src, L, layout, "sd_half_step(src)")
    _lattice(dst, L, layout, "sd_half_step(dst)")
    _check(lib().sd_half_step(_ptr(src), _ptr(dst), L, layout, which, float(J), float(q), seed, stream, t, flags,
                              _stream(hip_stream)))


def _run_sizes(name, sigma, tau, L, layout, k_steps, obs, obs_every) -> None:
    _lattice(sigma, L, layout, f"{name}(sigma)")
    _lattice(tau, L, layout, f"{name}(tau)")
    if obs is not None and obs_every:
        _need(obs, 24 * (k_steps // obs_every), f"{name}(obs)")


def sd_run(sigma, tau, L, layout, J, q, seed, stream, step0, k_steps, obs=None, obs_every=0, flags=0,
           hip_stream=None) -> None:
    _run_sizes("sd_run", sigma, tau, L, layout, k_steps, obs, obs_every)
    _check(lib().sd_run(_ptr(sigma), _ptr(tau), L, layout, float(J), float(q), seed, stream, step0, k_steps,
                        _ptr(obs), obs_every, flags, _stream(hip_stream)))


def sd_run_noalloc(sigma, tau, L, layout, J, q, seed, stream, step0, k_steps, obs=None, obs_every=0, flags=0,
                   hip_stream=None) -> None:
    _run_sizes("sd_run_noalloc", sigma, tau, L, layout, k_steps, obs, obs_every)
    _check(lib().sd_run_noalloc(_ptr(sigma), _ptr(tau), L, layout, float(J), float(q), seed, stream, step0, k_steps,
                                _ptr(obs), obs_every, flags, _stream(hip_stream)))


def sd_run_many(sigmas, taus, L, layout, J, q, seed, streams, step0, k_steps, obs=None, obs_every=0, flags=0,
                hip_stream=None) -> None:
    """Chains of one size advanced together; sigmas, taus: lists of device
    lattices; J, q, streams: one value per chain; obs: [n, k_steps // obs_every, 3]."""
    n = len(sigmas)
    if not (len(taus) == len(J) == len(q) == len(streams) == n):
        raise ValueError("sd_run_many: one sigma, tau, J, q and stream per chain")
    for a in range(n):
        _lattice(sigmas[a], L, layout, f"sd_run_many(sigma[{a}])")
        _lattice(taus[a], L, layout, f"sd_run_many(tau[{a}])")
    if obs is not None and obs_every:
        _need(obs, 24 * n * (k_steps // obs_every), "sd_run_many(obs)")
    sp = (ctypes.c_void_p * max(n, 1))(*[_ptr(t).value for t in sigmas])
    tp = (ctypes.c_void_p * max(n, 1))(*[_ptr(t).value for t in taus])
    Ja = (ctypes.c_double * max(n, 1))(*[float(x) for x in J])
    qa = (ctypes.c_double * max(n, 1))(*[float(x) for x in q])
    sa = (ctypes.c_uint32 * max(n, 1))(*[int(x) for x in streams])
    _check(lib().sd_run_many(ctypes.cast(sp, ctypes.c_void_p), ctypes.cast(tp, ctypes.c_void_p), n, L, layout,
                             ctypes.cast(Ja, ctypes.c_void_p), ctypes.cast(qa, ctypes.c_void_p), seed,
                             ctypes.cast(sa, ctypes.c_void_p), step0, k_steps, _ptr(obs), obs_every, flags,
                             _stream(hip_stream)))


def sd_observe(sigma, tau, L, layout, out3, hip_stream=None) -> None:
    _lattice(sigma, L, layout, "sd_observe(sigma)")
    _lattice(tau, L, layout, "sd_observe(tau)")
    _need(out3, 24, "sd_observe(out3)")
    _check(lib().sd_observe(_ptr(sigma), _ptr(tau), L, layout, _ptr(out3), _stream(hip_stream)))


def sd_corr_row(sigma, L, layout, rmax, out, hip_stream=None) -> None:
    _lattice(sigma, L, layout, "sd_corr_row(sigma)")
    _need(out, 8 * (rmax + 1), "sd_corr_row(out)")
    _check(lib().sd_corr_row(_ptr(sigma), L, layout, rmax, _ptr(out), _stream(hip_stream)))


def sd_corr_row_many(sigmas, L, layout, rmax, out, hip_stream=None) -> None:
    """D(r) of several lattices of one size; sigmas: list of device lattices;
    out: [len(sigmas), rmax + 1] int64."""
    n = len(sigmas)
    for a in range(n):
        _lattice(sigmas[a], L, layout, f"sd_corr_row_many(sigma[{a}])")
    _need(out, 8 * n * (rmax + 1), "sd_corr_row_many(out)")
    sp = (ctypes.c_void_p * max(n, 1))(*[_ptr(x).value for x in sigmas])
    _check(lib().sd_corr_row_many(ctypes.cast(sp, ctypes.c_void_p), n, L, layout, rmax, _ptr(out),
                                  _stream(hip_stream)))


def sd_corr_diag(sigma, L, layout, lmax, out, hip_stream=None) -> None:
    _lattice(sigma, L, layout, "sd_corr_diag(sigma)")
    _need(out, 16 * (lmax + 1), "sd_corr_diag(out)")
    _check(lib().sd_corr_diag(_ptr(sigma), L, layout, lmax, _ptr(out), _stream(hip_stream)))


def sd_trajectory(sigma0, traj, L, layout, J, q, seed, stream, step0, k_steps, hip_stream=None) -> None:
    _lattice(sigma0, L, layout, "sd_trajectory(sigma0)")
    _need(traj, (2 * k_steps + 1) * sd_lattice_bytes(L, layout), "sd_trajectory(traj)")
    _check(lib().sd_trajectory(_ptr(sigma0), _ptr(traj), L, layout, float(J), float(q), seed, stream, step0,
                               k_steps, _stream(hip_stream)))


def sd_trajectories(sigma0, traj, n_traj, L, layout, J, q, seed, stream0, step0, k_steps, hip_stream=None) -> None:
    nb = sd_lattice_bytes(L, layout)
    _need(sigma0, max(n_traj, 0) * nb, "sd_trajectories(sigma0)")
    _need(traj, max(n_traj, 0) * (2 * k_steps + 1) * nb, "sd_trajectories(traj)")
    _check(lib().sd_trajectories(_ptr(sigma0), _ptr(traj), n_traj, L, layout, float(J), float(q), seed, stream0, step0,
                                 k_steps, _stream(hip_stream)))


def _traj_bytes(n_traj, n_lat, L) -> int:
    return max(n_traj, 0) * max(n_lat, 0) * (L * L // 8 if L > 0 else 0)


def sd_loglik_counts(traj, n_traj, n_lat, L, counts12, hip_stream=None) -> None:
    _need(traj, _traj_bytes(n_traj, n_lat, L), "sd_loglik_counts(traj)")
    _need(counts12, 96, "sd_loglik_counts(counts12)")
    _check(lib().sd_loglik_counts(_ptr(traj), n_traj, n_lat, L, _ptr(counts12), _stream(hip_stream)))


def sd_loglik_fwd(counts12, Jq, ll, hip_stream=None) -> None:
    _need(counts12, 96, "sd_loglik_fwd(counts12)")
    _need(Jq, 8, "sd_loglik_fwd(Jq)")
    _need(ll, 4, "sd_loglik_fwd(ll)")
    _check(lib().sd_loglik_fwd(_ptr(counts12), _ptr(Jq), _ptr(ll), _stream(hip_stream)))


def sd_loglik_bwd(counts12, Jq, g_out, grad, hip_stream=None) -> None:
    _need(counts12, 96, "sd_loglik_bwd(counts12)")
    _need(Jq, 8, "sd_loglik_bwd(Jq)")
    _need(g_out, 4, "sd_loglik_bwd(g_out)")
    _need(grad, 8, "sd_loglik_bwd(grad)")
    _check(lib().sd_loglik_bwd(_ptr(counts12), _ptr(Jq), _ptr(g_out), _ptr(grad), _stream(hip_stream)))


def sd_loglik_stats(traj, n_traj, n_lat, L, stats6, hip_stream=None) -> None:
    _need(traj, _traj_bytes(n_traj, n_lat, L), "sd_loglik_stats(traj)")
    _need(stats6, 48, "sd_loglik_stats(stats6)")
    _check(lib().sd_loglik_stats(_ptr(traj), n_traj, n_lat, L, _ptr(stats6), _stream(hip_stream)))


def sd_loglik_fwd_stats(stats6, Jq, ll, hip_stream=None) -> None:
    _need(stats6, 48, "sd_loglik_fwd_stats(stats6)")
    _need(Jq, 8, "sd_loglik_fwd_stats(Jq)")
    _need(ll, 4, "sd_loglik_fwd_stats(ll)")
    _check(lib().sd_loglik_fwd_stats(_ptr(stats6), _ptr(Jq), _ptr(ll), _stream(hip_stream)))


def sd_loglik_bwd_stats(stats6, Jq, g_out, grad, hip_stream=None) -> None:
    _need(stats6, 48, "sd_loglik_bwd_stats(stats6)")
    _need(Jq, 8, "sd_loglik_bwd_stats(Jq)")
    _need(g_out, 4, "sd_loglik_bwd_stats(g_out)")
    _need(grad, 8, "sd_loglik_bwd_stats(grad)")
    _check(lib().sd_loglik_bwd_stats(_ptr(stats6), _ptr(Jq), _ptr(g_out), _ptr(grad), _stream(hip_stream)))


def sd_propp_wilson(samples, work, n_samples, L, J, q, seed, stream0, step_end, T0, T_max,
                    hip_stream=None) -> list:
    """Coupling-from-the-past samples into `samples`; returns T_used (n_samples ints)."""
    nb = sd_lattice_bytes(L, SD_P64)
    _need(samples, max(n_samples, 0) * nb, "sd_propp_wilson(samples)")
    _need(work, 4 * max(n_samples, 0) * nb, "sd_propp_wilson(work)")
    T_used = (ctypes.c_int64 * max(n_samples, 1))()
    _check(lib().sd_propp_wilson(_ptr(samples), _ptr(work), n_samples, L, J, q, seed, stream0, step_end, T0, T_max,
                                 ctypes.cast(T_used, ctypes.c_void_p), _stream(hip_stream)))
    return list(T_used[:n_samples])


def sd_replica_lattice_bytes(L: int) -> int:
    return int(lib().sd_replica_lattice_bytes(L))


def sd_replica_run(sigma, tau, L, J, q, seed, stream, step0, k_steps, hip_stream=None) -> None:
    """64 chains sharing one stream; J and q: 64 floats each (host)."""
    nb = sd_replica_lattice_bytes(L)
    if nb:
        _need(sigma, nb, "sd_replica_run(sigma)")
        _need(tau, nb, "sd_replica_run(tau)")
    Ja = (ctypes.c_double * 64)(*[float(x) for x in J])
    qa = (ctypes.c_double * 64)(*[float(x) for x in q])
    if len(J) != 64 or len(q) != 64:
        raise ValueError("sd_replica_run needs 64 values of J and of q")
    _check(lib().sd_replica_run(_ptr(sigma), _ptr(tau), L, ctypes.cast(Ja, ctypes.c_void_p),
                                ctypes.cast(qa, ctypes.c_void_p), seed, stream, step0, k_steps, _stream(hip_stream)))


def sd_replica_observe(sigma, tau, L, out, hip_stream=None) -> None:
    nb = sd_replica_lattice_bytes(L)
    if nb:
        _need(sigma, nb, "sd_replica_observe(sigma)")
        _need(tau, nb, "sd_replica_observe(tau)")
    _need(out, 192 * 8, "sd_replica_observe(out)")
    _check(lib().sd_replica_observe(_ptr(sigma), _ptr(tau), L, _ptr(out), _stream(hip_stream)))


class sd_batch_plan:
    """Owner of a libshaken batch plan handle (sd_batch_plan_destroy on close)."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)

    def close(self):
        if self.handle:
            lib().sd_batch_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sd_batch_plan_create(J, q, L, stream, layout=SD_P64, seed=1, k_steps=1, obs_every=1, flags=0,
                         tune_cache_path=None) -> sd_batch_plan:
    n = len(L)
    arr = (sd_chain_desc * n)()
    for i in range(n):
        arr[i].J, arr[i].q, arr[i].L, arr[i].stream = float(J[i]), float(q[i]), int(L[i]), int(stream[i])
    h = ctypes.c_void_p(0)
    path = tune_cache_path.encode() if tune_cache_path else None
    _check(lib().sd_batch_plan_create(ctypes.byref(h), arr, n, layout, seed, k_steps, obs_every, flags, path))
    return sd_batch_plan(h.value)


def sd_batch_lattice_bytes(plan: sd_batch_plan) -> int:
    return int(lib().sd_batch_lattice_bytes(plan.handle))


def sd_batch_trace_len(plan: sd_batch_plan) -> int:
    return int(lib().sd_batch_trace_len(plan.handle))


def sd_batch_chain_offset(plan: sd_batch_plan, chain: int, which: int) -> int:
    return int(lib().sd_batch_chain_offset(plan.handle, chain, which))


def sd_batch_launch_shape(plan: sd_batch_plan, bucket: int):
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().sd_batch_launch_shape(plan.handle, bucket, *[ctypes.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


def sd_batch_init(plan: sd_batch_plan, lattices, kind, p_up=0.5, hip_stream=None) -> None:
    _need(lattices, sd_batch_lattice_bytes(plan), "sd_batch_init(lattices)")
    _check(lib().sd_batch_init(plan.handle, _ptr(lattices), kind, float(p_up), _stream(hip_stream)))


def _batch_sizes(name, plan, lattices, traces) -> None:
    _need(lattices, sd_batch_lattice_bytes(plan), f"{name}(lattices)")
    _need(traces, 8 * sd_batch_trace_len(plan), f"{name}(traces)")


def sd_batch_run(plan: sd_batch_plan, lattices, traces, step0=0, hip_stream=None) -> None:
    _batch_sizes("sd_batch_run", plan, lattices, traces)
    _check(lib().sd_batch_run(plan.handle, _ptr(lattices), _ptr(traces), step0, _stream(hip_stream)))


def sd_batch_run_direct(plan: sd_batch_plan, lattices, traces, step0=0, hip_stream=None) -> None:
    _batch_sizes("sd_batch_run_direct", plan, lattices, traces)
    _check(lib().sd_batch_run_direct(plan.handle, _ptr(lattices), _ptr(traces), step0, _stream(hip_stream)))


def sd_batch_bucket_times(plan: sd_batch_plan, bucket: int):
    """(start_ms, end_ms) of a bucket's launch in the plan's last run (graph or
    direct), from the device's wall clock; synchronises the device."""
    a, b = ctypes.c_float(), ctypes.c_float()
    _check(lib().sd_batch_bucket_times(plan.handle, bucket, ctypes.byref(a), ctypes.byref(b)))
    return float(a.value), float(b.value)


def sd_batch_plan_destroy(plan: sd_batch_plan) -> None:
    plan.close()


def sd_tune(L: int, layout: int, tune_cache_path=None, hip_stream=None) -> None:
    path = tune_cache_path.encode() if tune_cache_path else None
    _check(lib().sd_tune(L, layout, path, _stream(hip_stream)))


def sd_tuned_choice(L: int, layout: int):
    """(mode, width, blocks, threads) that sd_run uses for (L, layout)."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().sd_tuned_choice(L, layout, *[ctypes.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


def sd_debug_fastdiv(n: int, d: int) -> int:
    return int(lib().sd_debug_fastdiv(n, d))


# ---------------------------------------------------------------------------
# Device memory helpers (plumbing: shapes and dtypes of lattice tensors).
# ---------------------------------------------------------------------------
def new_lattice(L: int, layout: int, device="cuda") -> torch.Tensor:
    """An uninitialised lattice tensor: int8 [L, L] for SD_I8, int64 [L, L/64]
    for SD_P64 (flat [L*L/64] when L % 64 != 0: rows do not start on a word),
    int32 [L, L/32] for SD_P32 (the packed bytes are the same)."""
    nbytes = sd_lattice_bytes(L, layout)
    if nbytes == 0:
        raise ValueError(f"unsupported lattice L={L} layout={layout}")
    if layout == SD_I8:
        return torch.empty((L, L), dtype=torch.int8, device=device)
    if layout == SD_P64:
        if L % 64:
            return torch.empty((L * L // 64,), dtype=torch.int64, device=device)
        return torch.empty((L, L // 64), dtype=torch.int64, device=device)
    return torch.empty((L, L // 32), dtype=torch.int32, device=device)
