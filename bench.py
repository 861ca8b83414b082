"""Benchmark of the shaken-dynamics hot path on one MI355X.

Headline (`value`): spin updates per ns of one chain on a 16384 x 16384 torus,
bit-packed 64 spins per word, random start, J = q = 0.5, observables (M, A, B)
recorded every 10 steps.  One step = two half-steps = 2 L^2 spin updates.
W untimed warm-up steps are followed by exactly K timed steps.

Also reported on the same JSON line:
  roofline      - the half-step kernel's algorithmic HBM rate against the 8 TB/s
                  peak (the 70% target), and the VALU roofline that binds it
  cpu_baseline  - the CPU oracle on a bounded sample of the same workload: one
                  pinned thread, and (all_cores) one chain per host core at
                  once; the GPU's lattices after the same steps are compared
                  with the oracle's
  int8_sweep    - 1024^2 int8 lattices at q = J in {0.2, ..., 1.0}, 10^4 steps
                  each, (M, A, B) every step, D(r <= 512) every 100 steps
  batched_scan  - 4096 chains, (q, J) on a 64 x 64 grid, L in {128, 256, 512},
                  5000 steps, (M, A, B) every step: one hipGraph launch vs the
                  same chains run one sd_run each (timed on a sample)
  loglik        - 256 trajectories of 256^2 lattices, 2000 steps at
                  (J, q) = (0.45, 0.7): bandwidth of the 12-count and the
                  paired-statistics kernels, FP32 gradient error against FP64
                  and the gradient ascent from (0.2, 0.2)
  replicas      - 64 chains sharing one stream, one bit each, on 4096^2 at
                  (q, J) = (1, 1.5 k / 63): spin updates/ns over the chains

Other modes (one JSON object each): --critical-scan, --coalescence,
--propp-wilson, --table1, --replicas, --traffic-from.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin updates/ns (1 GPU, L=16384 packed) + batched-scan chain-steps/s vs plain"

# MI355X unit counts used for the ALU roofline: 256 CUs x 4 SIMDs x 16 lanes at
# 2.4 GHz issue 39.32e12 32-bit VALU lane operations per second.
N_SIMD = 256 * 4
CLOCK_HZ = 2.4e9
VALU_PEAK_OPS = N_SIMD * 16 * CLOCK_HZ
HBM_PEAK_GBS = 8000.0
# Algorithmic VALU operations per spin update of the half-step:
# Philox4x32-10 work of the stream contract, 4 calls per 64 sites plus one tail
# call per undecided site (1/256 of them), 10 rounds of 2 multiplies + 2
# three-way XORs each, and the bit-sliced comparison, 8 planes x (1 select +
# 2 logic ops) per 32 sites.
PHILOX_CALLS_PER_SITE = 4.0 / 64.0 + 1.0 / 256.0
OPS_PER_SPIN_UPDATE = PHILOX_CALLS_PER_SITE * 10 * 4 + 8 * 3 / 32.0
# Algorithmic HBM bytes per spin update of a packed half-step: the site's bit
# of the source lattice read and its new bit written (neighbour words are
# re-reads served by the caches).
ALG_BYTES_PER_SPIN_UPDATE = 0.25


# Sources whose content determines the half-step kernel; a traffic figure from
# hardware counters is reported only while their hash matches the one recorded
# with the counters.
KERNEL_SOURCES = ["paper_1908_07341_amd/csrc/k_update.hip", "paper_1908_07341_amd/csrc/sd_device.hpp",
                  "paper_1908_07341_amd/csrc/sd_kernels.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_half_step_L16384_traffic.json")


def kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """(HBM bytes per half-step launch, kernel it was measured on, VALU wave
    instructions per launch) from the committed counter record, or Nones when
    there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, None, None
    if rec.get("kernel_sha256") != kernel_hash():
        return None, None, None
    return rec.get("bytes_per_launch"), rec.get("kernel"), rec.get("valu_insts_per_launch")


def traffic_from_counters(fetch_csv: str, write_csv: str, sq_csv: str | None = None,
                          copy_bytes: int = 512 * 1024 * 1024) -> dict:
    """HBM bytes per launch of the half-step kernels from two rocprofv3 --pmc
    runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of the --calibrate-copy
    bench.  Each counter is scaled by the factor that maps its reading for the
    device copy of copy_bytes to the bytes that copy moves.  With the SQ run's
    CSV, also the VALU wave instructions per launch (SQ_INSTS_VALU)."""
    import csv

    def per_kernel(path, counter):
        vals, copy = {}, None
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter:
                    continue
                name, v = row["Kernel_Name"], float(row["Counter_Value"])
                if name == "__amd_rocclr_copyBuffer" and (copy is None or v > copy):
                    copy = v
                elif "k_half_step" in name:
                    vals.setdefault(name, []).append(v)
        return {k: sum(v) / len(v) for k, v in vals.items()}, copy

    fetch, fetch_copy = per_kernel(fetch_csv, "FETCH_SIZE")
    write, write_copy = per_kernel(write_csv, "WRITE_SIZE")
    f_fac = copy_bytes / (fetch_copy * 1024.0)
    w_fac = copy_bytes / (write_copy * 1024.0)
    kernels = {}
    for k in fetch:
        if k in write:
            kernels[k] = {"fetch_kib": fetch[k], "write_kib": write[k],
                          "bytes": f_fac * fetch[k] * 1024.0 + w_fac * write[k] * 1024.0}
    # the plain half-step A kernel (no observables) stands for the launch:
    # template arguments <layout, half-step, paired, complemented, observables>
    def plain_a(name):
        if "k_half_step<" not in name:
            return False
        args = [a.strip() for a in name.split("<", 1)[1].split(">", 1)[0].split(",")]
        return len(args) == 5 and args[1] == "0" and args[4] == "false"

    main = min((k for k in kernels if plain_a(k)), key=lambda k: kernels[k]["bytes"], default=None)
    valu = None
    if sq_csv and main:
        sums = {}
        with open(sq_csv) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] == "SQ_INSTS_VALU" and row["Kernel_Name"] == main:
                    sums[row["Dispatch_Id"]] = sums.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
        valu = sum(sums.values()) / len(sums) if sums else None
    return {"kernel_sha256": kernel_hash(), "kernel": main,
            "bytes_per_launch": kernels[main]["bytes"] if main else None, "valu_insts_per_launch": valu,
            "fetch_factor": f_fac, "write_factor": w_fac, "copy_bytes": copy_bytes, "kernels": kernels}


def calibrate_copy(torch, mib: int = 512) -> None:
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiling run."""
    n = mib * 1024 * 1024
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {n} bytes")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--L", type=int, default=16384)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-scan leg")
    p.add_argument("--no-loglik", action="store_true", help="skip the log-likelihood leg")
    p.add_argument("--no-replicas", action="store_true", help="skip the replica-coded chains leg")
    p.add_argument("--no-c2", action="store_true", help="skip the 1024^2 int8 sweep leg")
    p.add_argument("--batch-steps", type=int, default=5000)
    p.add_argument("--plain-sample", type=int, default=32, help="chains per lattice size timed one sd_run each")
    p.add_argument("--plain-full", action="store_true", help="time all 4096 chains one sd_run each")
    p.add_argument("--cpu-steps", type=int, default=2)
    p.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1908_07341_amd", "tune_cache.json"))
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run one 512 MiB device copy first (counter calibration runs)")
    p.add_argument("--critical-scan", action="store_true",
                   help="only the critical-curve scan of section 3.1 (moments of m on a (q, J) grid)")
    p.add_argument("--scan-grid", type=int, default=80)
    p.add_argument("--scan-L", type=int, default=200)
    p.add_argument("--scan-warm", type=int, default=300000)
    p.add_argument("--scan-rec", type=int, default=300000)
    p.add_argument("--coalescence", action="store_true",
                   help="only the coalescence times of section 3.2 (32x32, monotone coupling)")
    p.add_argument("--replicas", action="store_true",
                   help="only the replica-coded chains (64 chains per word sharing one stream)")
    p.add_argument("--replica-L", type=int, default=4096)
    p.add_argument("--replica-steps", type=int, default=100)
    p.add_argument("--propp-wilson", action="store_true",
                   help="only the coupling-from-the-past samples (32x32, J near the square-lattice critical value)")
    p.add_argument("--table1", action="store_true",
                   help="only the diagonal-correlation comparison with Table 1 (32x32, all (q, J) rows)")
    p.add_argument("--cpu-plan", action="store_true",
                   help="only the oracle on the CPU baseline plan's workloads (C1, a C2 point, 64 C4 chains, "
                        "a C5 sample), one pinned core per job")
    p.add_argument("--traffic-from", nargs="+", metavar="CSV",
                   help="write the half-step counter record from the rocprofv3 counter CSVs of the FETCH_SIZE "
                        "and WRITE_SIZE runs (and optionally the SQ run) and exit")
    return p.parse_args()


def bench_c2(sd, torch, tune_cache, L=1024, n_steps=10000, corr_every=100, rmax=512):
    """The five-point q = J sweep on 1024^2 int8 lattices: random start, 10^4
    steps per point with (M, A, B) every step and D(r <= 512) every 100 steps,
    stream = point index.  The five chains advance together through
    sd_run_many (whole-step launches of up to eight steps for all five, each
    workgroup a band of rows with its halo in LDS, records fused in) and
    their D(r) through one sd_corr_row_many call per measurement; for
    comparison the same sweep with one sd_run per point, on a stream each and
    on a single stream (a 1024^2 half-step alone fills a small part of the
    device, so those are bound by launches)."""
    sd.sd_tune(L, sd.SD_I8, tune_cache)
    points = [0.2, 0.4, 0.6, 0.8, 1.0]
    n_pts = len(points)
    n_blk = n_steps // corr_every
    lat = [(sd.new_lattice(L, sd.SD_I8), sd.new_lattice(L, sd.SD_I8)) for _ in points]
    obs = torch.empty((n_pts, n_steps, 3), dtype=torch.int64, device="cuda")
    obs_blk = torch.empty((n_blk, n_pts, corr_every, 3), dtype=torch.int64, device="cuda")
    D = torch.empty((n_pts, n_blk, rmax + 1), dtype=torch.int64, device="cuda")
    D_blk = torch.empty((n_blk, n_pts, rmax + 1), dtype=torch.int64, device="cuda")
    cur = torch.cuda.current_stream()
    side = [torch.cuda.Stream() for _ in points]
    sigmas, taus = [x for x, _ in lat], [y for _, y in lat]

    def init():
        for a, (sigma, _) in enumerate(lat):
            sd.sd_init(sigma, L, sd.SD_I8, sd.SD_INIT_RANDOM, 0.5, 1, a)
        torch.cuda.synchronize()

    def timed(body):
        init()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        body()
        e1.record(cur)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def many():
        for blk in range(n_blk):
            sd.sd_run_many(sigmas, taus, L, sd.SD_I8, points, points, 1, list(range(n_pts)), corr_every * blk,
                           corr_every, obs_blk[blk], 1)
            sd.sd_corr_row_many(sigmas, L, sd.SD_I8, rmax, D_blk[blk])

    def per_point(streams):
        def body():
            for st in set(streams):
                st.wait_stream(cur)
            for blk in range(n_blk):
                for a, (qj, (sigma, tau)) in enumerate(zip(points, lat)):
                    sd.sd_run(sigma, tau, L, sd.SD_I8, qj, qj, 1, a, corr_every * blk, corr_every,
                              obs[a, corr_every * blk:corr_every * (blk + 1)], 1, hip_stream=streams[a])
                    sd.sd_corr_row(sigma, L, sd.SD_I8, rmax, D[a, blk], hip_stream=streams[a])
            for st in set(streams):
                cur.wait_stream(st)
        return body

    timed(many)   # warm-up: first launches of every kernel
    ms_many = timed(many)
    fin_many = [sigma.clone() for sigma in sigmas]
    obs_many = obs_blk.permute(1, 0, 2, 3).reshape(n_pts, n_steps, 3).clone()
    D_many = D_blk.permute(1, 0, 2).clone()
    ms_one = timed(per_point([cur] * n_pts))
    ms_streams = timed(per_point(side))
    same = all(torch.equal(x, y) for x, y in zip(fin_many, sigmas)) and torch.equal(obs_many, obs) and \
        torch.equal(D_many, D)
    updates = 2.0 * L * L * n_steps * n_pts
    m_last = (obs[:, -1000:, 0].double().abs().mean(dim=1) / (L * L)).cpu().numpy()
    c1 = (D[:, -20:, 1].double().mean(dim=1) / (L * L)).cpu().numpy()
    return {"workload": f"{L}x{L} int8, q = J in {points}, random start, {n_steps} steps per point, "
                        f"(M, A, B) every step, D(r <= {rmax}) every {corr_every} steps",
            "spin_updates_per_ns": updates / (ms_many * 1e6), "seconds": ms_many / 1e3,
            "path": "sd_run_many: the five chains in whole-step launches of up to eight steps; "
                    "their D(r) in one sd_corr_row_many call",
            "hbm_algorithmic_GBps": 2.0 * updates / (ms_many * 1e-3) / 1e9,
            "spin_updates_per_ns_sd_run_5_streams": updates / (ms_streams * 1e6),
            "spin_updates_per_ns_sd_run_one_stream": updates / (ms_one * 1e6),
            "identical_to_sd_run_per_point": bool(same),
            "D0_equals_L2": bool((D[:, :, 0] == L * L).all().item()),
            "abs_m_last_1000": [round(float(x), 4) for x in m_last],
            "C1_row_last_20": [round(float(x), 4) for x in c1]}


PREROLL_S = 0.5   # untimed half-steps on scratch lattices before the timed region


def preroll(sd, torch, L, seconds=PREROLL_S):
    """Untimed work on scratch lattices of the benchmark's size for a fixed
    wall time, so that the timed steps start with the GPU at its working
    clocks whatever K is (a short timed region would otherwise include the
    clock ramp).  The chain that is timed is not touched."""
    a, b = sd.new_lattice(L, sd.SD_P64), sd.new_lattice(L, sd.SD_P64)
    sd.sd_init(a, L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, 2, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        sd.sd_run(a, b, L, sd.SD_P64, 0.5, 0.5, 2, 0, n, 20, None, 0)
        torch.cuda.synchronize()
        n += 20
    return {"seconds": time.perf_counter() - t0, "steps": n}


LAUNCH_REPS = 250   # steps timed without observables for the per-launch duration


def bench_single(sd, torch, L, K, W):
    J = q = 0.5
    obs_every = 10
    sigma = sd.new_lattice(L, sd.SD_P64)
    tau = sd.new_lattice(L, sd.SD_P64)
    sd.sd_init(sigma, L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, 1, 0)
    if W:
        sd.sd_run(sigma, tau, L, sd.SD_P64, J, q, 1, 0, 0, W, None, 0)
    obs = torch.zeros((max(K // obs_every, 1), 3), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    pre = preroll(sd, torch, L)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sd.sd_run(sigma, tau, L, sd.SD_P64, J, q, 1, 0, W, K, obs, obs_every)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    m = obs[-1, 0].item() / (L * L)
    # per-launch duration of the half-step kernel: LAUNCH_REPS further steps
    # without observables (only the two half-step kernels run), timed with HIP
    # events on the stream they are launched on
    e2 = torch.cuda.Event(enable_timing=True)
    e3 = torch.cuda.Event(enable_timing=True)
    e2.record(stream)
    sd.sd_run(sigma, tau, L, sd.SD_P64, J, q, 1, 0, W + K, LAUNCH_REPS, None, 0)
    e3.record(stream)
    torch.cuda.synchronize()
    launch_ms = e2.elapsed_time(e3) / (2 * LAUNCH_REPS)
    return dict(wall_s=wall, event_ms=ev_ms, launch_ms=launch_ms, m_final=m, preroll=pre)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_cpu(sd, torch, L, n_steps):
    """The oracle on the first n_steps of the headline chain (same start, seed
    and stream), on one host core (the thread pinned to the first CPU it may
    use), and the GPU's lattices after the same steps compared with the
    oracle's, byte for byte."""
    from oracle import oracle as orc
    orc.build(force=False)
    cores = sorted(os.sched_getaffinity(0))
    s0 = orc.init(L, orc.INIT_RANDOM, 0.5, 1, 0)
    os.sched_setaffinity(0, {cores[0]})
    try:
        t0 = time.perf_counter()
        ref_s, ref_t, _ = orc.run(s0, 0.5, 0.5, 1, 0, 0, n_steps)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, set(cores))
    del s0
    sigma, tau = sd.new_lattice(L, sd.SD_P64), sd.new_lattice(L, sd.SD_P64)
    sd.sd_init(sigma, L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, 1, 0)
    sd.sd_run(sigma, tau, L, sd.SD_P64, 0.5, 0.5, 1, 0, 0, n_steps, None, 0)
    torch.cuda.synchronize()
    from paper_1908_07341_amd import inputs
    same = (np.array_equal(sigma.view(torch.uint8).view(-1).cpu().numpy(), inputs.pack_bits(ref_s)) and
            np.array_equal(tau.view(torch.uint8).view(-1).cpu().numpy(), inputs.pack_bits(ref_t)))
    del ref_s, ref_t
    ups = 2.0 * L * L * n_steps / dt
    return {"value": ups / 1e9, "unit": "spin updates/ns", "cores": 1, "kind": "oracle",
            "sample": f"{n_steps} full step(s) of the {L}x{L} chain (J=q=0.5, random start, seed 1, stream 0) on "
                      f"one host core (thread pinned to CPU {cores[0]}) in {dt:.1f} s",
            "seconds": dt, "cpu_model": cpu_model(), "host_cpus": len(cores),
            "gpu_lattices_bit_identical": bool(same),
            "all_cores": bench_cpu_all_cores(L, n_steps)}


def bench_cpu_all_cores(L, n_steps, max_cores=16):
    """The same oracle step on every host core at once: independent chains
    (streams 0..n-1), one per thread; the oracle's C loop runs without the
    interpreter lock, so the threads run in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as orc
    n = max(1, min(len(os.sched_getaffinity(0)), max_cores))
    starts = [orc.init(L, orc.INIT_RANDOM, 0.5, 1, a) for a in range(n)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=n) as ex:
        list(ex.map(lambda a: orc.run(starts[a], 0.5, 0.5, 1, a, 0, n_steps)[2], range(n)))
    dt = time.perf_counter() - t0
    del starts
    ups = 2.0 * L * L * n_steps * n / dt
    return {"value": ups / 1e9, "unit": "spin updates/ns", "cores": n,
            "sample": f"{n} independent {L}x{L} chains (streams 0..{n - 1}), {n_steps} full step(s) each, "
                      f"one thread per core, in {dt:.1f} s"}


def bench_cpu_plan(n_c5=8):
    """The oracle on the workloads of the CPU baseline plan, each job on a
    host core of its own (the thread pinned with sched_setaffinity), all jobs
    at once: C1 in full (64^2 all +1, J=0.4, q=0.6, 10^4 steps, records every
    step); one C2 point in full (1024^2, q=J=0.6, 10^4 steps, records every
    step, D(r <= 512) every 100); 64 chains of the C4 scan (all three sizes,
    5000 steps, records every step), spread over the remaining cores; and
    n_c5 trajectories of the C5 set in full (256^2, 2000 steps: the chain
    and the 12 counts of its transitions).  No GPU work."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as orc
    from paper_1908_07341_amd import inputs
    orc.build(force=False)
    cores = sorted(os.sched_getaffinity(0))[:16]   # at most the CPU share of one GPU
    if len(cores) < 4:
        raise SystemExit("--cpu-plan needs at least 4 host cores")

    def pinned(core, fn, name):
        def run():
            os.sched_setaffinity(0, {core})
            t0 = time.perf_counter()
            out = fn()
            log(f"[cpu-plan] {name} done on CPU {core} in {time.perf_counter() - t0:.1f} s")
            return time.perf_counter() - t0, out
        return run

    def c1():
        s0 = np.ones((64, 64), np.int8)
        return orc.run(s0, 0.4, 0.6, 1, 0, 0, 10000, obs_every=1)[2].shape[0]

    def c2():
        L, n_steps, every = 1024, 10000, 100
        sig = orc.init(L, orc.INIT_RANDOM, 0.5, 1, 2)
        tau = None
        t0 = time.perf_counter()
        for blk in range(n_steps // every):
            sig, tau, _ = orc.run(sig, 0.6, 0.6, 1, 2, every * blk, every, obs_every=1, tau=tau)
            orc.corr_row(sig, 512)
            if (blk + 1) % 10 == 0:
                log(f"[cpu-plan] C2: {every * (blk + 1)} of {n_steps} steps in {time.perf_counter() - t0:.0f} s")
        return n_steps

    qv, Jv, Lv = inputs.scan_table()
    rng = np.random.default_rng(5)
    chains = []
    for size in (128, 256, 512):
        chains += rng.choice(np.flatnonzero(Lv == size), size=21 if size != 512 else 22, replace=False).tolist()

    def c4_chain(c):
        Lc = int(Lv[c])
        s0 = orc.init(Lc, orc.INIT_RANDOM, 0.5, 1, c)
        orc.run(s0, float(Jv[c]), float(qv[c]), 1, c, 0, 5000, obs_every=1)
        return 2.0 * Lc * Lc * 5000

    def c5_one(a):
        L, k = 256, 2000
        X = orc.trajectory(orc.init(L, orc.INIT_RANDOM, 0.5, 1, a), 0.45, 0.7, 1, a, 0, k)
        orc.loglik_counts(X[None])
        return 2 * k * L * L

    jobs = [("C1", cores[0], c1), ("C2", cores[1], c2)]
    c5_cores = cores[2:3]
    c4_cores = cores[3:]
    results = {}
    with ThreadPoolExecutor(max_workers=len(cores)) as ex:
        futs = {name: ex.submit(pinned(core, fn, name)) for name, core, fn in jobs}

        def c4_worker(core, mine):
            os.sched_setaffinity(0, {core})
            t0 = time.perf_counter()
            ups = sum(c4_chain(c) for c in mine)
            log(f"[cpu-plan] {len(mine)} C4 chains done on CPU {core} in {time.perf_counter() - t0:.1f} s")
            return time.perf_counter() - t0, ups

        def c5_worker(core):
            os.sched_setaffinity(0, {core})
            t0 = time.perf_counter()
            n = sum(c5_one(a) for a in range(n_c5))
            log(f"[cpu-plan] {n_c5} C5 trajectories done on CPU {core} in {time.perf_counter() - t0:.1f} s")
            return time.perf_counter() - t0, n

        f4 = [ex.submit(c4_worker, core, chains[i::len(c4_cores)]) for i, core in enumerate(c4_cores)]
        f5 = ex.submit(c5_worker, c5_cores[0])
        dt1, n1 = futs["C1"].result()
        dt2, n2 = futs["C2"].result()
        r4 = [f.result() for f in f4]
        dt5, n5 = f5.result()
    ups4 = sum(u for _, u in r4)
    core_s4 = sum(t for t, _ in r4)
    results["C1"] = {"what": "64x64 all +1, J=0.4, q=0.6, 10^4 steps, (M,A,B) every step, one core",
                     "seconds": dt1, "spin_updates_per_ns": 2.0 * 64 * 64 * 10000 / dt1 / 1e9}
    results["C2_one_point"] = {"what": "1024x1024 random start, q=J=0.6, 10^4 steps, (M,A,B) every step, "
                                       "D(r<=512) every 100 steps, one core",
                               "seconds": dt2, "spin_updates_per_ns": 2.0 * 1024 * 1024 * 10000 / dt2 / 1e9}
    results["C4_64_chains"] = {"what": f"{len(chains)} chains of the scan (21 of 128^2, 21 of 256^2, 22 of 512^2), "
                                       f"5000 steps, (M,A,B) every step, on {len(c4_cores)} cores",
                               "wall_seconds": max(t for t, _ in r4), "core_seconds": core_s4,
                               "spin_updates_per_ns_per_core": ups4 / core_s4 / 1e9,
                               "chain_steps_per_s_per_core": len(chains) * 5000 / core_s4}
    results["C5_sample"] = {"what": f"{n_c5} trajectories of 256^2, 2000 steps at (0.45, 0.7): chain and "
                                    f"counts of every transition, one core",
                            "seconds": dt5, "transitions_per_ns": n5 / dt5 / 1e9,
                            "full_set_seconds_estimated": dt5 * 256 / n_c5}
    return {"cpu_model": cpu_model(), "host_cpus": len(cores), "kind": "oracle", "jobs": results}


def bench_batched(sd, torch, inputs, K, plain_sample, tune_cache, plain_full=False):
    """The (q, J) scan as one hipGraph launch of the batch plan, its load
    balance (from a direct run with per-bucket times), and the same chains run
    one sd_run each ("plain launches"), back to back with one synchronisation
    at the end, on one stream and on four: all 4096 chains with plain_full,
    else plain_sample chains per lattice size with the time scaled to the
    whole scan per size."""
    qv, Jv, Lv = inputs.scan_table()
    n = len(qv)
    streams = np.arange(n, dtype=np.uint32)
    seed = 1
    t_plan = time.perf_counter()
    plan = sd.sd_batch_plan_create(Jv, qv, Lv, streams, layout=sd.SD_P64, seed=seed, k_steps=K, obs_every=1,
                                   tune_cache_path=tune_cache)
    t_plan = time.perf_counter() - t_plan
    shapes = []
    b = 0
    while True:
        try:
            shapes.append(sd.sd_batch_launch_shape(plan, b))
        except sd.ShakenError:
            break
        b += 1
    lat = torch.empty(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
    traces = torch.empty(sd.sd_batch_trace_len(plan), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan, lat, sd.SD_INIT_RANDOM, 0.5)
    start = lat.clone()
    torch.cuda.synchronize()
    # first launch captures and instantiates the graph (untimed), the second is timed
    sd.sd_batch_run(plan, lat, traces, 0)
    torch.cuda.synchronize()
    lat.copy_(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sd.sd_batch_run(plan, lat, traces, 0)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    batch_rate = n * K / t_batch
    # load balance of the timed graph run: each bucket's first start and last
    # end, stamped on the device by its own workgroups
    times = [sd.sd_batch_bucket_times(plan, i) for i in range(len(shapes))]
    span = max(e for _, e in times)
    busy = sum(e - s_ for s_, e in times)
    # the same run as plain launches (no graph) must give the same chains
    graph_lat, graph_tr = lat.clone(), traces.clone()
    lat.copy_(start)
    sd.sd_batch_run_direct(plan, lat, traces, 0)
    torch.cuda.synchronize()
    # Buckets steal from later buckets' queues, so a bucket whose grid becomes
    # resident only when an earlier one ends can find its queue empty: it
    # then runs for microseconds and did none of the scan's work.  Such
    # launches are left out of the working-bucket efficiency.
    working = [(s_, e) for s_, e in times if e - s_ > 0.01 * span]
    busy_w = sum(e - s_ for s_, e in working)
    # the buckets share their queues, so the balance that matters is how
    # close together they end (a grid that becomes resident late has had
    # its chains taken by the others meanwhile)
    end_spread = (max(e for _, e in working) - min(e for _, e in working)) / span
    same_direct = bool(torch.equal(lat, graph_lat) and torch.equal(traces, graph_tr))
    # plain: one sd_run per chain (sd_run's launch choice tuned for each size)
    for size in sorted(set(Lv.tolist())):
        sd.sd_tune(int(size), sd.SD_P64, tune_cache)
    sizes = sorted(set(Lv.tolist()))
    if plain_full:
        sample = list(range(n))
    else:
        rng = np.random.default_rng(0)
        sample = []
        for size in sizes:
            idx = np.flatnonzero(Lv == size)
            sample += rng.choice(idx, size=min(plain_sample, len(idx)), replace=False).tolist()
    bufs = []
    for c in sample:
        Lc = int(Lv[c])
        nb = sd.sd_lattice_bytes(Lc, sd.SD_P64)
        so = sd.sd_batch_chain_offset(plan, c, 0)
        bufs.append((c, Lc, start[so:so + nb].clone().view(torch.int64),
                     torch.empty(nb // 8, dtype=torch.int64, device="cuda"),
                     torch.empty((K, 3), dtype=torch.int64, device="cuda")))
    cur = torch.cuda.current_stream()
    side = [torch.cuda.Stream() for _ in range(4)]

    def plain(n_streams):
        for c, Lc, sig, tau, obs in bufs:
            so = sd.sd_batch_chain_offset(plan, c, 0)
            sig.view(torch.uint8).copy_(start[so:so + sig.numel() * 8])
        torch.cuda.synchronize()
        sts = [cur] if n_streams == 1 else side[:n_streams]
        for st in sts:
            st.wait_stream(cur)
        t_start = time.perf_counter()
        for i, (c, Lc, sig, tau, obs) in enumerate(bufs):
            sd.sd_run(sig, tau, Lc, sd.SD_P64, float(Jv[c]), float(qv[c]), seed, int(streams[c]), 0, K, obs, 1,
                      hip_stream=sts[i % len(sts)])
            if plain_full and (i + 1) % 256 == 0:
                log(f"[bench] plain launches on {n_streams} stream(s): {i + 1} of {len(bufs)} chains enqueued "
                    f"in {time.perf_counter() - t_start:.0f} s")
        for st in sts:
            cur.wait_stream(st)
        torch.cuda.synchronize()
        return time.perf_counter() - t_start

    t1 = plain(1)
    t4 = plain(4)
    identical = True
    tr = traces.view(n, K * 3)
    for c, Lc, sig, tau, obs in bufs:
        so = sd.sd_batch_chain_offset(plan, c, 0)
        identical &= bool(torch.equal(sig.view(torch.uint8), lat[so:so + sig.numel() * 8]))
        identical &= bool(torch.equal(obs.view(-1), tr[c]))
    # the sample's time scaled to the whole scan by lattice area
    total_cost = float((Lv.astype(np.float64) ** 2).sum())
    sample_cost = float(sum(Lc * Lc for _, Lc, _, _, _ in bufs))
    scale = total_cost / sample_cost
    plain1, plain4 = t1 * scale, t4 * scale
    plan.close()
    return {
        "workload": f"{n} chains, q in [0,2] x J in [0,1.5] on a 64x64 grid, L from {{128,256,512}} "
                    f"(numpy default_rng(1)), packed-64, random starts, {K} steps, (M,A,B) every step",
        "chain_steps_per_s": batch_rate, "seconds": t_batch,
        "spin_updates_per_ns": 2.0 * total_cost * K / t_batch / 1e9,
        "load_balance": {"source": "the timed graph run: each bucket's first start and last end on the device "
                                   "wall clock",
                         "bucket_start_end_ms": [[round(s_, 2), round(e, 2)] for s_, e in times],
                         "span_ms": span, "end_spread": end_spread,
                         "efficiency": busy_w / (len(working) * span),
                         "working_buckets": len(working), "efficiency_all_launches": busy / (len(times) * span),
                         "direct_run_identical_to_graph": same_direct},
        "plain": {"chains_run": len(bufs), "all_chains": bool(plain_full),
                  "seconds_one_stream": t1, "seconds_four_streams": t4,
                  "scan_seconds_one_stream": plain1, "scan_seconds_four_streams": plain4,
                  "chain_steps_per_s_one_stream": n * K / plain1, "chain_steps_per_s_four_streams": n * K / plain4,
                  "scaled_by_area": not plain_full, "bit_identical": identical},
        "speedup_vs_plain_one_stream": plain1 / t_batch, "speedup_vs_plain_four_streams": plain4 / t_batch,
        "plan_seconds": t_plan, "launch_shapes": [list(s_) for s_ in shapes],
        "plain_run_choices": {int(z): list(sd.sd_tuned_choice(int(z), sd.SD_P64)) for z in sizes},
    }


LL_PREROLL_S = 1.0   # untimed launches of each statistics kernel before it is timed


def bench_loglik(sd, torch, n_traj=256, L=256, k=2000):
    from paper_1908_07341_amd import autograd as AG
    J, q = 0.45, 0.7
    nb = sd.sd_lattice_bytes(L, sd.SD_P64)
    n_lat = 2 * k + 1
    traj = torch.empty((n_traj, n_lat, nb // 8), dtype=torch.int64, device="cuda")
    starts = torch.empty((n_traj, nb // 8), dtype=torch.int64, device="cuda")
    for a in range(n_traj):
        sd.sd_init(starts[a], L, sd.SD_P64, sd.SD_INIT_RANDOM, 0.5, 1, a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sd.sd_trajectories(starts, traj, n_traj, L, sd.SD_P64, J, q, 1, 0, 0, k)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    counts = torch.empty(12, dtype=torch.int64, device="cuda")
    stats = torch.empty(6, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn, out, reps=10):
        # untimed launches of the same kernel for a fixed wall time first, so
        # that the timed ones run at the working clocks
        t_pre = time.perf_counter()
        while time.perf_counter() - t_pre < LL_PREROLL_S:
            fn(traj, n_traj, n_lat, L, out)
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn(traj, n_traj, n_lat, L, out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = timed(sd.sd_loglik_counts, counts)
    ms_st = timed(sd.sd_loglik_stats, stats)
    gbs = traj.numel() * 8 / (ms * 1e-3) / 1e9
    gbs_st = traj.numel() * 8 / (ms_st * 1e-3) / 1e9
    ch = counts.cpu().numpy()
    sh = stats.cpu().numpy()
    pair_map = [ch[2 * j] + ch[2 * j + 1] + ch[2 * (5 - j)] + ch[2 * (5 - j) + 1] for j in range(3)]
    pair_map += [ch[2 * j + 1] + ch[2 * (5 - j)] for j in range(3)]
    stats_consistent = bool(np.array_equal(sh, np.array(pair_map)))
    # gradient at the ascent start, against FP64 from the same integer counts
    Jq = torch.tensor([0.2, 0.2], dtype=torch.float32, device="cuda", requires_grad=True)
    ll = AG.loglik(Jq, stats)
    (g,) = torch.autograd.grad(ll, Jq)
    g64 = _fp64_grad(ch, 0.2, 0.2)
    rel = float(np.max(np.abs(g.cpu().numpy().astype(np.float64) - g64) / np.abs(g64)))
    # gradient ascent on LL / N from (0.2, 0.2), on the paired statistics
    N = float(ch.sum())
    x = torch.tensor([0.2, 0.2], dtype=torch.float32, device="cuda", requires_grad=True)
    for _ in range(300):
        (gg,) = torch.autograd.grad(AG.loglik(x, stats) / N, x)
        with torch.no_grad():
            x += 0.5 * gg
    est = x.detach().cpu().numpy().tolist()
    mle, se = _fp64_newton(ch)
    within = bool(all(abs(e - t) < 3 * s_ for e, t, s_ in zip(est, (J, q), se)))
    del traj
    return {"workload": f"{n_traj} trajectories of {L}x{L}, {k} steps at (J,q)=({J},{q}), random starts",
            "transitions": int(N), "trajectory_GB": n_traj * n_lat * nb / 1e9, "generate_seconds": t_gen,
            "timing": f"{LL_PREROLL_S} s of untimed launches of each kernel, then 10 launches timed with HIP events",
            "counts_ms": ms, "counts_GBps": gbs, "counts_hbm_frac": gbs / HBM_PEAK_GBS,
            "stats_ms": ms_st, "stats_GBps": gbs_st, "stats_hbm_frac": gbs_st / HBM_PEAK_GBS,
            "stats_equal_pair_map_of_counts": stats_consistent,
            "grad_rel_err_vs_fp64_at_start": rel, "ascent_estimate": est,
            "fp64_mle": mle.tolist(), "standard_errors": se.tolist(), "ascent_within_3_se": within}


def critical_J(q):
    """J_c(q) of eq. (12): the critical curve of the shaken dynamics."""
    t = np.tanh(q)
    return np.arctanh(np.sqrt(t * t + 1.0) - t)


def bench_critical_scan(sd, torch, n_grid, L, warm, rec, tune_cache):
    """Section 3.1: chains on an n_grid x n_grid grid of (q, J) in (0, 2)^2 (cell
    midpoints), L x L torus from all -1, `warm` steps, then the mean and the
    variance of m over `rec` steps (per-chain moments kept on the device)."""
    vals = 2.0 * (np.arange(n_grid) + 0.5) / n_grid
    qg, Jg = np.meshgrid(vals, vals, indexing="ij")
    qv, Jv = qg.reshape(-1), Jg.reshape(-1)
    n = len(qv)
    Lv = np.full(n, L)
    streams = np.arange(n, dtype=np.uint32)
    t0 = time.perf_counter()
    plan_w = sd.sd_batch_plan_create(Jv, qv, Lv, streams, seed=1, k_steps=warm, obs_every=0,
                                     tune_cache_path=tune_cache)
    plan_r = sd.sd_batch_plan_create(Jv, qv, Lv, streams, seed=1, k_steps=rec, obs_every=1,
                                     flags=sd.SD_FLAG_MOMENTS, tune_cache_path=tune_cache)
    t_plan = time.perf_counter() - t0
    lat = torch.zeros(sd.sd_batch_lattice_bytes(plan_r), dtype=torch.uint8, device="cuda")
    mom = torch.zeros(sd.sd_batch_trace_len(plan_r), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan_w, lat, sd.SD_INIT_DOWN)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sd.sd_batch_run(plan_w, lat, None, 0)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    log(f"[bench] scan warm-up {warm} steps in {t_warm:.1f} s")
    t0 = time.perf_counter()
    sd.sd_batch_run(plan_r, lat, mom, warm)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    plan_w.close()
    plan_r.close()
    S = mom.cpu().numpy().reshape(n, 5).astype(np.float64)
    N = float(L * L)
    mean_m = S[:, 0] / (rec * N)
    var_m = S[:, 1] / (rec * N * N) - mean_m ** 2
    mean_abs = S[:, 2] / (rec * N)
    var_g = var_m.reshape(n_grid, n_grid)
    per_q = []
    for a in range(n_grid):
        b = int(np.argmax(var_g[a]))
        per_q.append({"q": round(float(vals[a]), 4), "J_at_max_var": round(float(vals[b]), 4),
                      "J_c": round(float(critical_J(vals[a])), 4), "max_var": round(float(var_g[a, b]), 4)})
    dev = np.array([abs(r["J_at_max_var"] - r["J_c"]) for r in per_q])
    big = var_m >= 0.03
    dist = np.abs(Jv[big] - critical_J(qv[big]))
    updates = 2.0 * n * N * (warm + rec)
    return {"workload": f"{n} chains: (q, J) on a {n_grid}x{n_grid} grid of cell midpoints in (0,2)^2, "
                        f"{L}x{L} torus from all -1, {warm} warm-up + {rec} recorded steps",
            "seconds_warm": t_warm, "seconds_record": t_rec, "plan_seconds": t_plan,
            "spin_updates_per_ns": updates / ((t_warm + t_rec) * 1e9),
            "grid_step": 2.0 / n_grid,
            "max_var_J_minus_Jc": {"mean": float(dev.mean()), "max": float(dev.max()),
                                   "within_one_grid_step": int((dev <= 2.0 / n_grid + 1e-9).sum())},
            "points_var_ge_0.03": int(big.sum()),
            "their_J_minus_Jc": {"mean": float(dist.mean()) if big.any() else None,
                                 "max": float(dist.max()) if big.any() else None},
            "per_q": per_q,
            "mean_abs_m_far_below_curve": float(mean_abs[Jv < critical_J(qv) - 0.2].mean()),
            "mean_abs_m_far_above_curve": float(mean_abs[Jv > critical_J(qv) + 0.2].mean())}


def coalescence_times(sd, torch, J, q, L, n_pairs, seed=1, chunk=1000, max_steps=200000, stream0=0):
    """Coalescence times of the monotone coupling (section 3.2): pair p is a
    chain from all +1 and one from all -1 sharing stream stream0 + p, so both
    draw the same uniforms.  The coupling keeps sigma_top >= sigma_bottom site
    by site, hence the two lattices are equal exactly when their
    magnetisations are: T_p = first step with M_top = M_bottom (-1 if none
    within max_steps).  Runs as one batch plan, chunk steps per launch."""
    n = 2 * n_pairs
    streams = np.repeat(np.arange(stream0, stream0 + n_pairs, dtype=np.uint32), 2)
    plan = sd.sd_batch_plan_create(np.full(n, J), np.full(n, q), np.full(n, L), streams, seed=seed, k_steps=chunk,
                                   obs_every=1)
    lat = torch.zeros(sd.sd_batch_lattice_bytes(plan), dtype=torch.uint8, device="cuda")
    tr = torch.zeros(sd.sd_batch_trace_len(plan), dtype=torch.int64, device="cuda")
    sd.sd_batch_init(plan, lat, sd.SD_INIT_DOWN)
    nb = sd.sd_lattice_bytes(L, sd.SD_P64)
    for p_ in range(n_pairs):
        off = sd.sd_batch_chain_offset(plan, 2 * p_, 0)
        lat[off:off + nb].fill_(0xFF)
    T = torch.full((n_pairs,), -1, dtype=torch.int64, device="cuda")
    steps = torch.arange(1, chunk + 1, device="cuda")
    step = 0
    while step < max_steps:
        sd.sd_batch_run_direct(plan, lat, tr, step)
        M = tr.view(n, chunk, 3)[:, :, 0]
        eq = M[0::2] == M[1::2]
        first = torch.where(eq, steps, chunk + 1).min(dim=1).values
        newly = (T < 0) & (first <= chunk)
        T = torch.where(newly, step + first, T)
        step += chunk
        if bool((T >= 0).all()):
            break
    plan.close()
    return T.cpu().numpy()


def bench_coalescence(sd, torch, L=32, n_pairs=256):
    """Mean coalescence time on a 32x32 torus for J = q (the isotropic
    honeycomb model whose critical point is J = q = 0.6585) and at points
    just below and above the critical curve J_c(q) of eq. (12)."""
    rows = []
    t0 = time.perf_counter()
    pts = [(x, x) for x in (0.3, 0.4, 0.5, 0.55, 0.6, 0.63, 0.6585, 0.68, 0.7)]
    for qq in (0.2, 1.0, 2.5):
        jc = float(critical_J(qq))
        pts += [(qq, jc - 0.05), (qq, jc), (qq, jc + 0.05)]
    for idx, (q, J) in enumerate(pts):
        T = coalescence_times(sd, torch, J, q, L, n_pairs, seed=1, stream0=1000 * idx)
        done = T[T >= 0]
        rows.append({"q": round(q, 4), "J": round(J, 4), "J_minus_Jc": round(J - float(critical_J(q)), 4),
                     "pairs": n_pairs, "coalesced": int(len(done)),
                     "mean_T": float(done.mean()) if len(done) else None,
                     "median_T": float(np.median(done)) if len(done) else None,
                     "max_T": int(done.max()) if len(done) else None})
        log(f"[bench] coalescence q={q:.4f} J={J:.4f}: {rows[-1]['mean_T']} ({len(done)}/{n_pairs})")
    return {"workload": f"{L}x{L} torus, {n_pairs} coupled pairs per point (all +1 / all -1, shared stream), "
                        f"cap 200000 steps", "rows": rows, "seconds": time.perf_counter() - t0}


def bench_replicas(sd, torch, L, K):
    """64 chains per 64-bit word sharing seed and stream, at the 64 (q, J)
    points of one row of the scan grid (q = 1, J from 0 to 1.5), L x L from
    random starts: spin updates/ns over all chains, with HIP events around the
    timed steps, and the algorithmic HBM rate (one 8-byte word read and one
    written per site and half-step: 0.25 B per spin update)."""
    J = list(1.5 * np.arange(64) / 63)
    q = [1.0] * 64
    nb = sd.sd_replica_lattice_bytes(L)
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    sig = torch.randint(-2 ** 62, 2 ** 62, (nb // 8,), dtype=torch.int64, device="cuda", generator=g)
    tau = torch.empty_like(sig)
    sd.sd_replica_run(sig, tau, L, J, q, 1, 0, 0, 2)   # warm-up
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sd.sd_replica_run(sig, tau, L, J, q, 1, 0, 2, K)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    updates = 2.0 * 64 * L * L * K
    out = torch.empty(192, dtype=torch.int64, device="cuda")
    sd.sd_replica_observe(sig, tau, L, out)
    m = (out.view(64, 3)[:, 0].double() / (L * L)).abs().cpu().numpy()
    rate = updates / (ms * 1e6)
    return {"workload": f"64 chains sharing one stream, {L}x{L}, (q, J) = (1, 1.5 k / 63) for k = 0..63, "
                        f"random start, {K} steps", "spin_updates_per_ns": rate, "ms": ms,
            "half_step_us": ms * 1e3 / (2 * K), "hbm_algorithmic_GBps": rate * 0.25,
            "hbm_frac": rate * 0.25 / HBM_PEAK_GBS, "abs_m_lowest_J": float(m[0]), "abs_m_highest_J": float(m[-1])}


def bench_propp_wilson(sd, torch, L=32, n=512):
    """Exact samples of the stationary law by coupling from the past (the
    Propp-Wilson sampler on the monotone coupling of section 3.2) on a 32x32
    torus at a few (q, J): per point the wall time, the coalescence times and
    the sample means of m and |m|."""
    from paper_1908_07341_amd import inputs
    nb = sd.sd_lattice_bytes(L, sd.SD_P64)
    samples = torch.empty((n, nb), dtype=torch.uint8, device="cuda")
    work = torch.empty(4 * n * nb, dtype=torch.uint8, device="cuda")
    rows = []
    t_all = time.perf_counter()
    for idx, (q, J) in enumerate([(1.0, 0.30), (1.0, 0.38), (2.5, 0.30), (2.5, 0.38), (2.5, 0.42), (4.0, 0.38)]):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = np.array(sd.sd_propp_wilson(samples, work, n, L, J, q, 1, 10000 * idx, 1 << 28, 16, 1 << 24))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        host = samples.cpu().numpy()
        lat = np.stack([inputs.unpack_bits(host[p], L) for p in range(n)]).astype(np.int64)
        m = lat.mean(axis=(1, 2))
        ok = T > 0
        rows.append({"q": q, "J": J, "samples": n, "coalesced": int(ok.sum()), "seconds": dt,
                     "samples_per_s": n / dt, "mean_T": float(T[ok].mean()) if ok.any() else None,
                     "max_T": int(T.max()), "mean_m": float(m[ok].mean()), "mean_abs_m": float(np.abs(m[ok]).mean()),
                     "sd_m": float(m[ok].std())})
        log(f"[bench] propp-wilson q={q} J={J}: {n} samples in {dt:.2f} s, mean T {rows[-1]['mean_T']}")
    return {"workload": f"{L}x{L} torus, {n} samples per point, T from 16 doubling to at most 2^24, "
                        f"time 0 at step index 2^28, seed 1", "rows": rows, "seconds": time.perf_counter() - t_all}


def bench_table1(sd, torch, burn=2000, n_meas=4000, every=5, L=32):
    """Time-averaged diagonal correlations C(l) = D(l) / L^2 on a 32x32 torus at
    every (q, J) row of Table 1 (section 3.3), next to the printed values
    (tests/golden/table1_diagonal_correlations.txt)."""
    ells = [1, 2, 4, 8, 16]
    paper = {}
    with open(os.path.join(ROOT, "tests", "golden", "table1_diagonal_correlations.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            qs, Js, sup, d, *vals = line.split()
            paper.setdefault((float(qs), float(Js)), {"supercritical": sup == "1"})[d] = [float(v) for v in vals]
    layout, lmax = sd.SD_P32, max(ells)
    rows = []
    t0 = time.perf_counter()
    for idx, ((q, J), ref) in enumerate(paper.items()):
        sigma, tau = sd.new_lattice(L, layout), sd.new_lattice(L, layout)
        sd.sd_init(sigma, L, layout, sd.SD_INIT_RANDOM, 0.5, 1, idx)
        sd.sd_run(sigma, tau, L, layout, J, q, 1, idx, 0, burn, None, 0)
        acc = torch.zeros(2 * (lmax + 1), dtype=torch.int64, device="cuda")
        out = torch.empty_like(acc)
        step = burn
        for _ in range(n_meas):
            sd.sd_run(sigma, tau, L, layout, J, q, 1, idx, step, every, None, 0)
            step += every
            sd.sd_corr_diag(sigma, L, layout, lmax, out)
            acc += out
        C = (acc.cpu().numpy().reshape(2, lmax + 1) / (n_meas * L * L))
        ours = {"NW-SE": [round(float(C[1, l]), 3) for l in ells], "SW-NE": [round(float(C[0, l]), 3) for l in ells]}
        rows.append({"q": q, "J": J, "supercritical": ref["supercritical"], "ours": ours,
                     "paper": {"NW-SE": ref["NW-SE"], "SW-NE": ref["SW-NE"]}})
    torch.cuda.synchronize()
    agree = sum((r["ours"]["NW-SE"][0] > r["ours"]["SW-NE"][0]) == (r["paper"]["NW-SE"][0] > r["paper"]["SW-NE"][0])
                for r in rows)
    mad = float(np.mean([abs(a - b) for r in rows for d in ("NW-SE", "SW-NE")
                         for a, b in zip(r["ours"][d], r["paper"][d])]))
    return {"workload": f"{L}x{L} torus, random start, {burn} burn-in steps, {n_meas} measurements every {every} "
                        f"steps, seed 1, stream = row index", "l": ells, "rows": rows,
            "sign_of_NWSE_minus_SWNE_at_l1_agrees": f"{agree}/{len(rows)}", "mean_abs_diff_vs_paper": mad,
            "seconds": time.perf_counter() - t0}


def _fp64_grad(c, J, q, exact=False):
    """FP64 gradient of the LL of the 12 counts at (J, q), rounded to FP32
    first unless exact (the point the FP32 kernels see)."""
    if not exact:
        J, q = float(np.float32(J)), float(np.float32(q))
    gJ = gq = 0.0
    for k in range(3):
        for cp in range(2):
            a, b = 2 * k - 2, 2 * cp - 1
            h = J * a + q * b
            d = float(c[2 * (2 * k + cp) + 1] - c[2 * (2 * k + cp)])
            N = float(c[2 * (2 * k + cp) + 1] + c[2 * (2 * k + cp)])
            gJ += a * (d - N * math.tanh(h))
            gq += b * (d - N * math.tanh(h))
    return np.array([gJ, gq])


def _fp64_hessian(c, J, q):
    H = np.zeros((2, 2))
    for k in range(3):
        for cp in range(2):
            a, b = 2 * k - 2, 2 * cp - 1
            h = J * a + q * b
            n = float(c[2 * (2 * k + cp)] + c[2 * (2 * k + cp) + 1])
            H -= n / math.cosh(h) ** 2 * np.array([[a * a, a * b], [a * b, b * b]])
    return H


def _fp64_newton(c):
    """FP64 maximum of the LL of the 12 counts (Newton from (0.2, 0.2)) and
    its standard errors from the inverse Fisher information."""
    theta = np.array([0.2, 0.2])
    for _ in range(30):
        theta = theta - np.linalg.solve(_fp64_hessian(c, *theta), _fp64_grad(c, *theta, exact=True))
    return theta, np.sqrt(np.diag(np.linalg.inv(-_fp64_hessian(c, *theta))))


def main():
    args = parse()
    if args.traffic_from:
        if len(args.traffic_from) not in (2, 3):
            raise SystemExit("--traffic-from takes FETCH_CSV WRITE_CSV [SQ_CSV]")
        rec = traffic_from_counters(*args.traffic_from)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps({"kernel": rec["kernel"], "bytes_per_launch": rec["bytes_per_launch"]}))
        return
    if args.cpu_plan:
        print(json.dumps({"cpu_plan": bench_cpu_plan()}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the shaken-dynamics path here is "
                                   "built and measured for a single MI355X (a chain would shard by row bands "
                                   "with one halo row exchanged per half-step, batched chains and "
                                   "trajectories by whole chains)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1908_07341_amd as sd
    from paper_1908_07341_amd import inputs
    sd.lib()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.table1:
        print(json.dumps({"table1": bench_table1(sd, torch)}), flush=True)
        return
    if args.coalescence:
        print(json.dumps({"coalescence": bench_coalescence(sd, torch)}), flush=True)
        return
    if args.replicas:
        print(json.dumps({"replicas": bench_replicas(sd, torch, args.replica_L, args.replica_steps)}), flush=True)
        return
    if args.propp_wilson:
        print(json.dumps({"propp_wilson": bench_propp_wilson(sd, torch)}), flush=True)
        return
    if args.critical_scan:
        out = bench_critical_scan(sd, torch, args.scan_grid, args.scan_L, args.scan_warm, args.scan_rec,
                                  args.tune_cache)
        print(json.dumps({"critical_scan": out}), flush=True)
        return
    L, K, W = args.L, args.steps, args.warmup
    if args.calibrate_copy:
        calibrate_copy(torch)
    t0 = time.perf_counter()
    sd.sd_tune(L, sd.SD_P64, args.tune_cache)
    log(f"[bench] sd_tune L={L}: choice {sd.sd_tuned_choice(L, sd.SD_P64)} in {time.perf_counter() - t0:.2f} s")
    log(f"[bench] single chain L={L} K={K} W={W}")
    choice = sd.sd_tuned_choice(L, sd.SD_P64)
    r = bench_single(sd, torch, L, K, W)
    updates = 2.0 * L * L * K
    value = updates / (r["wall_s"] * 1e9)
    log(f"[bench] {value:.1f} spin updates/ns; half-step launch {r['launch_ms']*1e3:.1f} us")
    per_launch_updates = L * L
    launch_s = r["launch_ms"] * 1e-3
    hbm_gbs = ALG_BYTES_PER_SPIN_UPDATE * per_launch_updates / launch_s / 1e9
    alu_achieved = OPS_PER_SPIN_UPDATE * per_launch_updates / launch_s / 1e12
    alu_peak = VALU_PEAK_OPS / 1e12
    traffic, traffic_kernel, valu_per_launch = measured_traffic()
    # the measured instruction stream beside the algorithmic op count: VALU
    # wave instructions per 64 words and the share of the launch they take to
    # issue (4 cycles per wave64 instruction on each of the 1024 SIMDs)
    valu_measured = None
    if valu_per_launch:
        issue_s = valu_per_launch * 4.0 / (N_SIMD * CLOCK_HZ)
        valu_measured = {"valu_insts_per_64_words": valu_per_launch / (per_launch_updates / 64 / 64),
                         "valu_issue_us": issue_s * 1e6, "valu_issue_frac": issue_s / launch_s,
                         "source": "SQ_INSTS_VALU of the committed counter record"}
    blocks = choice[2]
    kernel = {1: "single-workgroup LDS kernel"}.get(
        choice[0], f"k_half_step on {choice[1]}-bit words, {blocks} workgroups of 256 threads")
    out = {
        "metric": METRIC, "value": value, "unit": "spin updates/ns", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": r["wall_s"] * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"single chain {L}x{L} periodic, bit-packed 64 spins/word, random start (p=0.5), "
                               f"J=0.5, q=0.5, observables (M,A,B) every 10 steps",
                   "L": L, "layout": "P64", "J": 0.5, "q": 0.5, "obs_every": 10, "seed": 1},
        # HBM roofline of the half-step kernel (the figure the 70% target is
        # set on) from its algorithmic bytes, and beside it the VALU roofline
        # that actually binds it
        "roofline": {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": traffic, "traffic_kernel": traffic_kernel,
                     "kernel": kernel, "launch_us": r["launch_ms"] * 1e3, "launches_timed": 2 * LAUNCH_REPS,
                     "bytes_per_spin_update": ALG_BYTES_PER_SPIN_UPDATE, "target_frac": 0.70,
                     "binding_resource": "alu",
                     "alu": {"achieved": alu_achieved, "peak": alu_peak, "unit": "T lane-ops/s",
                             "frac": alu_achieved / alu_peak, "ops_per_spin_update": OPS_PER_SPIN_UPDATE,
                             "hbm_frac_at_alu_peak": ALG_BYTES_PER_SPIN_UPDATE * VALU_PEAK_OPS /
                             OPS_PER_SPIN_UPDATE / 1e9 / HBM_PEAK_GBS, "measured": valu_measured},
                     "tuned_choice": list(choice), "preroll": r["preroll"]},
        "m_final": r["m_final"],
    }
    if not args.no_c2:
        log("[bench] 1024^2 int8 sweep")
        out["int8_sweep"] = bench_c2(sd, torch, args.tune_cache)
        log(f"[bench] sweep {out['int8_sweep']['spin_updates_per_ns']:.0f} spin updates/ns")
    if not args.no_batch:
        log(f"[bench] batched scan, {args.batch_steps} steps")
        out["batched_scan"] = bench_batched(sd, torch, inputs, args.batch_steps, args.plain_sample, args.tune_cache,
                                            args.plain_full)
        # how close the three concurrent buckets come to the single large chain, per spin update
        out["batched_scan"]["rate_vs_single_chain"] = out["batched_scan"]["spin_updates_per_ns"] / value
        log(f"[bench] batched {out['batched_scan']['chain_steps_per_s']:.3g} chain-steps/s, "
            f"x{out['batched_scan']['speedup_vs_plain_four_streams']:.1f} vs plain on 4 streams, load balance "
            f"{out['batched_scan']['load_balance']['efficiency']:.3f}, bucket ends within "
            f"{100 * out['batched_scan']['load_balance']['end_spread']:.1f} %")
    if not args.no_loglik:
        log("[bench] log-likelihood")
        out["loglik"] = bench_loglik(sd, torch)
        log(f"[bench] counts {out['loglik']['counts_GBps']:.0f} GB/s, paired stats {out['loglik']['stats_GBps']:.0f} GB/s")
    if not args.no_replicas:
        log("[bench] replica-coded chains")
        out["replicas"] = bench_replicas(sd, torch, args.replica_L, args.replica_steps)
        log(f"[bench] replicas {out['replicas']['spin_updates_per_ns']:.0f} spin updates/ns over 64 chains")
    if not args.no_cpu:
        log(f"[bench] CPU oracle, {args.cpu_steps} step(s) at L={L}")
        out["cpu_baseline"] = bench_cpu(sd, torch, L, args.cpu_steps)
        log(f"[bench] CPU {out['cpu_baseline']['value']:.4f} spin updates/ns")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
