"""Throughput of the fused D2Q9 pseudopotential lattice update on one MI355X.

Workload: four 2048 x 2048 periodic lattices, each a flat liquid slab in the
middle half of the domain (tanh interfaces of width 2, seeded U(+-1e-3) noise)
of the Carnahan-Starling EOS (a=1, b=4, R=1 convention) at reduced
temperatures 0.6, 0.7, 0.8 and 0.9, BGK tau = 1, G = -1, eps = 1.73, sigma = 1.
One bench step advances each of the four lattices by one time step.  The
four lattices form one batch (the library's batch entry points), so one
kernel launch covers all four, and the library takes two time steps per
launch (the two-step pass: read the populations once, compute both steps,
write once); an odd step count ends with one single-step launch.  The
launch shape is fixed per storage mode (SLAB_LAUNCH, the fastest of launch
sweeps of this workload); --launch sets another, --autotune lets the
library's batch autotuner pick one.
--one-by-one gives each lattice launches of its own instead; the default line
carries that rate too (`one_lattice_per_launch`).  Inputs are resident in HBM
before timing.

Before the timed region at least WARMUP_FLOOR_STEPS untimed steps run (more
if --warmup asks for more), and the timed steps are enqueued right behind
them with no host synchronisation in between, so the GPU does not idle into
the timed region; every step, warm-up included, is checked for a sticky
domain error after the timed region.

Output: one JSON line.  `value` is lattice updates per second over the timed
steps (MLUPS).  `roofline` prices the dominant kernel (the batched two-step
pass; the batched single step with --fusion 1) at the algorithmic bytes of a
cell update, one read and one write of its populations (144 B in FP64,
72 / 36 / 44 B in the reduced-precision modes), times the updates one launch
makes (two per cell of the four lattices for the two-step pass), over its
average launch duration timed with HIP events on the library's stream,
against the 8 TB/s HBM peak.  Because a
two-step launch reads and writes the populations once for two updates, that
fraction can exceed 1; `roofline.per_launch_hbm` gives the launch's own
bytes (one read and one write per cell) against the peak, against a plain
device copy measured in the same run, and (FP64) against the stream probe: the
same population access pattern without the arithmetic (lbm_probe_stream).  `traffic` is the counter-measured HBM
bytes per launch while the kernel source is the one the counters were taken
on.

With the default FP64 BGK workload the line also carries
  `precision`: the same workload in the FP32-, FP16- and per-cell-FP16-shifted
      storage modes (a few hundred timed steps each), rate and speedup;
  `serving`: a reduced seeded serving stream (Poisson arrivals) through the
      continuous-batching server in each reduced-precision mode, p50/p99
      time-to-result against the same jobs run one after another on the plain
      FP64 path;
  `cpu_baseline`: the CPU oracle on a bounded sample of the same workload, at
      one thread and at all host threads, median of three runs each.

--storage f32 / f16 / f16l runs the slab workload in that storage mode alone;
--collision mrt with the MRT collision (moment matrix of Appendix A, Lambda =
diag(1, ..., 1, 1/tau, 1/tau) as in the paper's oscillation runs).
--workload batch measures 256 uneven droplet lattices in one batch;
--workload serve the full 64-job serving stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extras] [--serve-jobs J]
                       [--storage f64|f32|f16|f16l] [--collision bgk|mrt]
                       [--fusion 1|2] [--one-by-one] [--launch BX,ROWS] [--autotune]
                       [--workload slab|batch|serve] [--jobs J]
       python bench.py --copy-calibration   (plain copy kernel for PMC scaling)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic bytes of one cell update: 9 populations read + 9 written (and,
# for f16l, the per-cell FP32 reference read and written).
BYTES_PER_UPDATE = {"f64": 144, "f32": 72, "f16": 36, "f16l": 44}
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E
# wave64 VALU instruction issue: 256 CUs x 4 SIMDs x 2.4 GHz, one FP32 (not
# packed) or FP64 instruction per 4 cycles per SIMD
VALU_PEAK_GIPS = 614.4
# storage modes whose two-step pass is bound by VALU issue (committed counters)
ISSUE_BOUND = ("f16", "f16l")
METRIC = "MLUPS/GPU and % HBM roofline (FP64 vs FP32/FP16-shifted); p50/p99 time-to-result"
N = 2048
TEMPS = (0.6, 0.7, 0.8, 0.9)
WARMUP_FLOOR_STEPS = 200      # untimed steps before any timed region
# Launch shape (threads per workgroup, segment rows) of the four-lattice batch
# per steps per launch and storage mode: the fastest of `--launch` sweeps of
# this workload (two-step pass, G cell updates/s: FP64 rows 24/32/37/48 gave
# 71.2/72.7/71.8/66.9; FP32 rows 12/16/21 137.2/136.6/136.1, within run-to-run
# noise; FP16 rows 24/30/37/48 176.7/181.5/185.1/169.1; per-cell FP16 the same
# rows 136.6/140.6/142.9/131.9).  Fixed, so that runs
# are reproducible and launch the shape the committed counters were taken on;
# --autotune times the candidates instead (lbm_batch_autotune), which cannot
# tell shapes 1% apart from run to run.
SLAB_LAUNCH = {2: {"f64": (256, 32), "f32": (256, 16), "f16": (256, 37), "f16l": (256, 37)},
               1: {"f64": (256, 5), "f32": (256, 5), "f16": (256, 5), "f16l": (256, 5)}}
PRECISION_STEPS = 400         # timed steps per reduced-precision mode
KERNEL_SRC = os.path.join(ROOT, "paper_2003_07968_amd", "csrc", "lbm_kernels.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{kernel}_{storage}_4x2048.json")
DTYPE = {"f64": "f64", "f32": "f32 (FP32-shifted storage)",
         "f16": "f32 arithmetic, f16-shifted storage",
         "f16l": "f32 arithmetic, f16 storage with per-cell f32 reference"}
# What limits each dominant kernel, from the committed counter profiles
# (profiles/pass2_4x2048_sq_counters.md, profiles/pass2_*_4x2048_traffic.md):
# counter-measured HBM bytes against a plain device copy, and VALU issue time
# (SQ_INSTS_VALU x 4 cycles per wave64 instruction over 1024 SIMDs at 2.4 GHz)
# against the launch time.
LIMITER = {
    ("pass2", "f64"): "hbm and latency: 1.06x the algorithmic bytes at about 5.5 TB/s, above a "
                      "plain device copy's rate and about 95% of the stream probe of the same "
                      "access pattern (roofline.per_launch_hbm.stream_probe_gbs); "
                      "VALU issue 33% of the launch, 40% of wave-cycles waiting on FP64 "
                      "dependencies at two waves per SIMD; a third wave per SIMD measured no "
                      "faster (profiles/pass2_4x2048_sq_counters.md)",
    ("pass2", "f32"): "hbm and issue: 1.06x the algorithmic bytes at about 5.3 TB/s, a plain "
                      "device copy's rate; VALU issue 61% of the launch "
                      "(profiles/pass2_4x2048_sq_counters.md)",
    ("pass2", "f16"): "valu: FP32 arithmetic issue 83% of the launch; HBM about 3.4 TB/s, 1.03x "
                      "the algorithmic bytes (profiles/pass2_4x2048_sq_counters.md)",
    ("pass2", "f16l"): "valu: FP32 arithmetic issue 90% of the launch; HBM about 3.2 TB/s, 1.05x "
                       "the algorithmic bytes (profiles/pass2_4x2048_sq_counters.md)",
}


def err(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def counter_record(kernel, storage, shape=None):
    """The committed rocprofv3 counter record of `kernel` ("pass2" or "step")
    in this storage mode, if it was taken on the current kernel source and,
    when `shape` (block_x, seg_rows) is given, at that launch shape (the
    traffic of a launch depends on its segments' halo rows)."""
    path = TRAFFIC_FILE.format(kernel=kernel, storage=storage)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != source_digest():
        return None
    if shape is not None and list(rec.get("launch_block_x_seg_rows") or []) != list(shape):
        return None
    return rec


def measured_traffic(kernel, storage, shape=None):
    """HBM bytes per launch from the committed counter runs, or None."""
    rec = counter_record(kernel, storage, shape)
    return rec.get("bytes_per_launch") if rec else None


def valu_roofline(kernel, storage, launch_ms, shape=None):
    """VALU issue of one launch against the chip's issue rate: the launch's
    wave64 VALU instructions (SQ_INSTS_VALU of the committed counter run; the
    count is fixed by the code and the launch shape) over its live average
    duration, against 1024 SIMDs x 2.4 GHz / 4 cycles per wave64 FP32 or FP64
    instruction = 614.4 G instructions/s.  None without a current record."""
    rec = counter_record(kernel, storage, shape)
    if not rec or not rec.get("valu_insts_per_launch"):
        return None
    achieved = rec["valu_insts_per_launch"] / (launch_ms / 1e3) / 1e9
    return {"unit": "G wave64 VALU instructions/s", "achieved": round(achieved, 1),
            "peak": VALU_PEAK_GIPS, "frac": round(achieved / VALU_PEAK_GIPS, 4),
            "insts_per_launch": rec["valu_insts_per_launch"]}


def copy_calibration():
    import torch
    n = 1 << 27  # 128 Mi doubles = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    err(f"copy calibration: 5 copies of {a.numel() * 8} bytes (read + write each)")


def copy_bandwidth_gbs(reps=5):
    """Bandwidth of a plain device copy (torch copy_ of 1 GiB of FP64: 1 GiB
    read + 1 GiB written per copy), the best of `reps`, in GB/s."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return 2 * (1 << 30) / (best / 1e3) / 1e9


def stream_probe_gbs(reps=5, launches=10, seg_rows=(4, 8, 16, 32)):
    """Bandwidth of the step kernels' population access pattern without their
    arithmetic (lbm_probe_stream: nine FP64 planes pulled as one time step
    pulls them, non-temporal stores) on a 2048 x 8192 lattice, the cells of
    one launch of the four-lattice batch: 144 B per cell over the best of
    `reps` samples of `launches` launches, at the best of the segment
    lengths, in GB/s."""
    import torch
    from paper_2003_07968_amd import lbm
    nx, ny = N, N * len(TEMPS)
    n = lbm.lbm_probe_stream_bytes(nx, ny) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    best = None
    for rows in seg_rows:
        for _ in range(3):
            lbm.lbm_probe_stream(a, b, nx, ny, rows)
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(launches):
                lbm.lbm_probe_stream(a, b, nx, ny, rows)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / launches
            best = ms if best is None else min(best, ms)
    del a, b
    return 144.0 * nx * ny / (best / 1e3) / 1e9


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(runs=3, steps_one=2, steps_all=6):
    """The CPU oracle on one 2048 x 2048 slab of the workload (T_r = 0.8): the
    median of `runs` timings of `steps_one` steps at one thread and of
    `steps_all` steps at all host threads (about 20 s of CPU work)."""
    import statistics
    from oracle import lbmref
    from paper_2003_07968_amd import workloads as W
    p, rho0 = W.slab_case(n=N, tr=0.8)
    P = lbmref.make_params(p["nx"], p["ny"], tau=p["tau"], G=p["G"], epsilon=p["epsilon"],
                           sigma=p["sigma"], eos=(p["eos_a"], p["eos_b"], p["eos_c"],
                                                  p["eos_k"]), T=p["T"])
    f = lbmref.init(P, rho0)
    all_threads = lbmref.threads()
    lbmref.step(P, f, 1)  # warm the pages

    def median_rate(threads, steps):
        lbmref.set_threads(threads)
        rates, secs = [], []
        for _ in range(runs):
            t0 = time.perf_counter()
            lbmref.step(P, f, steps)
            el = time.perf_counter() - t0
            rates.append(N * N * steps / el / 1e6)
            secs.append(el)
        return statistics.median(rates), sum(secs)

    one, s_one = median_rate(1, steps_one)
    full, s_full = median_rate(all_threads, steps_all)
    lbmref.set_threads(all_threads)
    return {"value": round(full, 3), "unit": "MLUPS", "cores": all_threads, "kind": "oracle",
            "sample": f"one 2048x2048 slab (T_r=0.8), median of {runs} runs of {steps_all} "
                      f"oracle steps at {all_threads} threads ({s_full:.1f} s) and of "
                      f"{steps_one} steps at 1 thread ({s_one:.1f} s)",
            "single_thread": {"value": round(one, 3), "unit": "MLUPS", "cores": 1},
            "cpu_model": cpu_model()}


def run_batch(args):
    """256 independent droplet lattices (sides log-uniform in [64, 512], T_r
    U[0.55, 0.95], sigma U[1/8, 4], R0 U[0.15, 0.35] side, seed 6) stepped by
    one batched launch per two steps (the two-step pass) or per step, as the
    autotuner finds faster (--fusion 1: single steps only), with FP32-shifted
    storage, shape chosen by the autotuner,
    8-step HIP graphs replayed.  Beside it, the same lattices in FP64 stepped
    each on its own (the plain path: one two-step launch per lattice per two
    steps)."""
    import torch
    from paper_2003_07968_amd import lbm
    from paper_2003_07968_amd import workloads as W

    storage = args.storage if args.storage != "f64" else "f32"
    stream = torch.cuda.Stream()  # graphs cannot be captured on the null stream
    with torch.cuda.stream(stream):
        cases = W.batch_case(count=256, seed=6, storage=storage)
        cells = sum(p["nx"] * p["ny"] for p, _ in cases)
        lats = [lbm.Lattice(p, r) for p, r in cases]
        batch = lbm.Batch(len(lats))
        if args.fusion is not None:
            batch.set_fusion(args.fusion)
        for lat in lats:
            batch.add(lat)
        bx, rows, us = batch.autotune()  # shape, and one or two steps per launch
        fusion = batch.fusion()
        err(f"batch of {len(lats)} lattices, {cells} cells; autotuned block {bx}, "
            f"rows {rows}: {us:.1f} us/step")
        batch.step(args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        batch.step(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        gpu_ms = e0.elapsed_time(e1)
        for lat in lats:
            lat.sync()
        err(f"timed {args.steps} batched steps: {gpu_ms:.2f} ms")

        # the plain path on the same lattices: FP64 storage, each lattice on
        # its own (two steps per launch)
        seq_steps = 2 * max(4, args.steps // 20)
        plain = []
        for p, r in cases:
            q = dict(p)
            q["storage"], q["rho_ref"] = 0, 0.0
            plain.append(lbm.Lattice(q, r))
        for lat in plain:
            lat.step(2)
        torch.cuda.synchronize()
        e2 = torch.cuda.Event(enable_timing=True)
        e3 = torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        for _ in range(seq_steps // 2):
            for lat in plain:
                lat.step(2)
        e3.record(stream)
        torch.cuda.synchronize()
        plain_ms = e2.elapsed_time(e3)
        for lat in plain:
            lat.sync()
    mlups = cells * args.steps / (gpu_ms / 1e3) / 1e6
    plain_mlups = cells * seq_steps / (plain_ms / 1e3) / 1e6
    bpc = BYTES_PER_UPDATE[storage]
    step_ms = gpu_ms / args.steps
    launches = args.steps // fusion + args.steps % fusion
    launch_ms = gpu_ms / launches
    achieved = bpc * cells / (launch_ms / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32 arithmetic, f32-shifted storage",
                  "f16": "f32 arithmetic, f16-shifted storage",
                  "f16l": "f32 arithmetic, f16 storage with per-cell f32 reference"}[storage],
        "data": "synthetic",
        "config": {
            "workload": "batch of 256 D2Q9 droplet lattices, sides log-uniform [64, 512], "
                        "T_r U[0.55,0.95], sigma U[1/8,4], R0 U[0.15,0.35] side, seed 6; "
                        f"one batched launch per {fusion} step(s), 8-step HIP "
                        "graphs, autotuned shape",
            "storage": storage, "lattices": len(lats), "cells": cells,
            "steps_per_launch": fusion, "bytes_per_cell_and_launch": bpc,
            "launch_block_x_seg_rows": [bx, rows],
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": ("batch2_kernel (two steps per launch)" if fusion == 2 else
                       "batch_step_kernel (one step per launch)"),
            "kernel_avg_ms": round(launch_ms, 5),
        },
        "plain_fp64_sequential": {
            "value": round(plain_mlups, 1), "unit": "MLUPS", "steps": seq_steps,
            "speedup_of_batch": round(mlups / plain_mlups, 2),
        },
    }
    print(json.dumps(out), flush=True)


def _percentiles(x):
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    return {"p50_s": round(float(np.percentile(x, 50)), 4),
            "p99_s": round(float(np.percentile(x, 99)), 4),
            "mean_s": round(float(x.mean()), 4)}


def serve_stream(jobs, arrivals, storage, arena_bytes, quantum):
    """Run the jobs through the serving loop in real time: each is submitted at
    its arrival time; returns time-to-result per job, the makespan and the
    server's counters."""
    import numpy as np
    from paper_2003_07968_amd import lbm
    from paper_2003_07968_amd import workloads as W
    srv = lbm.Server(arena_bytes=arena_bytes, max_resident=128, quantum=quantum, max_bypass=16)
    order = np.argsort(arrivals, kind="stable")
    done_at, ids = {}, {}
    nxt = 0
    t0 = time.perf_counter()
    while len(done_at) < len(jobs):
        now = time.perf_counter() - t0
        while nxt < len(jobs) and arrivals[order[nxt]] <= now:
            k = int(order[nxt])
            p, rho0, n = jobs[k]
            q = dict(p)
            q["storage"] = W.STORAGE[storage]
            q["rho_ref"] = W.shift_reference(rho0, storage)
            ids[srv.submit(q, rho0, n)] = k
            nxt += 1
        st = srv.stats()
        if st["queued"] == 0 and st["resident"] == 0:
            if nxt < len(jobs):
                time.sleep(max(0.0, arrivals[order[nxt]] - (time.perf_counter() - t0)))
            continue
        srv.advance()
        t = time.perf_counter() - t0
        for job, status, rho, f in srv.poll():
            if status != lbm.LBM_OK:
                raise RuntimeError(f"job {job} failed with status {status}")
            done_at[ids[job]] = t
    stats = srv.stats()
    srv.close()
    ttr = [done_at[k] - arrivals[k] for k in range(len(jobs))]
    return ttr, max(done_at.values()), stats


def serve_measure(count, modes=("f32", "f16", "f16l")):
    """Continuous batching of a seeded Poisson stream of `count` jobs (sides
    log-uniform in [64, 1024], steps U[2000, 50000], droplet or slab, seed 7)
    in each reduced-precision storage mode, against the same jobs run one
    after another on the plain FP64 path (first come, first served).  The
    arrival rate is 0.8 x the capacity: the throughput of the same jobs, cut to
    2000 steps each, all submitted at once, measured on the second of two such
    runs (the first one pays the arena's first use and the clocks' ramp from
    idle, about 15 % of its 0.3 s)."""
    import numpy as np
    import torch
    from paper_2003_07968_amd import lbm
    from paper_2003_07968_amd import workloads as W

    jobs = W.serve_case(count=count, seed=7, storage="f32")
    work = np.array([p["nx"] * p["ny"] * n for p, _, n in jobs], dtype=np.float64)
    arena = 48 << 30
    quantum = 128

    cal = [(p, r, 2000) for p, r, _ in jobs]
    for _ in range(2):
        _, span, st = serve_stream(cal, np.zeros(len(cal)), "f32", arena, quantum)
    capacity = st["cell_steps"] / span
    rate = 0.8 * capacity / work.mean()
    arrivals = W.poisson_arrivals(len(jobs), rate, seed=7)
    err(f"{len(jobs)} jobs, {work.sum():.3e} cell updates; capacity {capacity / 1e6:.0f} MLUPS "
        f"-> arrival rate {rate:.2f} jobs/s")

    served = {}
    for storage in modes:
        ttr, span, st = serve_stream(jobs, arrivals, storage, arena, quantum)
        served[storage] = dict(_percentiles(ttr), mlups=round(st["cell_steps"] / span / 1e6, 1),
                               makespan_s=round(span, 3), rounds=st["rounds"],
                               arena_peak_bytes=st["arena_peak"])
        err(f"served {storage}: {served[storage]}")

    # sequential FP64: each job alone (init, steps, density to the host), its
    # service time measured; first-come-first-served completion times follow
    stream = torch.cuda.Stream()
    service = np.zeros(len(jobs))
    with torch.cuda.stream(stream):
        for k, (p, rho0, n) in enumerate(jobs):
            q = dict(p)
            q["storage"], q["rho_ref"] = 0, 0.0
            torch.cuda.synchronize()
            t = time.perf_counter()
            lat = lbm.Lattice(q, rho0)
            lat.step(n)
            lat.moments()["rho"].cpu()
            lat.sync()
            service[k] = time.perf_counter() - t
            del lat
    finish, ttr_seq = 0.0, []
    for k in np.argsort(arrivals, kind="stable"):
        finish = max(finish, arrivals[k]) + service[k]
        ttr_seq.append(finish - arrivals[k])
    seq = dict(_percentiles(ttr_seq), mlups=round(work.sum() / service.sum() / 1e6, 1),
               makespan_s=round(finish, 3))
    err(f"sequential fp64: {seq}")
    return {
        "jobs": len(jobs), "cell_updates": float(work.sum()), "arrival_rate_per_s": round(rate, 3),
        "capacity_mlups": round(capacity / 1e6, 1), "quantum_steps": quantum,
        "arena_bytes": arena, "served": served, "sequential_fp64": seq,
        "p50_speedup_vs_sequential_fp64": {m: round(seq["p50_s"] / v["p50_s"], 2)
                                           for m, v in served.items()},
        "p99_speedup_vs_sequential_fp64": {m: round(seq["p99_s"] / v["p99_s"], 2)
                                           for m, v in served.items()},
    }


def run_serve(args):
    """The full serving stream (--jobs, default 64) as its own line."""
    res = serve_measure(args.jobs)
    out = {
        "metric": METRIC, "value": res["served"]["f32"]["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 arithmetic, f32-shifted storage", "data": "synthetic",
        "config": {
            "workload": f"serving stream of {res['jobs']} D2Q9 jobs, Poisson arrivals at "
                        f"{res['arrival_rate_per_s']:.2f}/s (0.8 x measured capacity), sides "
                        "log-uniform [64, 1024], steps U[2000, 50000], droplet or slab, T_r "
                        "U[0.55,0.95], sigma U[1/8,4], seed 7; continuous batching, "
                        "HBM-footprint admission",
        },
        "serving": res,
    }
    print(json.dumps(out), flush=True)


def serving_summary(count):
    """The serving part of the default line: a reduced stream of `count` jobs."""
    res = serve_measure(count)
    res["note"] = (f"reduced stream: the first {count} jobs of the 64-job recipe "
                   "(bench.py --workload serve runs all 64)")
    return res


def run_slab(storage, collision, fusion, steps, warmup, one_by_one=False, shape=None,
             autotune=False):
    """The four-temperature 2048^2 slab workload in one storage mode.  The four
    lattices are advanced together through the library's batch entry points
    (one launch covers all four lattices, two time steps per launch), with
    the launch shape `shape` (block_x, seg_rows), by default SLAB_LAUNCH's,
    or the one the batch autotuner picks; with one_by_one each lattice gets
    launches of its own instead.  Untimed warm-up (at least
    WARMUP_FLOOR_STEPS steps), then `steps` timed steps enqueued right behind
    it, bracketed by events on the library's stream, with events at about
    every tenth of the paired steps for the spread.  Every lattice's sticky
    error word is checked after the timed region (it covers the warm-up
    too)."""
    import torch
    from paper_2003_07968_amd import lbm
    from paper_2003_07968_amd import workloads as W

    stream = torch.cuda.Stream()  # graphs of the batch cannot be captured on the null stream
    with torch.cuda.stream(stream):
        lats = []
        for tr in TEMPS:
            p, rho0 = W.slab_case(n=N, tr=tr)
            p["storage"] = W.STORAGE[storage]
            p["rho_ref"] = W.shift_reference(rho0, storage)
            p["collision"] = W.COLLISION[collision]
            lats.append(lbm.Lattice(p, rho0))
            if fusion is not None:
                lats[-1].set_fusion(fusion)
        if one_by_one:
            batch = None
            launch = list(lats[0].launch())
            fus = lats[0].fusion()
        else:
            batch = lbm.Batch(len(lats))
            if fusion is not None:
                batch.set_fusion(fusion)
            for lat in lats:
                batch.add(lat)
            if autotune:
                batch.autotune()
            else:
                batch.set_launch(fusion or 2, *(shape or SLAB_LAUNCH[fusion or 2][storage]))
            fus, bx, rows = batch.launch()
            launch = [bx, rows]
        torch.cuda.synchronize()
        err(f"{storage}: lattices ready, {fus} step(s) per launch, "
            f"{'one lattice per launch' if one_by_one else 'four lattices per launch'}, "
            f"launch shape {launch}")

        def advance(nsteps):
            if batch is not None:
                batch.step(nsteps)
                return
            for _ in range(nsteps // 2):
                for lat in lats:
                    lat.step(2)
            for _ in range(nsteps % 2):
                for lat in lats:
                    lat.step(1)

        e0 = torch.cuda.Event(enable_timing=True)
        em = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        pairs, odd = divmod(steps, 2)
        blk = max(1, pairs // 10)
        marks = []
        wsteps = max(warmup, WARMUP_FLOOR_STEPS)
        wsteps += wsteps % 2          # whole pairs, so the timed region starts on a pair
        t0 = time.perf_counter()
        advance(wsteps)
        e0.record(stream)
        done_pairs = 0
        while done_pairs < pairs:
            n = min(blk, pairs - done_pairs)
            advance(2 * n)
            done_pairs += n
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            marks.append((n, ev))
        em.record(stream)
        advance(odd)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for lat in lats:
            lat.sync()   # raises on a sticky domain error (warm-up or timed steps)
    gpu_ms = e0.elapsed_time(e1)
    pair_ms = e0.elapsed_time(em)
    block_rates, prev = [], e0
    for n, ev in marks:
        ms = prev.elapsed_time(ev)
        if ms > 0:
            block_rates.append(N * N * len(lats) * 2 * n / (ms / 1e3) / 1e6)
        prev = ev
    err(f"{storage}: {wsteps} warm-up steps, then {steps} timed steps: {gpu_ms:.2f} ms on the "
        f"stream ({wall * 1e3:.1f} ms wall including the warm-up)")
    # lattices one launch covers, and launches per pair of steps
    per_launch = 1 if one_by_one else len(lats)
    launches_per_pair = len(lats) // per_launch * (1 if fus == 2 else 2)
    if fus == 2 and pairs > 0:
        kernel, launch_ms = "pass2", pair_ms / (pairs * launches_per_pair)
        kname = ("sweep2_kernel (two steps per launch" if one_by_one else
                 "batch2_kernel (two steps per launch, four lattices per launch")
    else:
        kernel = "step"
        launch_ms = gpu_ms / (steps * len(lats) // per_launch)
        kname = ("sweep_kernel (one step per launch" if one_by_one else
                 "batch_step_kernel (one step per launch, four lattices per launch")
    timed_launches = (pairs * launches_per_pair + odd * len(lats) // per_launch
                      if fus == 2 else steps * len(lats) // per_launch)
    res = {"mlups": N * N * len(lats) * steps / (gpu_ms / 1e3) / 1e6, "gpu_ms": gpu_ms,
           "launch_ms": launch_ms, "kernel": kernel, "kernel_name": kname, "fusion": fus,
           "launch": launch, "lattices": len(lats), "lattices_per_launch": per_launch,
           "timed_launches": timed_launches, "warmup_steps": wsteps,
           "block_rates": block_rates if len(block_rates) >= 5 else []}
    del batch, lats
    torch.cuda.synchronize()
    return res


def one_by_one_rate(batched_mlups, steps=PRECISION_STEPS):
    """The default workload with launches of one lattice each (the
    single-lattice two-step kernel, four launches per pair of steps), beside
    the batched figure of the line."""
    r = run_slab("f64", "bgk", None, steps, 0, one_by_one=True)
    upl = 2 if r["kernel"] == "pass2" else 1
    achieved = BYTES_PER_UPDATE["f64"] * upl * N * N / (r["launch_ms"] / 1e3) / 1e9
    return {"value": round(r["mlups"], 1), "unit": "MLUPS", "steps": steps,
            "kernel": r["kernel_name"] + ", f64 storage, bgk)",
            "kernel_avg_ms": round(r["launch_ms"], 5),
            "launch_block_x_seg_rows_workgroups": list(r["launch"]),
            "roofline_frac": round(achieved / HBM_PEAK_GBS, 4),
            "batched_over_one_by_one": round(batched_mlups / r["mlups"], 3)}


def precision_rates(f64_mlups):
    """The slab workload in each reduced-precision storage mode (BGK, default
    launch), PRECISION_STEPS timed steps each: rate, the dominant kernel's
    launch time and the roofline fraction of its own bytes per update."""
    out = {"steps": PRECISION_STEPS}
    for st in ("f32", "f16", "f16l"):
        r = run_slab(st, "bgk", None, PRECISION_STEPS, 0)
        upl = 2 if r["kernel"] == "pass2" else 1
        bpu = BYTES_PER_UPDATE[st]
        achieved = bpu * upl * N * N * r["lattices_per_launch"] / (r["launch_ms"] / 1e3) / 1e9
        out[st] = {"value": round(r["mlups"], 1), "unit": "MLUPS",
                   "speedup_vs_f64": round(r["mlups"] / f64_mlups, 3),
                   "bytes_per_cell_update": bpu, "steps_per_launch": r["fusion"],
                   "lattices_per_launch": r["lattices_per_launch"],
                   "launch_block_x_seg_rows": list(r["launch"][:2]),
                   "kernel_avg_ms": round(r["launch_ms"], 5),
                   "roofline_frac": round(achieved / HBM_PEAK_GBS, 4),
                   "per_launch_hbm_frac": round(achieved / upl / HBM_PEAK_GBS, 4),
                   "valu": valu_roofline(r["kernel"], st, r["launch_ms"], r["launch"][:2]),
                   "limiter": LIMITER.get((r["kernel"], st))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--storage", choices=sorted(BYTES_PER_UPDATE), default="f64")
    ap.add_argument("--collision", choices=("bgk", "mrt"), default="bgk")
    ap.add_argument("--workload", choices=("slab", "batch", "serve"), default="slab")
    ap.add_argument("--fusion", type=int, choices=(1, 2), default=None,
                    help="time steps per launch (default: the library's choice)")
    ap.add_argument("--jobs", type=int, default=64, help="jobs in the serving stream")
    ap.add_argument("--serve-jobs", type=int, default=24,
                    help="jobs in the reduced serving stream of the default line")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision and serving parts of the default line")
    ap.add_argument("--one-by-one", action="store_true",
                    help="slab workload: launches of one lattice each instead of one batch")
    ap.add_argument("--launch", default=None, metavar="BX,ROWS",
                    help="slab workload: this batch launch shape instead of SLAB_LAUNCH's")
    ap.add_argument("--autotune", action="store_true",
                    help="slab workload: the batch autotuner's launch shape")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the lattice update here runs on a single MI355X; "
              "run it with --gpus 1 (multi-GPU sharding is described, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration()
        return

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return

    shape = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    res = run_slab(args.storage, args.collision, args.fusion, args.steps, args.warmup,
                   args.one_by_one, shape, args.autotune)
    n_lat = res["lattices"]
    bpu = BYTES_PER_UPDATE[args.storage]
    kernel = res["kernel"]
    upl = 2 if kernel == "pass2" else 1
    launch_s = res["launch_ms"] / 1e3
    cells = N * N * res["lattices_per_launch"]   # cells one launch covers
    # the roofline of one cell update: one read and one write of its
    # populations (bpu bytes) at peak bandwidth; a two-step launch makes two
    # updates per cell with one read and one write, so its update rate can
    # exceed that figure
    achieved = bpu * upl * cells / launch_s / 1e9
    launch_gbs = bpu * cells / launch_s / 1e9
    # the committed counter records are of the batched launch
    counters = args.collision == "bgk" and not args.one_by_one
    traffic = measured_traffic(kernel, args.storage, res["launch"][:2]) if counters else None
    copy_gbs = copy_bandwidth_gbs()
    probe_gbs = stream_probe_gbs() if args.storage == "f64" else None
    mlups = res["mlups"]

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["gpu_ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {
            "workload": "D2Q9 2048x2048 periodic flat slab, T_r in {0.6,0.7,0.8,0.9} "
                        "(four lattices), tau=1, Carnahan-Starling a=1 b=4 R=1, G=-1, "
                        "eps=1.73, sigma=1, W=2, seeded +-1e-3 noise",
            "storage": args.storage, "collision": args.collision,
            "lattices": n_lat, "nx": N, "ny": N,
            "steps_per_launch": res["fusion"],
            "lattices_per_launch": res["lattices_per_launch"],
            "bytes_per_cell_update": bpu,
            "launch_block_x_seg_rows": list(res["launch"][:2]),
            "launch_from": ("each lattice's default" if args.one_by_one else
                            "batch autotuner" if args.autotune else
                            "--launch" if shape else "bench table (SLAB_LAUNCH)"),
            "timed_launches": res["timed_launches"],
            "untimed_warmup_steps": res["warmup_steps"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": f"{res['kernel_name']}, {args.storage} storage, {args.collision})",
            "kernel_avg_ms": round(res["launch_ms"], 5),
            "updates_per_launch_per_cell": upl,
            "limiter": LIMITER.get((kernel, args.storage)) if counters else None,
            "valu": (valu_roofline(kernel, args.storage, res["launch_ms"], res["launch"][:2])
                     if counters else None),
            "per_launch_hbm": {
                "bytes": bpu * cells,
                "achieved": round(launch_gbs, 1),
                "frac": round(launch_gbs / HBM_PEAK_GBS, 4),
                "copy_kernel_gbs": round(copy_gbs, 1),
                "frac_of_copy": round(launch_gbs / copy_gbs, 4),
                "stream_probe_gbs": round(probe_gbs, 1) if probe_gbs else None,
                "frac_of_stream_probe": round(launch_gbs / probe_gbs, 4) if probe_gbs else None,
            },
        },
    }
    # the issue-bound modes (FP16 storage, FP32 arithmetic) are priced against
    # the VALU issue rate, the HBM figures kept beside it
    rf = out["roofline"]
    if args.storage in ISSUE_BOUND and rf["valu"] is not None:
        v = rf.pop("valu")
        rf["hbm"] = {k: rf[k] for k in ("achieved", "peak", "unit", "frac")}
        rf.update(bound="alu", achieved=v["achieved"], peak=v["peak"], unit=v["unit"],
                  frac=v["frac"], valu_insts_per_launch=v["insts_per_launch"])
    if res["block_rates"]:
        import numpy as np
        br = res["block_rates"]
        out["value_spread"] = {
            "blocks": len(br), "unit": "MLUPS",
            "p10": round(float(np.percentile(br, 10)), 1),
            "p50": round(float(np.percentile(br, 50)), 1),
            "p90": round(float(np.percentile(br, 90)), 1)}
    if args.storage == "f64" and args.collision == "bgk" and not args.no_extras:
        out["one_lattice_per_launch"] = one_by_one_rate(mlups)
        out["precision"] = precision_rates(mlups)
        out["serving"] = serving_summary(args.serve_jobs)
    if not args.no_cpu_baseline and args.storage == "f64":
        err("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
