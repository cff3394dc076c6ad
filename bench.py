#!/usr/bin/env python3
"""Benchmark: R factor of a tall-skinny matrix by TSQR on one MI355X.

Workload (the paper's problem at production size): one instance of
m = 2^22 rows by n = 50 columns, FP64, entries uniform[-1,1) from seed 1,
resident in HBM before timing starts.  A step is one full pass of the hot path
(leaf factorisations + reduction tree + finalisation) through one C-ABI call,
which launches a small kernel that clears the tree counters and then the fused
leaf+tree kernel.  Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 50] [--warmup 30] [--no-cpu-baseline] [--no-batched]
        [--no-mixed] [--no-learned] [--no-q] [--no-library] [--no-tuning]

The warmup is long enough (about 50 ms of kernel time) for the GPU clocks to
settle before the timed steps.  The handle follows the shipped tuning table
(paper_1002_4250_amd/tuning_gfx950.json, written by the autotuner); at the
benchmark's shapes it selects the built-in defaults.

The ``mixed`` object measures 256 FP32-stored instances of 2^16 x 50 with
condition numbers 1..1e8: FP32 TSQR followed by one FP64 correction, against
the plain FP64 batched TSQR of the same data and the FP32 TSQR alone, with
sampled accuracy against the oracle.

The ``q_factor`` object times A = QR with Q formed explicitly from the stored
reflectors on the plain instance, with torch.linalg.qr beside it for context.

The ``batched`` object of the line measures the ragged batch (4096 instances,
m log-uniform in [64, 65536], n = 50, FP32) three ways: one batched launch per
step, a Python loop of single-matrix calls, and the same loop captured once
in a HIP graph and replayed.

The ``small_instance`` object times the small case (m = 256, n = 50, FP64)
per call back to back, per call with a host
synchronization, and per replay of the call captured in a HIP graph.
``host`` records the CPU model and core counts; ``cpu_baseline_all_cores`` runs
the paper's method on every usable host core (oracle block QRs in threads,
then the oracle's operator over a binary tree) beside the one-core oracle.

Roofline: the path is bound by the FP64 vector FMA rate (arithmetic
intensity 2n/8 = 12.5 flop/byte against a ridge of 78.6/8 = 9.8), so
``roofline`` reports the kernel's algorithmic 2*m*n^2 flops per launch divided
by its average launch duration (HIP events on the launch stream) against the
78.6 TFLOP/s FP64 vector peak.  ``cpu_baseline`` times the CPU oracle (plain
single-threaded Householder in C) factoring the full instance twice.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "core-kernel instances/sec + % roofline at oracle-matched accuracy, plain vs batched"
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3    # the published FP32 vector peak (counts packed FP32 issue)
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tsqr_leaf_tree_f64_m4194304_n50_traffic.json")


def measured_traffic():
    """HBM bytes per launch of the leaf+tree kernel from the committed counter
    runs (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None if
    the kernel sources changed since those counters were taken."""
    try:
        from paper_1002_4250_amd import build as b
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        if rec.get("kernel_source_digest") != b._digest(b.KERNEL_DEPS):
            return None
        return rec["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def to_device_colmajor(torch, A):
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda").t()


def time_plain(torch, tsqr, Ad, steps, warmup):
    """(ms per step over the timed region, mean kernel ms from per-launch events, R)."""
    m, n = Ad.shape
    h = tsqr.handle(0)
    ws = tsqr.workspace(m, n, Ad.dtype)
    R = torch.empty((n, n), dtype=Ad.dtype, device="cuda").t()
    for _ in range(warmup):
        tsqr.geqr_r(Ad, R=R, ws=ws, h=h)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for a, b in ev:
        a.record()
        tsqr.geqr_r(Ad, R=R, ws=ws, h=h)
        b.record()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t0.elapsed_time(t1) / steps
    ms_kernel = sum(a.elapsed_time(b) for a, b in ev) / steps
    return ms_step, ms_kernel, wall, R


def time_phases(torch, tsqr, Ad, flops):
    """Where the FP64 kernel's time goes, from the per-leaf clock stamps of
    tsqr_geqr_r_f64_stamped: launches run back to back after plain ones, as
    in the timed loop (a launch after an idle gap runs slower while the
    clocks come back up); of the last three, the one with the median span."""
    import numpy as np
    m, n = Ad.shape
    h = tsqr.handle(0)
    ws = tsqr.workspace(m, n, Ad.dtype)
    R = torch.empty((n, n), dtype=Ad.dtype, device="cuda").t()
    leaves = tsqr.tsqr_plan_info(h, m, n, tsqr.TSQR_F64)[1]
    bufs = [torch.zeros((leaves, 4), dtype=torch.int64, device="cuda") for _ in range(5)]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in bufs]
    for _ in range(20):
        tsqr.geqr_r(Ad, R=R, ws=ws, h=h)
    for buf, (a, b) in zip(bufs, ev):
        a.record()
        tsqr.geqr_r_stamped(Ad, R=R, ws=ws, h=h, stamps=buf)
        b.record()
    torch.cuda.synchronize()
    khz = tsqr.device_clock_khz(h)
    runs = []
    for buf in bufs[2:]:
        st = buf.cpu().numpy()
        runs.append(((st[:, 2].max() - st[:, 0].min()) / khz, st))
    runs.sort(key=lambda r: r[0])
    st = runs[1][1]
    t0 = st[:, 0].min()
    leaf_end = (st[:, 1] - t0) / khz
    root = int(np.argmax(st[:, 3] >= 100))
    span = float((st[root, 2] - t0) / khz)
    leaf_ms = float(leaf_end.max())
    return {"span_ms": span, "starts_within_ms": float((st[:, 0].max() - t0) / khz),
            "leaf_phase_ms": leaf_ms, "leaf_phase_end_min_ms": float(leaf_end.min()),
            "tree_ms": span - leaf_ms, "tree_levels": int(st[root, 3] - 100),
            "leaf_phase_TFLOPs": flops / (leaf_ms * 1e-3) / 1e12,
            "leaf_phase_frac": flops / (leaf_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "spans_ms_of_3_launches": [float(r[0]) for r in runs],
            "event_ms_of_the_same_3_launches": [a.elapsed_time(b) for a, b in ev[2:]]}


def time_small(torch, tsqr, inputs, reps=200):
    """Latency of the small instance (m = 256, n = 50, FP64, seed 0; the
    automatic policy gives two leaves of 128 rows, so one chunk per leaf and
    one merge): per call in a back-to-back loop (HIP events), per call with a
    host synchronization after each (wall clock, launch overhead included),
    and per replay of the call captured in a HIP graph."""
    import numpy as np
    A = inputs.uniform(256, 50, 0)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    h = tsqr.handle(0)
    ws = tsqr.workspace(256, 50, torch.float64, h=h)
    R = torch.empty((50, 50), dtype=torch.float64, device="cuda").t()

    def call():
        tsqr.geqr_r(Ad, R=R, ws=ws, h=h)

    for _ in range(20):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    us_loop = e0.elapsed_time(e1) / reps * 1e3
    lat = []
    for _ in range(reps):
        t = time.perf_counter()
        call()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
    us_sync = float(np.median(lat) * 1e6)
    us_graph = None
    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            call()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        ref = R.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            call()
        for _ in range(10):
            g.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        us_graph = e0.elapsed_time(e1) / reps * 1e3
        if not torch.equal(R, ref):
            log("small instance: graph replay differs from the eager call")
            us_graph = None
    except RuntimeError as e:
        log(f"small instance: graph capture failed: {e}")
    lr, lv = tsqr.tsqr_plan_info(h, 256, 50, tsqr.TSQR_F64)
    log(f"small m=256 n=50 fp64: {us_loop:.1f} us/call back to back, {us_sync:.1f} us with a sync, "
        f"graph replay {us_graph if us_graph is None else round(us_graph, 1)} us")
    return {"workload": "m=256 n=50 fp64 uniform[-1,1) seed 0", "leaves": lv, "leaf_rows": lr,
            "us_per_call_back_to_back": us_loop, "us_per_call_synchronized": us_sync,
            "us_per_graph_replay": us_graph, "calls": reps}


def host_info():
    """CPU model and core counts of the host the benchmark runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def time_q(torch, tsqr, Ad, steps, warmup, library=True):
    """A = Q R with Q formed explicitly (tsqr_geqr_qr_f64) on the same FP64
    instance, checked by Q^T Q = I and Q R = A; the library QR of torch
    (rocSOLVER) on the same matrix is timed beside it for context."""
    m, n = Ad.shape
    h = tsqr.handle(0)
    ws = torch.empty(tsqr.tsqr_qr_workspace_bytes(h, m, n), dtype=torch.uint8, device="cuda")
    Q = torch.empty((n, m), dtype=Ad.dtype, device="cuda").t()
    R = torch.empty((n, n), dtype=Ad.dtype, device="cuda").t()

    def timed(fn, k, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    k = max(1, min(steps, 20))
    ms_q = timed(lambda: tsqr.geqr_qr(Ad, Q=Q, R=R, ws=ws, h=h), k, min(warmup, 10))
    orth = float(torch.linalg.norm(Q.t() @ Q - torch.eye(n, dtype=Ad.dtype, device="cuda")).item()) / n ** 0.5
    resid = float(((Q @ R - Ad).norm() / Ad.norm()).item())
    lib_ms = lib_r_ms = None
    if library:
        try:
            lib_ms = timed(lambda: torch.linalg.qr(Ad, mode="reduced"), 3, 1)
            lib_r_ms = timed(lambda: torch.linalg.qr(Ad, mode="r"), 3, 1)
        except RuntimeError as e:      # the library path is context only
            log(f"q: torch.linalg.qr unavailable: {e}")
    # the same call in FP32 (input: the FP32 rounding of A)
    A32 = Ad.float().t().contiguous().t()
    ws32 = torch.empty(tsqr.tsqr_qr_workspace_bytes(h, m, n, tsqr.TSQR_F32), dtype=torch.uint8, device="cuda")
    Q32 = torch.empty((n, m), dtype=torch.float32, device="cuda").t()
    R32 = torch.empty((n, n), dtype=torch.float32, device="cuda").t()
    ms_q32 = timed(lambda: tsqr.geqr_qr(A32, Q=Q32, R=R32, ws=ws32, h=h), k, min(warmup, 10))
    orth32 = float(torch.linalg.norm(Q32.double().t() @ Q32.double()
                                     - torch.eye(n, dtype=torch.float64, device="cuda")).item()) / n ** 0.5
    del A32, ws32, Q32, R32
    # Q^T B without forming Q: the factorization keeping its reflectors, then
    # the replay on one right-hand side and on 50
    del Q
    torch.cuda.empty_cache()
    fz = tsqr.Factorization(Ad, h=h)
    ms_geqrf = timed(lambda: tsqr.Factorization(Ad, h=h), max(1, k // 4), 2)
    b1 = Ad[:, :1].contiguous()
    c1 = torch.empty((1, n), dtype=Ad.dtype, device="cuda").t()
    ms_qt1 = timed(lambda: fz.apply_qt(b1, C=c1), k, min(warmup, 10))
    c50 = torch.empty((n, n), dtype=Ad.dtype, device="cuda").t()
    ms_qt50 = timed(lambda: fz.apply_qt(Ad, C=c50), k, min(warmup, 10))
    qt_err = float(((c50 - fz.R).norm() / fz.R.norm()).item())      # Q^T A = R
    del fz, b1, c1, c50
    torch.cuda.empty_cache()
    log(f"q: geqrf (reflectors kept) {ms_geqrf:.3f} ms; apply Q^T to 1 column {ms_qt1:.3f} ms, "
        f"to 50 columns {ms_qt50:.3f} ms (Q^T A vs R: {qt_err:.1e})")
    flops = 4.0 * m * n * n        # factorization 2mn^2 + forming Q 2mn^2 (LAPACK's counts for m >> n)
    gbs_min = 16.0 * m * n / (ms_q * 1e-3) / 1e9
    log(f"q: fp32 {ms_q32:.3f} ms per QR with Q, orthogonality {orth32:.1e}")
    log(f"q: {ms_q:.3f} ms per QR with Q ({flops / (ms_q * 1e-3) / 1e12:.2f} TFLOP/s at 4mn^2); "
        f"orth {orth:.1e} resid {resid:.1e}; torch.linalg.qr {lib_ms} ms (mode r {lib_r_ms} ms)")
    return {
        "workload": f"A = QR with explicit Q, m={m} n={n} fp64 (the plain instance)",
        "value": 1000.0 / ms_q, "unit": "instances/s", "ms_per_step": ms_q, "steps": k,
        "achieved_TFLOPs_4mn2": flops / (ms_q * 1e-3) / 1e12,
        "frac_fp64_vector_peak": flops / (ms_q * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
        "min_hbm_GBs_read_A_write_Q": gbs_min,
        "orthogonality": orth, "residual": resid,
        "torch_linalg_qr_reduced_ms": lib_ms, "torch_linalg_qr_r_ms": lib_r_ms,
        "fp32": {"value": 1000.0 / ms_q32, "unit": "instances/s", "ms_per_step": ms_q32,
                 "achieved_TFLOPs_4mn2": flops / (ms_q32 * 1e-3) / 1e12, "orthogonality": orth32},
        "apply_qt": {"what": "tsqr_geqrf_f64 (R and the reflectors) then tsqr_apply_qt_f64 = Q^T B without "
                             "forming Q", "geqrf_ms": ms_geqrf, "k1_ms": ms_qt1, "k50_ms": ms_qt50,
                     "k50_achieved_TFLOPs_2mn2k_equiv": 2.0 * m * n * n / (ms_qt50 * 1e-3) / 1e12,
                     "QtA_vs_R_relF": qt_err},
    }


def schedule_from_stamps(np, st, khz):
    """The batched launch's schedule from its per-workgroup (start, end)
    clock stamps: the span, the most workgroups resident at once (the
    slots), the busy fraction of slots x span, when the last workgroup
    started (the dispatcher's queue is empty from then on) and how the slots
    drain after it."""
    st = st - st[:, 0].min()
    start, end = st[:, 0] / khz, st[:, 1] / khz          # ms
    span = float(end.max())
    dur = end - start
    t = np.concatenate([start, end])
    d = np.concatenate([np.ones(len(st), np.int64), -np.ones(len(st), np.int64)])
    o = np.lexsort((d, t))
    active = np.cumsum(d[o])
    slots = int(active.max())
    full_at = float(t[o][int(np.argmax(active == slots))])
    last_start = float(start.max())
    drain = span - last_start
    in_drain = np.clip(np.minimum(end, span) - np.maximum(start, last_start), 0.0, None).sum()
    cap = slots * span
    return {"span_ms": span, "slots": slots, "busy_fraction": float(dur.sum() / cap),
            "all_slots_busy_at_ms": full_at, "last_start_ms": last_start, "drain_ms": drain,
            "mean_busy_slots_in_drain": float(in_drain / drain) if drain > 0 else None,
            "idle_fraction_in_drain": float((slots * drain - in_drain) / cap),
            "idle_fraction_before_drain": float((slots * last_start - (dur.sum() - in_drain)) / cap)}


def time_batched(torch, tsqr, inputs, steps, warmup, n=50, count=4096, single_loop=True):
    """The ragged batch: batched launch vs looped single-matrix calls (the
    loop, 8192 launches per pass, is skipped with single_loop=False, e.g.
    under a counter-collecting profiler)."""
    import numpy as np
    t = time.perf_counter()
    flat, sizes, offsets = inputs.batched_uniform(count, n, 64, 65536, seed=2, dtype=np.float32)
    log(f"batched: {count} instances, {int(sizes.sum())} rows in total, n={n} fp32 "
        f"(generated in {time.perf_counter() - t:.1f} s)")
    Ad = torch.from_numpy(flat).cuda()
    del flat
    plan = tsqr.BatchPlan(sizes, offsets, n, torch.float32)
    tiles, leaves, L = plan.info()
    R = torch.empty((count, n, n), dtype=torch.float32, device="cuda")

    def timed(fn, k, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms_batched = timed(lambda: plan.run(Ad, R), steps, warmup)
    Rb = R.clone()
    # the schedule, measured: launches with per-workgroup clock stamps (they
    # cost no measurable time), back to back after plain ones as in the timed
    # loop (a launch after an idle gap runs slower while the clocks ramp up);
    # of the last three, the one with the median span is kept
    khz = tsqr.device_clock_khz(tsqr.handle(0))
    bufs = [torch.zeros((max(tiles, 1), 2), dtype=torch.int64, device="cuda") for _ in range(5)]
    for _ in range(3):
        plan.run(Ad, R)
    for buf in bufs:
        plan.run_stamped(Ad, R, buf)
    torch.cuda.synchronize()
    runs = []
    for buf in bufs[2:]:
        st = buf.cpu().numpy()
        runs.append(((st[:, 1].max() - st[:, 0].min()) / khz, st))
    del bufs
    runs.sort(key=lambda r: r[0])
    schedule = schedule_from_stamps(np, runs[1][1], khz)
    schedule["spans_ms_of_3_launches"] = [float(r[0]) for r in runs]
    schedule["same_R_as_plain_launch"] = bool(torch.equal(R, Rb))
    log(f"batched schedule: span {schedule['span_ms']:.3f} ms on {schedule['slots']} slots, busy "
        f"{100 * schedule['busy_fraction']:.1f}%; queue empty at {schedule['last_start_ms']:.3f} ms, then "
        f"{schedule['drain_ms']:.3f} ms of drain at {schedule['mean_busy_slots_in_drain'] or 0:.0f} busy slots on average")

    # the batched launch captured in a HIP graph and replayed (checked against the eager result)
    ms_batched_graph = None
    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.run(Ad, R)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        gb = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gb):
            plan.run(Ad, R)
        ms_batched_graph = timed(gb.replay, steps, 2)
        if not torch.equal(R, Rb):
            log("batched graph replay differs from the eager launch")
            ms_batched_graph = None
        del gb
    except RuntimeError as e:
        log(f"graph capture of the batched launch failed: {e}")
    if not single_loop:
        sum_rows = int(sizes.sum())
        tflops = 2.0 * sum_rows * n * n / (ms_batched * 1e-3) / 1e12
        log(f"batched: {ms_batched:.3f} ms/step ({count / ms_batched * 1e3:.0f} instances/s, {tflops:.2f} TFLOP/s)")
        del Ad, R, plan
        torch.cuda.empty_cache()
        return {"workload": f"ragged batch {count} instances n={n} fp32", "value": count / (ms_batched * 1e-3),
                "unit": "instances/s", "ms_per_step": ms_batched, "tiles": tiles, "leaf_rows": L,
                "schedule": schedule, "plain_loop": None}
    # looped single-matrix calls over the same device data, one shared workspace
    h = tsqr.handle(0)
    views = [Ad[int(o):int(o) + int(m) * n].view(n, int(m)).t() for m, o in zip(sizes, offsets)]
    ws_bytes = max(tsqr.tsqr_workspace_bytes(h, int(m), n, tsqr.TSQR_F32) for m in set(sizes.tolist()))
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device="cuda")
    Rl = torch.empty((count, n, n), dtype=torch.float32, device="cuda")
    outs = [Rl[b].t() for b in range(count)]

    def loop():
        for b in range(count):
            tsqr.geqr_r(views[b], R=outs[b], ws=ws, h=h)

    loop_steps = max(1, min(steps, 3))
    ms_loop = timed(loop, loop_steps, 1)
    same_as_loop = None
    # the same loop captured once in a HIP graph (no per-call host overhead)
    ms_graph = None
    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            loop()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            loop()
        ms_graph = timed(g.replay, loop_steps, 1)
    except RuntimeError as e:
        log(f"graph capture of the loop failed: {e}")
    torch.cuda.synchronize()
    # each batched instance equals the corresponding single call up to the tree shape
    diff = float(((Rl - Rb).norm() / Rb.norm()).item())
    same_as_loop = diff
    sum_rows = int(sizes.sum())
    flops = 2.0 * sum_rows * n * n
    tflops = flops / (ms_batched * 1e-3) / 1e12
    gbs = 4.0 * sum_rows * n / (ms_batched * 1e-3) / 1e9
    log(f"batched: {ms_batched:.3f} ms/step ({count / ms_batched * 1e3:.0f} instances/s, {tflops:.2f} TFLOP/s); "
        f"graph replay {ms_batched_graph if ms_batched_graph is None else round(ms_batched_graph, 3)} ms; "
        f"loop {ms_loop:.2f} ms; graph loop {ms_graph if ms_graph is None else round(ms_graph, 3)} ms")
    out = {
        "workload": f"ragged batch {count} instances m log-uniform [64, 65536] (sum {sum_rows}) n={n} fp32 "
                    "uniform[-1,1) seed 2",
        "value": count / (ms_batched * 1e-3), "unit": "instances/s", "ms_per_step": ms_batched,
        "tiles": tiles, "leaf_rows": L, "schedule": schedule,
        "graph_replay": None if ms_batched_graph is None else
        {"value": count / (ms_batched_graph * 1e-3), "ms_per_step": ms_batched_graph, "steps": steps},
        "plain_loop": {"value": count / (ms_loop * 1e-3), "ms_per_step": ms_loop, "steps": loop_steps},
        "plain_loop_graph": None if ms_graph is None else
        {"value": count / (ms_graph * 1e-3), "ms_per_step": ms_graph, "steps": loop_steps},
        "speedup_vs_loop": ms_loop / ms_batched,
        "speedup_vs_graph_loop": None if ms_graph is None else ms_graph / ms_batched,
        "rel_diff_vs_plain_calls": same_as_loop,
        "roofline": {"bound": "alu", "achieved": tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP32_TFLOPS, "hbm_GBs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS},
    }
    del Ad, R, Rl, plan
    torch.cuda.empty_cache()
    return out


def time_mixed(torch, tsqr, inputs, steps, warmup, batch=256, m=1 << 16, n=50, learned=True):
    """Conditioned batch stored in FP32: FP32 TSQR + FP64 correction vs the
    plain FP64 batched TSQR (on an FP64 copy) and the FP32 TSQR alone."""
    import concurrent.futures as cf
    import numpy as np
    t = time.perf_counter()
    kappas = 10.0 ** (8.0 * np.arange(batch) / (batch - 1))
    flat = np.empty(batch * m * n, dtype=np.float32)

    def gen(i):
        flat[i * m * n:(i + 1) * m * n] = inputs.conditioned(m, n, float(kappas[i]), seed=[3, i]).T.ravel()

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as pool:
        list(pool.map(gen, range(batch)))
    log(f"mixed: {batch} instances m={m} n={n} fp32 storage, kappa 1..1e8 (generated in {time.perf_counter() - t:.1f} s)")
    Ad = torch.from_numpy(flat).cuda()
    mp = tsqr.MixedPlan(batch, m, n)

    def timed(fn, k, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    k = max(1, min(steps, 10))
    R = torch.empty((batch, n, n), dtype=torch.float64, device="cuda")
    flags = torch.zeros(batch, dtype=torch.int32, device="cuda")

    def run_mixed():
        mp.launch(Ad, R, flags)      # asynchronous: the fallback decision is taken on the device

    ms_mixed = timed(run_mixed, k, min(warmup, 3))
    Rm = R.cpu().numpy()
    Rtm = mp.rtilde().cpu().numpy()
    fallbacks = int(flags.sum().item())
    # the same correction with R~ from the FP32 TSQR of a stratified sample of
    # 4096 rows (1/16 of each instance) instead of all of A
    sample_rows = 4096
    ms_ = tsqr.MixedPlan(batch, m, n, sample_rows=sample_rows, seed=1)
    Rs_d = torch.empty((batch, n, n), dtype=torch.float64, device="cuda")
    flags_s = torch.zeros(batch, dtype=torch.int32, device="cuda")
    ms_sampled = timed(lambda: ms_.launch(Ad, Rs_d, flags_s), k, min(warmup, 3))
    Rs = Rs_d.cpu().numpy()
    Rts = ms_.rtilde().cpu().numpy()
    fallbacks_s = int(flags_s.sum().item())
    del ms_, Rs_d
    learned = [learned_vs_sampled(torch, tsqr, Ad, batch, m, n, s_, timed, k, min(warmup, 3))
               for s_ in (256, 4096)] if learned else None
    sizes = np.full(batch, m, dtype=np.int64)
    offsets = np.arange(batch, dtype=np.int64) * m * n
    p32 = tsqr.BatchPlan(sizes, offsets, n, torch.float32)
    R32 = torch.empty((batch, n, n), dtype=torch.float32, device="cuda")
    ms_32 = timed(lambda: p32.run(Ad, R32), k, min(warmup, 3))
    A64 = Ad.double()
    p64 = tsqr.BatchPlan(sizes, offsets, n, torch.float64)
    R64 = torch.empty((batch, n, n), dtype=torch.float64, device="cuda")
    ms_64 = timed(lambda: p64.run(A64, R64), k, min(warmup, 3))
    R32 = R32.cpu().numpy()
    del A64, p64, R64, Ad
    torch.cuda.empty_cache()
    flops = 2.0 * batch * m * n * n
    log(f"mixed: {ms_mixed:.2f} ms ({fallbacks} fallbacks); sampled R~ ({sample_rows} rows) {ms_sampled:.2f} ms "
        f"({fallbacks_s} fallbacks); fp64 plain {ms_64:.2f} ms; fp32 alone {ms_32:.2f} ms")
    return {
        "workload": f"{batch} instances m={m} n={n}, A = U diag(kappa^(-j/49)) V^T stored in fp32, "
                    "kappa_i = 10^(8 i/255), seeds (3, i)",
        "value": batch / (ms_mixed * 1e-3), "unit": "instances/s", "ms_per_step": ms_mixed, "steps": k,
        "fallbacks_to_fp64": fallbacks,
        "plain_fp64_batched": {"value": batch / (ms_64 * 1e-3), "ms_per_step": ms_64,
                               "note": "on an fp64 copy of the same data (conversion untimed)"},
        "fp32_tsqr_alone": {"value": batch / (ms_32 * 1e-3), "ms_per_step": ms_32},
        "speedup_vs_plain_fp64": ms_64 / ms_mixed,
        "achieved_TFLOPs_2mn2": flops / (ms_mixed * 1e-3) / 1e12,
        "sampled_rtilde": {
            "what": f"R~ from the fp32 TSQR of a stratified sample of {sample_rows} rows (64-row blocks, "
                    "seed 1), then the same fp64 correction over all of A",
            "value": batch / (ms_sampled * 1e-3), "unit": "instances/s", "ms_per_step": ms_sampled,
            "fallbacks_to_fp64": fallbacks_s, "speedup_vs_plain_fp64": ms_64 / ms_sampled},
        "learned_rtilde": learned,
    }, (flat, kappas, Rm, R32, Rtm, Rs, Rts)


def learned_vs_sampled(torch, tsqr, Ad, batch, m, n, sample_rows, timed, k, w):
    """The learned correction of the sampled R~ against the un-learned one
    with the same sample: an MLP on features of R~ (library kernels, BF16
    matrix cores), trained here on 16 generated batches of the same shape
    (G diag(sigma) V^T with Gaussian G, a different family from the
    evaluation batch's orthonormal U), then run on the evaluation batch."""
    import numpy as np
    from paper_1002_4250_amd import surrogate
    plan = tsqr.MixedPlan(batch, m, n, sample_rows=sample_rows, seed=1)
    t = time.perf_counter()
    data = surrogate.gather(plan, 16, seed=1000)
    model = surrogate.Mlp(2 * n - 1, n, H=256, seed=1)
    steps = 600
    losses = surrogate.train(model, data, steps, minibatch=128, lr=1e-3, seed=2)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    del data
    R0 = torch.empty((batch, n, n), dtype=torch.float64, device="cuda")
    R1 = torch.empty_like(R0)
    f0 = torch.zeros(batch, dtype=torch.int32, device="cuda")
    f1 = torch.zeros_like(f0)
    ms_plain = timed(lambda: plan.launch(Ad, R0, f0), k, w)
    last = [None]

    def run_learned():
        last[0] = surrogate.learned_launch(model, plan, Ad, R1, f1)

    ms_learned = timed(run_learned, k, w)
    torch.cuda.synchronize()
    # the targets of the evaluation batch: how far the network's row factors
    # are from the ones the R of A asks for, against no correction
    ev = surrogate.Dataset(surrogate.features(plan.rtilde(), batch, n).reshape(2 * n - 1, batch),
                           surrogate.targets(R0, plan.rtilde(), batch, n).reshape(n, batch))
    mse_model, mse_zero = surrogate.predict_mse(model, ev)
    R, Rt0, Rt1 = R0.cpu().numpy(), plan.rtilde().cpu().numpy(), last[-1].cpu().numpy()
    k0 = np.array([np.linalg.cond(R[b].T @ np.linalg.inv(np.triu(Rt0[b].T.astype(np.float64))))
                   for b in range(batch)])
    k1 = np.array([np.linalg.cond(R[b].T @ np.linalg.inv(np.triu(Rt1[b].T.astype(np.float64))))
                   for b in range(batch)])
    fb0, fb1 = int(f0.sum().item()), int(f1.sum().item())
    log(f"learned R~ (sample {sample_rows}): trained in {t_train:.1f} s (loss {losses[-1]:.2e}); "
        f"kappa(A R~^-1) median {np.median(k0):.3f} -> {np.median(k1):.3f}, max {k0.max():.3f} -> {k1.max():.3f}; "
        f"{ms_plain:.2f} -> {ms_learned:.2f} ms; fallbacks {fb0} -> {fb1}")
    del plan
    return {
        "sample_rows": sample_rows,
        "training": {"instances": 16 * batch, "steps": steps, "minibatch": 128, "seconds": t_train,
                     "final_loss": losses[-1]},
        "target_mse_eval_batch": {"learned": mse_model, "zero_correction": mse_zero},
        "kappa_A_Rtilde_inv": {"unlearned_median": float(np.median(k0)), "learned_median": float(np.median(k1)),
                               "unlearned_max": float(k0.max()), "learned_max": float(k1.max()),
                               "learned_lower_fraction": float(np.mean(k1 < k0))},
        "fallbacks_to_fp64": {"unlearned": fb0, "learned": fb1},
        "instances_per_s": {"unlearned": batch / (ms_plain * 1e-3), "learned": batch / (ms_learned * 1e-3)},
        "ms_per_step": {"unlearned": ms_plain, "learned": ms_learned},
    }


def mixed_accuracy(oracle, np, data, m=1 << 16, n=50, picks=(0, 64, 128, 160, 192, 224, 255)):
    """Errors against the oracle (FP64 on the stored FP32 values) for sampled
    instances across the kappa range, for the mixed result and FP32 alone:
    relF (global forward error, dominated by R's leading rows), the row-scaled
    forward error (max over rows of ||dR_i|| / ||R_i||) and the backward error
    ||R^T R - A^T A||_F / ||A||_F^2 (independent of kappa).  The last two are
    the ones that separate an FP64-accurate R from an FP32 one at high kappa.
    Every instance is checked by tests/test_gpu_full_batches.py."""
    flat, kappas, Rm, R32, Rtm, Rs, Rts = data
    out = []

    def kappa_y(Ro, Rt):
        # kappa(A R~^-1) = kappa(R R~^-1), A = Q R
        return float(np.linalg.cond(Ro @ np.linalg.inv(np.triu(Rt.T.astype(np.float64)))))

    def rows(X, Y):
        ny = np.linalg.norm(Y, axis=1)
        return float(np.max(np.linalg.norm(X - Y, axis=1) / np.where(ny > 0, ny, 1.0)))

    for i in picks:
        A = np.asfortranarray(flat[i * m * n:(i + 1) * m * n].reshape(n, m).T.astype(np.float64))
        Ro = oracle.r_factor(A)
        nr = np.linalg.norm(Ro)
        Rmi, R32i = Rm[i].T, R32[i].T.astype(np.float64)
        out.append({"kappa": float(kappas[i]),
                    "relF_mixed": float(np.linalg.norm(Rmi - Ro) / nr),
                    "relF_fp32_alone": float(np.linalg.norm(R32i - Ro) / nr),
                    "row_scaled_mixed": rows(Rmi, Ro), "row_scaled_fp32_alone": rows(R32i, Ro),
                    "backward_error_mixed": oracle.gram_residual(A, Rmi),
                    "backward_error_fp32_alone": oracle.gram_residual(A, R32i),
                    "kappa_A_Rtilde_inv_mixed": kappa_y(Ro, Rtm[i]),
                    "row_scaled_sampled": rows(Rs[i].T, Ro),
                    "backward_error_sampled": oracle.gram_residual(A, Rs[i].T),
                    "kappa_A_Rtilde_inv_sampled": kappa_y(Ro, Rts[i])})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned correction of the sampled R~ (its training launches many small kernels)")
    ap.add_argument("--no-q", action="store_true")
    ap.add_argument("--no-library", action="store_true", help="skip timing torch.linalg.qr beside the Q factor")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the shipped tuning table")
    ap.add_argument("--no-single-loop", action="store_true",
                    help="skip the loop of 4096 single-matrix calls beside the batched launch")
    ap.add_argument("--m", type=int, default=1 << 22)
    ap.add_argument("--n", type=int, default=50)
    ap.add_argument("--profile-copy-bytes", type=int, default=0,
                    help="after timing, run one plain device-to-device copy of this many bytes (the "
                         "reference kernel that calibrates the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build runs on a single MI355X); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1002_4250_amd import autotune, inputs, tsqr

    if not torch.cuda.is_available():
        log("no GPU available")
        sys.exit(1)
    m, n = args.m, args.n
    h = tsqr.handle(0)
    # the launch configuration measured by the autotuner (paper_1002_4250_amd/tuning_gfx950.json)
    tuned = 0 if args.no_tuning else autotune.apply_default(h)
    leaf_rows, leaves = tsqr.tsqr_plan_info(h, m, n, tsqr.TSQR_F64)
    log(f"workload m={m} n={n} fp64: {leaves} leaves of {leaf_rows} rows")

    A = inputs.uniform(m, n, 1)
    Ad = to_device_colmajor(torch, A)
    ms_step, ms_kernel, wall, R = time_plain(torch, tsqr, Ad, args.steps, args.warmup)
    flops = 2.0 * m * n * n
    nbytes = 8.0 * m * n + 8.0 * n * n
    tflops = flops / (ms_kernel * 1e-3) / 1e12
    gbs = nbytes / (ms_kernel * 1e-3) / 1e9
    log(f"fp64: {ms_step * 1e3:.1f} us/step, kernel {ms_kernel * 1e3:.1f} us, {tflops:.2f} TFLOP/s, {gbs:.0f} GB/s")
    R64 = R.cpu().numpy()
    phases = time_phases(torch, tsqr, Ad, flops)
    log(f"fp64 phases: leaves done at {phases['leaf_phase_end_min_ms'] * 1e3:.0f}-{phases['leaf_phase_ms'] * 1e3:.0f} us "
        f"({phases['leaf_phase_TFLOPs']:.1f} TFLOP/s), then the tree's {phases['tree_levels']} levels "
        f"{phases['tree_ms'] * 1e3:.0f} us")
    qf = None if args.no_q else time_q(torch, tsqr, Ad, args.steps, args.warmup, library=not args.no_library)

    # FP32 variant of the same workload (input = RNE rounding of the FP64 draws)
    A32 = A.astype(np.float32)
    Ad32 = to_device_colmajor(torch, A32)
    del Ad
    ms_step32, ms_kernel32, _, R32 = time_plain(torch, tsqr, Ad32, args.steps, args.warmup)
    tflops32 = flops / (ms_kernel32 * 1e-3) / 1e12
    log(f"fp32: {ms_step32 * 1e3:.1f} us/step, kernel {ms_kernel32 * 1e3:.1f} us, {tflops32:.2f} TFLOP/s")
    R32 = R32.cpu().numpy().astype(np.float64)
    del Ad32

    batched = None if args.no_batched else time_batched(torch, tsqr, inputs, args.steps, args.warmup,
                                                        single_loop=not args.no_single_loop)
    mixed, mixed_data = (None, None) if args.no_mixed else time_mixed(torch, tsqr, inputs, args.steps, args.warmup,
                                                                            learned=not args.no_learned)
    small = time_small(torch, tsqr, inputs)
    host = host_info()

    cpu = cpu_all = None
    acc64 = acc32 = None
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline: oracle on the full instance, twice (single thread)...")
        reps = 2
        t = time.perf_counter()
        for _ in range(reps):
            Ro = oracle.r_factor(A)
        dt = time.perf_counter() - t
        cpu = {"value": reps / dt, "unit": "instances/s", "cores": 1, "kind": "oracle",
               "sample": f"the full instance m={m} n={n} fp64 seed 1 factored {reps} times ({dt:.1f} s in total, "
                         "plain Householder in C, compensated sums, one thread)"}
        # the paper's method on every usable host core: block QRs in threads,
        # then the operator over a binary tree (context, not the target)
        from oracle import parallel
        cores = max(1, min(int(host["usable_cpus"] or 1), 64))
        parallel.tsqr_r_threads(A[:1 << 16], cores)         # warm the threads
        t = time.perf_counter()
        Rp = parallel.tsqr_r_threads(A, cores)
        dtp = time.perf_counter() - t
        cpu_all = {"value": 1.0 / dtp, "unit": "instances/s", "cores": cores, "kind": "oracle_tsqr_threads",
                   "sample": f"the full instance m={m} n={n} fp64 seed 1 once ({dtp:.2f} s): {cores} row blocks "
                             "factored by the oracle in parallel threads, then merged with the oracle's operator "
                             "over a binary tree",
                   "relF_vs_oracle": float(np.linalg.norm(Rp - Ro) / np.linalg.norm(Ro))}
        log(f"cpu, all {cores} cores: {dtp:.2f} s per instance")
        acc64 = float(np.linalg.norm(R64 - Ro) / np.linalg.norm(Ro))
        Ro32 = oracle.r_factor(A32.astype(np.float64))
        acc32 = float(np.linalg.norm(R32 - Ro32) / np.linalg.norm(Ro32))
        log(f"accuracy vs oracle: fp64 {acc64:.2e}, fp32 {acc32:.2e}")
        if mixed is not None:
            mixed["accuracy_vs_oracle"] = mixed_accuracy(oracle, np, mixed_data)
            log("mixed accuracy: " + ", ".join(f"k={a['kappa']:.0e}: {a['relF_mixed']:.1e} (fp32 {a['relF_fp32_alone']:.1e})"
                                                 for a in mixed["accuracy_vs_oracle"]))

    if args.profile_copy_bytes > 0:
        src = torch.empty(args.profile_copy_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    traffic = measured_traffic()
    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_step,
        "unit": "instances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"tsqr_r_factor m={m} n={n} fp64 uniform[-1,1) seed 1, one instance per step",
                   "m": m, "n": n, "leaves": leaves, "leaf_rows": leaf_rows, "parallelism": "single GPU",
                   "tuning_table_entries": tuned},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": ("tsqr_leaf_tree4_kernel<double,50,8>" if leaves % 4 == 0 and leaves >= 4
                                else "tsqr_leaf_tree_kernel<double,50,8>"), "kernel_ms": ms_kernel,
                     "hbm_GBs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS, "phases": phases},
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "host": host,
        "small_instance": small,
        "accuracy": {"fp64_relF_vs_oracle": acc64, "fp32_relF_vs_oracle": acc32,
                     "gate_fp64": 1e-10, "gate_fp32": 1e-5},
        "fp32": {"value": 1000.0 / ms_step32, "unit": "instances/s", "ms_per_step": ms_step32,
                 "kernel_ms": ms_kernel32, "achieved_TFLOPs": tflops32, "peak": PEAK_FP32_TFLOPS,
                 "frac": tflops32 / PEAK_FP32_TFLOPS},
        "batched": batched,
        "mixed": mixed,
        "q_factor": qf,
        "wall_s_timed": wall,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
