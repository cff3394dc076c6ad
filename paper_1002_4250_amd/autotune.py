"""Autotuner for the launch configuration of the TSQR kernels.

What it chooses, per element type and compiled column width:
  - single-matrix calls, per row-count bucket: the rows per lane of the leaf
    kernel (chunk = 16 x that many rows) and the number of leaves per compute
    unit (hence the leaf size and the depth of the reduction tree);
  - batched plans: the rows per lane and the leaf size.
Every compiled rows-per-lane value is tried with several leaf counts; each
candidate runs through the C ABI on seeded uniform[-1, 1) inputs, timed with
HIP events (median of repeated runs after a warm-up), and the fastest wins.
Candidates that give the same launch geometry are timed once.

The result is a JSON table.  `apply(h, table)` loads it into a handle's
tuning table (`tsqr_tuning_add`), after which the automatic policy of that
handle follows it; options set with `tsqr_set_option` still take precedence.
The table measured on an MI355X ships as `tuning_gfx950.json` beside this file;
`apply_default(h)` loads it.

    python -m paper_1002_4250_amd.autotune [--out PATH] [--n 50] [--quick]
"""
from __future__ import annotations

import argparse
import datetime
import json
import os
import statistics
import sys

from . import inputs, tsqr

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
DTYPES = {"f64": tsqr.TSQR_F64, "f32": tsqr.TSQR_F32}
M_BUCKETS = [1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22]
WAVES_PER_CU = [1, 2, 4, 8, 16]
BATCH_LEAF_CHUNKS = [16, 32, 64, 128, 256]
M_MAX_LAST = (1 << 62)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def bucket_limits(ms):
    """Upper bound of each bucket: the geometric midpoint to the next one."""
    out = []
    for i, m in enumerate(ms):
        out.append(int((m * ms[i + 1]) ** 0.5) if i + 1 < len(ms) else M_MAX_LAST)
    return out


def _median_ms(torch, fn, reps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune_single(torch, h, dtype_name, n, m, reps, seed=1):
    """Fastest (rows_per_lane, waves_per_cu) for one (dtype, n, m), with every
    candidate's time in microseconds."""
    import numpy as np
    code = DTYPES[dtype_name]
    A = inputs.uniform(m, n, seed)
    if dtype_name == "f32":
        A = A.astype(np.float32)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    tdt = torch.float64 if dtype_name == "f64" else torch.float32
    R = torch.empty((n, n), dtype=tdt, device="cuda").t()
    seen = {}
    results = []
    try:
        for rpl in tsqr.tsqr_rows_per_lane_compiled(code, n):
            for w in WAVES_PER_CU:
                tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_ROWS_PER_LANE, rpl)
                tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_WAVES_PER_CU, w)
                geom = (rpl,) + tsqr.tsqr_plan_info(h, m, n, code)
                if geom in seen:
                    results.append((rpl, w, seen[geom]))
                    continue
                ws = torch.empty(max(tsqr.tsqr_workspace_bytes(h, m, n, code), 256), dtype=torch.uint8,
                                 device="cuda")
                us = 1e3 * _median_ms(torch, lambda: tsqr.geqr_r(Ad, R=R, ws=ws, h=h), reps, 3)
                seen[geom] = us
                results.append((rpl, w, us))
    finally:
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_ROWS_PER_LANE, 0)
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_WAVES_PER_CU, 0)
    best = min(results, key=lambda r: r[2])
    return best, results


def tune_batch(torch, h, dtype_name, n, data, reps):
    """Fastest (rows_per_lane, leaf_rows) for a ragged batch; `data` is
    (flat FP32 host array, sizes, offsets)."""
    flat, sizes, offsets = data
    code = DTYPES[dtype_name]
    tdt = torch.float64 if dtype_name == "f64" else torch.float32
    Ad = torch.from_numpy(flat).cuda().to(tdt)
    results = []
    try:
        for rpl in tsqr.tsqr_rows_per_lane_compiled(code, n):
            for k in BATCH_LEAF_CHUNKS:
                L = 16 * rpl * k
                tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_ROWS_PER_LANE, rpl)
                tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, L)
                plan = tsqr.BatchPlan(sizes, offsets, n, tdt, h=h)
                R = torch.empty((len(sizes), n, n), dtype=tdt, device="cuda")
                us = 1e3 * _median_ms(torch, lambda: plan.run(Ad, R), reps, 2)
                results.append((rpl, L, us))
                del plan
    finally:
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_ROWS_PER_LANE, 0)
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 0)
    best = min(results, key=lambda r: r[2])
    return best, results


def tune(n=50, dtypes=("f64", "f32"), buckets=M_BUCKETS, batch_count=4096, reps=7):
    import numpy as np
    import torch
    h = tsqr.tsqr_create(0)
    entries = []
    data = None
    if batch_count:
        # the ragged batch of the batched workload: heights log-uniform in [64, 65536]
        data = inputs.batched_uniform(batch_count, n, 64, 65536, seed=2, dtype=np.float32)
    try:
        limits = bucket_limits(buckets)
        for dn in dtypes:
            for m, mmax in zip(buckets, limits):
                (rpl, w, us), cands = tune_single(torch, h, dn, n, m, reps)
                _log(f"{dn} n={n} m={m}: rows/lane {rpl}, {w} leaves/CU, {us:.1f} us")
                entries.append({"dtype": dn, "n": n, "m_max": mmax, "m_tuned": m, "rows_per_lane": rpl,
                                "waves_per_cu": w, "leaf_rows": 0, "batch": False, "us": us,
                                "candidates": [list(c) for c in cands]})
            if batch_count:
                (rpl, L, us), cands = tune_batch(torch, h, dn, n, data, max(3, reps // 2))
                _log(f"{dn} n={n} batch of {batch_count}: rows/lane {rpl}, leaf {L} rows, {us:.1f} us")
                entries.append({"dtype": dn, "n": n, "m_max": 0, "m_tuned": None, "rows_per_lane": rpl,
                                "waves_per_cu": 0, "leaf_rows": L, "batch": True, "us": us,
                                "batch_instances": batch_count, "candidates": [list(c) for c in cands]})
    finally:
        tsqr.tsqr_destroy(h)
    return {"device": "gfx950", "created": datetime.date.today().isoformat(),
            "method": "median of HIP-event timings per candidate; seeded uniform[-1,1) inputs",
            "entries": entries}


def apply(h, table) -> int:
    """Load a table into the handle's tuning table; returns the entries applied."""
    k = 0
    for e in table.get("entries", []):
        tsqr.tsqr_tuning_add(h, DTYPES[e["dtype"]], e["n"], e["m_max"], e["rows_per_lane"], e["waves_per_cu"],
                             e["leaf_rows"], e["batch"])
        k += 1
    return k


def load(path=DEFAULT_TABLE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def apply_default(h) -> int:
    """Apply the shipped table, if present; returns the entries applied."""
    table = load()
    return apply(h, table) if table else 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--n", type=int, default=50)
    ap.add_argument("--quick", action="store_true", help="fewer buckets and repetitions (a smoke run)")
    args = ap.parse_args()
    if args.quick:
        table = tune(n=args.n, buckets=[1 << 12, 1 << 16], batch_count=256, reps=3)
    else:
        table = tune(n=args.n)
    table["command"] = "python -m paper_1002_4250_amd.autotune" + (" --quick" if args.quick else "") + \
        (f" --n {args.n}" if args.n != 50 else "")
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    _log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
