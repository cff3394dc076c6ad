"""Host-side checks of the benchmark's command-line contract and of the
autotuner's table handling (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

from paper_1002_4250_amd import autotune, tsqr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, cwd=ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_bench_without_gpu_fails_loudly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = run_bench("--steps", "1", "--warmup", "0")
    assert r.returncode != 0 and r.stdout.strip() == ""


def test_bucket_limits_cover_every_m():
    ms = autotune.M_BUCKETS
    lim = autotune.bucket_limits(ms)
    assert len(lim) == len(ms)
    assert all(m <= l for m, l in zip(ms, lim))
    assert all(a < b for a, b in zip(lim, lim[1:]))
    assert lim[-1] >= 1 << 40


def test_apply_synthetic_table_to_planning_handle(tmp_path):
    table = {"entries": [
        {"dtype": "f64", "n": 50, "m_max": 10000, "rows_per_lane": 6, "waves_per_cu": 2, "leaf_rows": 0,
         "batch": False, "us": 1.0, "candidates": [[6, 2, 1.0]]},
        {"dtype": "f32", "n": 50, "m_max": 0, "rows_per_lane": 12, "waves_per_cu": 0, "leaf_rows": 6144,
         "batch": True, "us": 1.0, "candidates": [[12, 6144, 1.0]]},
    ]}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(table))
    loaded = autotune.load(str(path))
    h = tsqr.tsqr_create_planning(256)
    plain = tsqr.tsqr_create_planning(256)
    try:
        assert autotune.apply(h, loaded) == 2
        # 10000 rows at 2 leaves per compute unit in 96-row chunks: 20-row leaves round up to one chunk
        assert tsqr.tsqr_plan_info(h, 10000, 50, tsqr.TSQR_F64) == (96, 105)
        # above the entry's m_max, and for the other element type: the built-in policy
        for m, code in ((20000, tsqr.TSQR_F64), (10000, tsqr.TSQR_F32)):
            assert tsqr.tsqr_plan_info(h, m, 50, code) == tsqr.tsqr_plan_info(plain, m, 50, code)
    finally:
        tsqr.tsqr_destroy(h)
        tsqr.tsqr_destroy(plain)
    assert autotune.load(str(tmp_path / "missing.json")) is None


def test_schedule_from_stamps_on_a_known_schedule():
    """Four slots: two 1 ms workgroups back to back on each, then one 2 ms
    workgroup alone (clock at 100 MHz, arbitrary origin)."""
    import importlib.util
    import numpy as np
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    st = np.array([(0, 1), (1, 2)] * 4 + [(2, 4)], dtype=np.int64) * 100000 + 12345
    s = bench.schedule_from_stamps(np, st, 100000)
    assert s["span_ms"] == 4.0 and s["slots"] == 4
    assert s["busy_fraction"] == 10.0 / 16.0
    assert s["last_start_ms"] == 2.0 and s["drain_ms"] == 2.0 and s["mean_busy_slots_in_drain"] == 1.0
    assert s["idle_fraction_in_drain"] == 6.0 / 16.0 and s["idle_fraction_before_drain"] == 0.0
