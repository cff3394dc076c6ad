"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/tsqr.h declares, and its planning and argument checks behave
as documented."""
import ctypes
import os
import re

import pytest

from paper_1002_4250_amd import tsqr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsqr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsqr_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(tsqr.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's functions
    assert sorted(n for n, _, _ in tsqr.SIGNATURES) == names


def test_header_constants_match_binding():
    text = open(HEADER).read()
    for name in ("TSQR_MAX_N", "TSQR_F64", "TSQR_F32", "TSQR_ERR_HIP", "TSQR_ERR_UNSUPPORTED",
                 "TSQR_ERR_NO_DEVICE", "TSQR_ERR_ALLOC", "TSQR_ERR_SCRATCH", "TSQR_OPT_LEAF_ROWS",
                 "TSQR_OPT_ROWS_PER_LANE", "TSQR_OPT_WAVES_PER_CU"):
        m = re.search(r"#define\s+%s\s+(\d+)" % name, text)
        assert m and int(m.group(1)) == getattr(tsqr, name), name
    m = re.search(r"#define\s+TSQR_NOALLOC_SCRATCH_BYTES\s+\(\(int64_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == tsqr.TSQR_NOALLOC_SCRATCH_BYTES


@pytest.fixture
def ph():
    h = tsqr.tsqr_create_planning(256)
    yield h
    tsqr.tsqr_destroy(h)


def test_null_handle_is_argument_one():
    L = tsqr.lib()
    assert L.tsqr_geqr_r_f64(None, 10, 2, None, 10, None, 2, None, 0, None) == -1
    assert L.tsqr_qr_uppers_f32(None, 4, None, None, None, None) == -1
    assert L.tsqr_workspace_bytes(None, 10, 2, 0) == -1
    assert L.tsqr_create(None, 0) == -1
    assert L.tsqr_set_option(None, 1, 0) == -1


def test_status_strings():
    assert tsqr.lib().tsqr_status_string(0) == b"success"
    assert b"invalid" in tsqr.lib().tsqr_status_string(-3)
    assert b"gfx950" in tsqr.lib().tsqr_status_string(tsqr.TSQR_ERR_NO_DEVICE)


def test_argument_checks_in_order(ph):
    L = tsqr.lib()
    f = L.tsqr_geqr_r_f64
    A, R, W = 4096, 8192, 256 * 1024
    assert f(ph, -1, 5, A, 10, R, 5, W, 1 << 30, None) == -2
    assert f(ph, 10, -1, A, 10, R, 5, W, 1 << 30, None) == -3
    assert f(ph, 10, 5, None, 10, R, 5, W, 1 << 30, None) == -4
    assert f(ph, 10, 5, A, 9, R, 5, W, 1 << 30, None) == -5
    assert f(ph, 10, 5, A, 10, None, 5, W, 1 << 30, None) == -6
    assert f(ph, 10, 5, A, 10, R, 4, W, 1 << 30, None) == -7
    assert f(ph, 10, 5, A, 10, R, 5, None, 1 << 30, None) == -8
    assert f(ph, 10, 5, A, 10, R, 5, W + 8, 1 << 30, None) == -8      # misaligned workspace
    need = tsqr.tsqr_workspace_bytes(ph, 10, 5, tsqr.TSQR_F64)
    assert f(ph, 10, 5, A, 10, R, 5, W, need - 1, None) == -9
    # all arguments valid: a planning handle stops before any HIP call
    assert f(ph, 10, 5, A, 10, R, 5, W, need, None) == tsqr.TSQR_ERR_NO_DEVICE
    assert f(ph, 10, 65, A, 10, R, 65, W, 1 << 30, None) == tsqr.TSQR_ERR_UNSUPPORTED
    assert f(ph, 10, 0, None, 10, None, 1, None, 0, None) == 0          # n = 0 is a no-op
    g = L.tsqr_qr_uppers_f64
    assert g(ph, -1, R, R, R, None) == -2
    assert g(ph, 3, None, R, R, None) == -3
    assert g(ph, 3, R, None, R, None) == -4
    assert g(ph, 3, R, R, None, None) == -5
    assert g(ph, 65, R, R, R, None) == tsqr.TSQR_ERR_UNSUPPORTED
    assert g(ph, 3, R, R, R, None) == tsqr.TSQR_ERR_NO_DEVICE


def test_plan_geometry(ph):
    # m = 2^22, n = 50 in FP64: leaves of whole chunks, about 4 per compute unit
    lr, P = tsqr.tsqr_plan_info(ph, 1 << 22, 50, tsqr.TSQR_F64)
    assert lr * P >= 1 << 22 and lr * (P - 1) < 1 << 22
    assert 256 * 2 <= P <= 256 * 8
    chunk = 16 * 8
    assert lr % chunk == 0
    ws = tsqr.tsqr_workspace_bytes(ph, 1 << 22, 50, tsqr.TSQR_F64)
    assert ws >= P * 4 + P * (50 * 51 // 2) * 8 and ws % 256 == 0
    # tiny m: one leaf of one chunk
    lr, P = tsqr.tsqr_plan_info(ph, 1, 3, tsqr.TSQR_F32)
    assert P == 1 and lr == 16 * 8
    # forced leaf size, rounded up to a chunk
    tsqr.tsqr_set_option(ph, tsqr.TSQR_OPT_LEAF_ROWS, 100)
    lr, P = tsqr.tsqr_plan_info(ph, 1000, 50, tsqr.TSQR_F64)
    assert lr == 128 and P == 8
    tsqr.tsqr_set_option(ph, tsqr.TSQR_OPT_LEAF_ROWS, 0)
    # m = 0 still has one (empty) leaf so that R = 0 is written
    assert tsqr.tsqr_plan_info(ph, 0, 7, tsqr.TSQR_F64)[1] == 1
    with pytest.raises(tsqr.TsqrError):
        tsqr.tsqr_plan_info(ph, 10, 65, tsqr.TSQR_F64)
    assert tsqr.lib().tsqr_set_option(ph, 99, 1) == -2
    assert tsqr.lib().tsqr_set_option(ph, 1, -5) == -3


def test_workspace_query_errors(ph):
    L = tsqr.lib()
    assert L.tsqr_workspace_bytes(ph, -1, 5, 0) == -2
    assert L.tsqr_workspace_bytes(ph, 5, -1, 0) == -3
    assert L.tsqr_workspace_bytes(ph, 5, 5, 7) == -4
    assert L.tsqr_workspace_bytes(ph, 5, 0, 0) == 0
    assert L.tsqr_workspace_bytes(ph, 5, 65, 0) == -1000 - tsqr.TSQR_ERR_UNSUPPORTED


def test_create_without_gpu_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert tsqr.lib().tsqr_create(ctypes.byref(h), 0) == tsqr.TSQR_ERR_NO_DEVICE
    assert not h.value


def _batch_create(h, sizes, n, dtype=tsqr.TSQR_F64, offsets=None, lda=None):
    import numpy as np
    sizes = np.asarray(sizes, dtype=np.int64)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum(sizes * n)[:-1]]).astype(np.int64) if len(sizes) else sizes
    return tsqr.tsqr_batch_plan_create(h, len(sizes), n, sizes, offsets, lda, dtype)


def test_batch_plan_tiles_and_workspace(ph):
    # ragged sizes: each instance is cut into ceil(m/L) leaves of L rows
    # (m = 0 still has one empty leaf that writes a zero R)
    sizes = [64, 1000, 0, 1, 65536, 4097]
    p = _batch_create(ph, sizes, 50)
    try:
        tiles, leaves, L = tsqr.tsqr_batch_plan_info(p)
        assert L == 64 * 16 * 8
        want = sum(max(1, -(-m // L)) for m in sizes)
        assert tiles == leaves == want
        tri = 50 * 51 // 2
        align = lambda x: (x + 255) // 256 * 256
        assert tsqr.tsqr_batch_workspace_bytes(p) == align(4 * leaves) + align(8 * tri * leaves)
    finally:
        tsqr.tsqr_batch_plan_destroy(p)
    # fp32 and a handle leaf size
    tsqr.tsqr_set_option(ph, tsqr.TSQR_OPT_LEAF_ROWS, 1000)
    p = _batch_create(ph, sizes, 16, tsqr.TSQR_F32)
    try:
        tiles, leaves, L = tsqr.tsqr_batch_plan_info(p)
        assert L == 1024
        assert tiles == sum(max(1, -(-m // 1024)) for m in sizes)
        assert tsqr.tsqr_batch_workspace_bytes(p) == (4 * tiles + 255) // 256 * 256 + \
            (4 * 136 * tiles + 255) // 256 * 256
    finally:
        tsqr.tsqr_batch_plan_destroy(p)


def _expected_schedule(sizes, offsets, ldas, L, tri):
    """The schedule enumerated from its definition: instance b is cut into
    max(1, ceil(m_b / L)) leaves of L rows (the last one ragged); its tree
    counters and triangle slots follow those of the instances before it; the
    tiles go out longest first, ties in (instance, leaf) order."""
    import numpy as np
    inst, tiles, first = [], [], 0
    for b, m in enumerate(sizes):
        P = max(1, -(-m // L))
        inst.append([offsets[b], m, ldas[b], L, P, first, first * tri])
        tiles += [(max(0, min(L, m - i * L)), b, i) for i in range(P)]
        first += P
    order = sorted(range(len(tiles)), key=lambda k: -tiles[k][0])      # sorted() is stable
    return (np.array(inst, dtype=np.int64).reshape(-1, 7),
            np.array([[tiles[k][1], tiles[k][2]] for k in order], dtype=np.int64).reshape(-1, 2))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_plan_schedule_is_bit_exact(ph, dtype):
    """The tile table and the per-instance table of a plan, read back from the
    library, equal an independent enumeration from their definition, entry
    for entry, on the ragged batch of the batched workload (4096 instances,
    heights log-uniform in [64, 65536]) with an lda above m and gaps between
    the instances."""
    import numpy as np
    from paper_1002_4250_amd import inputs
    sizes = [int(v) for v in inputs.batched_sizes()]
    n = 50
    ldas = [m + 7 for m in sizes]
    offsets, off = [], 0
    for m, ld in zip(sizes, ldas):
        offsets.append(off)
        off += ld * n + 13
    dt = tsqr.TSQR_F64 if dtype == "f64" else tsqr.TSQR_F32
    arr = lambda v: (ctypes.c_int64 * len(v))(*v)
    plan = ctypes.c_void_p()
    st = tsqr.lib().tsqr_batch_plan_create(ph, len(sizes), n, arr(sizes), arr(offsets), arr(ldas), dt,
                                           ctypes.byref(plan))
    assert st == 0
    try:
        tiles, leaves, L = tsqr.tsqr_batch_plan_info(plan.value)
        inst, sched = tsqr.tsqr_batch_plan_schedule(plan.value, len(sizes))
        want_inst, want_sched = _expected_schedule(sizes, offsets, ldas, L, n * (n + 1) // 2)
        assert leaves == want_inst[:, 4].sum() and tiles == len(want_sched)
        assert np.array_equal(inst, want_inst)
        assert np.array_equal(sched, want_sched)
    finally:
        tsqr.tsqr_batch_plan_destroy(plan.value)
    assert tsqr.lib().tsqr_batch_plan_schedule(None, None, None) == -1


def test_batch_plan_argument_checks(ph):
    import numpy as np
    L = tsqr.lib()
    P = ctypes.POINTER(ctypes.c_int64)
    m = (ctypes.c_int64 * 2)(10, 20)
    off = (ctypes.c_int64 * 2)(0, 100)
    out = ctypes.c_void_p()
    assert L.tsqr_batch_plan_create(None, 2, 4, m, off, None, 0, ctypes.byref(out)) == -1
    assert L.tsqr_batch_plan_create(ph, -1, 4, m, off, None, 0, ctypes.byref(out)) == -2
    assert L.tsqr_batch_plan_create(ph, 2, -1, m, off, None, 0, ctypes.byref(out)) == -3
    assert L.tsqr_batch_plan_create(ph, 2, 4, None, off, None, 0, ctypes.byref(out)) == -4
    bad_m = (ctypes.c_int64 * 2)(10, -1)
    assert L.tsqr_batch_plan_create(ph, 2, 4, bad_m, off, None, 0, ctypes.byref(out)) == -4
    assert L.tsqr_batch_plan_create(ph, 2, 4, m, None, None, 0, ctypes.byref(out)) == -5
    bad_off = (ctypes.c_int64 * 2)(0, -5)
    assert L.tsqr_batch_plan_create(ph, 2, 4, m, bad_off, None, 0, ctypes.byref(out)) == -5
    bad_lda = (ctypes.c_int64 * 2)(10, 19)
    assert L.tsqr_batch_plan_create(ph, 2, 4, m, off, bad_lda, 0, ctypes.byref(out)) == -6
    assert L.tsqr_batch_plan_create(ph, 2, 4, m, off, None, 7, ctypes.byref(out)) == -7
    assert L.tsqr_batch_plan_create(ph, 2, 4, m, off, None, 0, None) == -8
    assert L.tsqr_batch_plan_create(ph, 2, 65, m, off, None, 0, ctypes.byref(out)) == tsqr.TSQR_ERR_UNSUPPORTED
    # exec checks on a planning handle's plan
    assert L.tsqr_batch_plan_create(ph, 2, 4, m, off, None, 0, ctypes.byref(out)) == 0
    p = out.value
    try:
        need = L.tsqr_batch_workspace_bytes(p)
        buf = ctypes.create_string_buffer(need + 512)
        ws = (ctypes.addressof(buf) + 255) // 256 * 256
        assert L.tsqr_batch_exec(None, 1, 1, 4, ws, need, None) == -1
        assert L.tsqr_batch_exec(p, None, 1, 4, ws, need, None) == -2
        assert L.tsqr_batch_exec(p, 1, None, 4, ws, need, None) == -3
        assert L.tsqr_batch_exec(p, 1, 1, 3, ws, need, None) == -4
        assert L.tsqr_batch_exec(p, 1, 1, 4, None, need, None) == -5
        assert L.tsqr_batch_exec(p, 1, 1, 4, ws + 8, need, None) == -5
        assert L.tsqr_batch_exec(p, 1, 1, 4, ws, need - 1, None) == -6
        assert L.tsqr_batch_exec(p, 1, 1, 4, ws, need, None) == tsqr.TSQR_ERR_NO_DEVICE
    finally:
        L.tsqr_batch_plan_destroy(p)
    assert L.tsqr_batch_workspace_bytes(None) == -1
    assert L.tsqr_batch_plan_destroy(None) == 0


def test_batch_plan_empty(ph):
    import numpy as np
    p = tsqr.tsqr_batch_plan_create(ph, 0, 50, np.zeros(0, np.int64), np.zeros(0, np.int64), None, 0)
    try:
        assert tsqr.tsqr_batch_plan_info(p) == (0, 0, 64 * 16 * 8)
        # nothing to do: succeeds without touching any pointer
        assert tsqr.lib().tsqr_batch_exec(p, None, None, 50, None, 0, None) == 0
    finally:
        tsqr.tsqr_batch_plan_destroy(p)


def test_mixed_plan_checks_and_workspace(ph):
    L = tsqr.lib()
    out = ctypes.c_void_p()
    assert L.tsqr_mixed_plan_create(None, 2, 100, 8, 100, 800, ctypes.byref(out)) == -1
    assert L.tsqr_mixed_plan_create(ph, -1, 100, 8, 100, 800, ctypes.byref(out)) == -2
    assert L.tsqr_mixed_plan_create(ph, 2, -1, 8, 100, 800, ctypes.byref(out)) == -3
    assert L.tsqr_mixed_plan_create(ph, 2, 100, -1, 100, 800, ctypes.byref(out)) == -4
    assert L.tsqr_mixed_plan_create(ph, 2, 100, 8, 99, 800, ctypes.byref(out)) == -5
    assert L.tsqr_mixed_plan_create(ph, 2, 100, 8, 100, 799, ctypes.byref(out)) == -6
    assert L.tsqr_mixed_plan_create(ph, 2, 100, 8, 100, 800, None) == -7
    assert L.tsqr_mixed_plan_create(ph, 2, 100, 65, 100, 6500, ctypes.byref(out)) == tsqr.TSQR_ERR_UNSUPPORTED
    p = tsqr.tsqr_mixed_plan_create(ph, 3, 10000, 50, 10000, 500000)
    try:
        need = tsqr.tsqr_mixed_workspace_bytes(p)
        # FP32 batch workspace + R~ + Gram slots (one 52 x 52 slot per
        # workgroup) + flags + the FP64 fallback's batched workspace (a
        # triangle per leaf); no FP64 copy of any instance (the fallback reads
        # the FP32 storage)
        assert 3 * 52 * 52 * 8 + 3 * 1275 * 8 < need < 10000 * 50 * 8
        # R~ sits past the FP32 workspace, inside the workspace
        off = tsqr.tsqr_mixed_rtilde_offset(p)
        assert 0 <= off and off + 3 * 50 * 50 * 4 <= need
        buf = ctypes.create_string_buffer(need + 512)
        ws = (ctypes.addressof(buf) + 255) // 256 * 256
        assert L.tsqr_mixed_exec(None, 1, 1, 50, None, ws, need, None) == -1
        assert L.tsqr_mixed_exec(p, None, 1, 50, None, ws, need, None) == -2
        assert L.tsqr_mixed_exec(p, 1, None, 50, None, ws, need, None) == -3
        assert L.tsqr_mixed_exec(p, 1, 1, 49, None, ws, need, None) == -4
        assert L.tsqr_mixed_exec(p, 1, 1, 50, None, None, need, None) == -6
        assert L.tsqr_mixed_exec(p, 1, 1, 50, None, ws, need - 1, None) == -7
        assert L.tsqr_mixed_exec(p, 1, 1, 50, None, ws, need, None) == tsqr.TSQR_ERR_NO_DEVICE
    finally:
        tsqr.tsqr_mixed_plan_destroy(p)
    assert L.tsqr_mixed_workspace_bytes(None) == -1
    assert L.tsqr_mixed_rtilde_offset(None) == -1


def test_sampled_mixed_plan_checks_and_workspace(ph):
    L = tsqr.lib()
    out = ctypes.c_void_p()
    args = (2, 100, 8, 100, 800)
    assert L.tsqr_mixed_plan_create_sampled(None, *args, 32, 1, ctypes.byref(out)) == -1
    assert L.tsqr_mixed_plan_create_sampled(ph, -1, 100, 8, 100, 800, 32, 1, ctypes.byref(out)) == -2
    assert L.tsqr_mixed_plan_create_sampled(ph, 2, -1, 8, 100, 800, 32, 1, ctypes.byref(out)) == -3
    assert L.tsqr_mixed_plan_create_sampled(ph, 2, 100, -1, 100, 800, 32, 1, ctypes.byref(out)) == -4
    assert L.tsqr_mixed_plan_create_sampled(ph, 2, 100, 8, 99, 800, 32, 1, ctypes.byref(out)) == -5
    assert L.tsqr_mixed_plan_create_sampled(ph, 2, 100, 8, 100, 799, 32, 1, ctypes.byref(out)) == -6
    assert L.tsqr_mixed_plan_create_sampled(ph, *args, -1, 1, ctypes.byref(out)) == -7
    assert L.tsqr_mixed_plan_create_sampled(ph, *args, 32, 1, None) == -9
    full = tsqr.tsqr_mixed_plan_create(ph, 4, 65536, 50, 65536, 65536 * 50)
    samp = tsqr.tsqr_mixed_plan_create_sampled(ph, 4, 65536, 50, 65536, 65536 * 50, 4000, 7)
    # a sample of at least m rows (after rounding to 16) is the plain plan
    same = tsqr.tsqr_mixed_plan_create_sampled(ph, 4, 65536, 50, 65536, 65536 * 50, 65530, 7)
    try:
        wf = tsqr.tsqr_mixed_workspace_bytes(full)
        ws_ = tsqr.tsqr_mixed_workspace_bytes(samp)
        assert tsqr.tsqr_mixed_workspace_bytes(same) == wf
        # the sample buffer (4 x 4000 x 50 FP32) is added; the FP32
        # factorization of the samples (short leaves, a triangle each) needs
        # at most a few MB more
        assert ws_ >= 4 * 4000 * 50 * 4
        assert ws_ < wf + 4 * 4000 * 50 * 4 + (4 << 20)
    finally:
        for p in (full, samp, same):
            tsqr.tsqr_mixed_plan_destroy(p)


def test_qr_workspace_query(ph):
    L = tsqr.lib()
    F64, F32 = tsqr.TSQR_F64, tsqr.TSQR_F32
    assert L.tsqr_qr_workspace_bytes(None, 100, 10, F64) == -1
    assert L.tsqr_qr_workspace_bytes(ph, -1, 10, F64) == -2
    assert L.tsqr_qr_workspace_bytes(ph, 10, 11, F64) == -3
    assert L.tsqr_qr_workspace_bytes(ph, 100, 10, 7) == -4
    assert L.tsqr_qr_workspace_bytes(ph, 100, 0, F64) == 0
    assert L.tsqr_qr_workspace_bytes(ph, 100, 65, F64) == -1000 - tsqr.TSQR_ERR_UNSUPPORTED
    m, n = 100000, 50
    for code, w, fn in ((F64, 8, L.tsqr_geqr_qr_f64), (F32, 4, L.tsqr_geqr_qr_f32)):
        r_only = tsqr.tsqr_workspace_bytes(ph, m, n, code)
        need = tsqr.tsqr_qr_workspace_bytes(ph, m, n, code)
        assert need >= r_only + w * m * n and need % 256 == 0
        assert fn(ph, m, n, 1, m, 1, m, 1, n, None, need, None) == -10
        assert fn(ph, m, n, 1, m, 1, m, 1, n, 256, need - 1, None) == -11
        assert fn(ph, m, n, 1, m, 1, m, 1, n, 256, need, None) == tsqr.TSQR_ERR_NO_DEVICE
    assert tsqr.tsqr_qr_workspace_bytes(ph, m, n, F32) < tsqr.tsqr_qr_workspace_bytes(ph, m, n, F64)


def test_geqrf_and_apply_qt_argument_checks(ph):
    L = tsqr.lib()
    F64, F32 = tsqr.TSQR_F64, tsqr.TSQR_F32
    m, n = 100000, 50
    for code, geqrf, apply in ((F64, L.tsqr_geqrf_f64, L.tsqr_apply_qt_f64),
                               (F32, L.tsqr_geqrf_f32, L.tsqr_apply_qt_f32)):
        need = tsqr.tsqr_qr_workspace_bytes(ph, m, n, code)
        # the workspace also holds one n x 64 block per leaf for apply_qt
        leaves = tsqr.tsqr_plan_info(ph, m, n, code)[1]
        assert need >= leaves * n * 64 * (8 if code == F64 else 4)
        assert geqrf(None, m, n, 1, m, 1, n, 256, need, None) == -1
        assert geqrf(ph, -1, n, 1, m, 1, n, 256, need, None) == -2
        assert geqrf(ph, m, m + 1, 1, m, 1, n, 256, need, None) == -3
        assert geqrf(ph, m, n, None, m, 1, n, 256, need, None) == -4
        assert geqrf(ph, m, n, 1, m - 1, 1, n, 256, need, None) == -5
        assert geqrf(ph, m, n, 1, m, None, n, 256, need, None) == -6
        assert geqrf(ph, m, n, 1, m, 1, n - 1, 256, need, None) == -7
        assert geqrf(ph, m, n, 1, m, 1, n, None, need, None) == -8
        assert geqrf(ph, m, n, 1, m, 1, n, 256, need - 1, None) == -9
        assert geqrf(ph, m, n, 1, m, 1, n, 256, need, None) == tsqr.TSQR_ERR_NO_DEVICE
        k = 3
        assert apply(None, m, n, k, 1, m, 1, n, 256, need, None) == -1
        assert apply(ph, -1, n, k, 1, m, 1, n, 256, need, None) == -2
        assert apply(ph, m, m + 1, k, 1, m, 1, n, 256, need, None) == -3
        assert apply(ph, m, n, -1, 1, m, 1, n, 256, need, None) == -4
        assert apply(ph, m, n, k, None, m, 1, n, 256, need, None) == -5
        assert apply(ph, m, n, k, 1, m - 1, 1, n, 256, need, None) == -6
        assert apply(ph, m, n, k, 1, m, None, n, 256, need, None) == -7
        assert apply(ph, m, n, k, 1, m, 1, n - 1, 256, need, None) == -8
        assert apply(ph, m, n, k, 1, m, 1, n, None, need, None) == -9
        assert apply(ph, m, n, k, 1, m, 1, n, 256, need - 1, None) == -10
        assert apply(ph, m, n, k, 1, m, 1, n, 256, need, None) == tsqr.TSQR_ERR_NO_DEVICE
        # nothing to do: no checks of the pointers, no device needed
        assert apply(ph, m, n, 0, None, m, None, n, None, 0, None) == 0
        assert apply(ph, m, 65, k, 1, m, 1, 65, 256, need, None) == tsqr.TSQR_ERR_UNSUPPORTED


def test_tuning_table_steers_the_automatic_policy(ph):
    F64, F32 = tsqr.TSQR_F64, tsqr.TSQR_F32
    base = {m: tsqr.tsqr_plan_info(ph, m, 50, F64) for m in (1 << 16, 1 << 18, 1 << 20, 1 << 21)}
    # m <= 2^20: rows per lane 8, 8 leaves per compute unit
    tsqr.tsqr_tuning_add(ph, F64, 50, 1 << 20, 8, 8, 0, False)
    assert tsqr.tsqr_plan_info(ph, 1 << 20, 50, F64) == (512, 2048)
    assert tsqr.tsqr_plan_info(ph, 1 << 21, 50, F64) == base[1 << 21]        # above every m_max
    assert tsqr.tsqr_plan_info(ph, 1 << 20, 50, F32) == tsqr.tsqr_plan_info(ph, 1 << 20, 49, F32)
    # the smallest m_max that covers m wins; an explicit leaf size is rounded to
    # the entry's chunk (16 x 4 rows)
    tsqr.tsqr_tuning_add(ph, F64, 50, 1 << 16, 4, 0, 1000, False)
    assert tsqr.tsqr_plan_info(ph, 1 << 16, 50, F64) == (1024, 64)
    assert tsqr.tsqr_plan_info(ph, 1 << 18, 50, F64) == (128, 2048)
    # every column count that pads to the same compiled width shares the entry
    assert tsqr.tsqr_plan_info(ph, 1 << 16, 33, F64) == (1024, 64)
    assert tsqr.tsqr_plan_info(ph, 1 << 16, 16, F64) != (1024, 64)
    # handle options take precedence over the table
    tsqr.tsqr_set_option(ph, tsqr.TSQR_OPT_LEAF_ROWS, 256)
    assert tsqr.tsqr_plan_info(ph, 1 << 16, 50, F64) == (256, 256)
    tsqr.tsqr_set_option(ph, tsqr.TSQR_OPT_LEAF_ROWS, 0)
    # an entry with the same key replaces the earlier one
    tsqr.tsqr_tuning_add(ph, F64, 50, 1 << 16, 8, 0, 2048, False)
    assert tsqr.tsqr_plan_info(ph, 1 << 16, 50, F64) == (2048, 32)
    # batched plans take the batched entry (rows per lane 16: 256-row chunks)
    tsqr.tsqr_tuning_add(ph, F32, 50, 0, 16, 0, 4000, True)
    p = _batch_create(ph, [5000, 100, 9000], 50, tsqr.TSQR_F32)
    try:
        tiles, leaves, L = tsqr.tsqr_batch_plan_info(p)
        assert L == 4096 and tiles == 2 + 1 + 3
    finally:
        tsqr.tsqr_batch_plan_destroy(p)
    p = _batch_create(ph, [5000], 50, tsqr.TSQR_F64)          # no FP64 batched entry
    try:
        assert tsqr.tsqr_batch_plan_info(p)[2] == 64 * 16 * 8
    finally:
        tsqr.tsqr_batch_plan_destroy(p)
    # clearing restores the built-in policy
    tsqr.tsqr_tuning_clear(ph)
    for m, g in base.items():
        assert tsqr.tsqr_plan_info(ph, m, 50, F64) == g


def test_tuning_argument_checks(ph):
    L = tsqr.lib()
    F64, F32 = tsqr.TSQR_F64, tsqr.TSQR_F32
    assert L.tsqr_tuning_add(None, F64, 50, 10, 8, 0, 0, 0) == -1
    assert L.tsqr_tuning_add(ph, 7, 50, 10, 8, 0, 0, 0) == -2
    assert L.tsqr_tuning_add(ph, F64, 0, 10, 8, 0, 0, 0) == -3
    assert L.tsqr_tuning_add(ph, F64, 65, 10, 8, 0, 0, 0) == -3
    assert L.tsqr_tuning_add(ph, F64, 50, -1, 8, 0, 0, 0) == -4
    assert L.tsqr_tuning_add(ph, F64, 50, 10, 5, 0, 0, 0) == -5       # not compiled
    assert L.tsqr_tuning_add(ph, F64, 50, 10, 0, 0, 0, 0) == -5
    assert L.tsqr_tuning_add(ph, F64, 50, 10, 8, -1, 0, 0) == -6
    assert L.tsqr_tuning_add(ph, F64, 50, 10, 8, 0, -1, 0) == -7
    assert L.tsqr_tuning_clear(None) == -1
    assert tsqr.tsqr_rows_per_lane_compiled(F64, 50) == [4, 6, 8]
    assert tsqr.tsqr_rows_per_lane_compiled(F32, 50) == [8, 12, 16]
    assert tsqr.tsqr_rows_per_lane_compiled(F64, 9) == [8]
    assert L.tsqr_rows_per_lane_compiled(7, 50, None, 0) == -1
    assert L.tsqr_rows_per_lane_compiled(F64, 65, None, 0) == -2
    assert L.tsqr_rows_per_lane_compiled(F64, 50, None, 1) == -3
    assert L.tsqr_rows_per_lane_compiled(F64, 50, None, 0) == 3


def test_shipped_tuning_table_applies(ph):
    from paper_1002_4250_amd import autotune
    table = autotune.load()
    if table is None:
        pytest.skip("no tuning table shipped")
    assert autotune.apply(ph, table) == len(table["entries"]) > 0
    for e in table["entries"]:
        # each entry is the fastest of the candidates it records
        assert e["us"] == min(c[2] for c in e["candidates"]), e["dtype"]
        assert e["rows_per_lane"] in tsqr.tsqr_rows_per_lane_compiled(autotune.DTYPES[e["dtype"]], e["n"])
    singles = sorted(e["m_max"] for e in table["entries"] if not e["batch"] and e["dtype"] == "f64")
    assert singles == sorted(set(singles)) and singles[-1] >= 1 << 40


def test_binding_refuses_wrong_tensors():
    torch = pytest.importorskip("torch")
    cpu = torch.device("cpu")
    R = torch.empty((5, 5), dtype=torch.float64).t()
    assert tsqr._check_matrix(R, "R", 5, 5, torch.float64, cpu) == 5
    wide = torch.empty((5, 7), dtype=torch.float64).t()[:5, :]     # leading dimension 7
    assert tsqr._check_matrix(wide, "R", 5, 5, torch.float64, cpu) == 7
    with pytest.raises(TypeError):
        tsqr._check_matrix(R.float(), "R", 5, 5, torch.float64, cpu)
    with pytest.raises(ValueError):
        tsqr._check_matrix(torch.empty((5, 5), dtype=torch.float64), "R", 5, 5, torch.float64, cpu)  # row-major
    with pytest.raises(ValueError):
        tsqr._check_matrix(R[:4, :], "R", 5, 5, torch.float64, cpu)
    col = torch.empty((3, 8), dtype=torch.float64)[:, 0:1]           # a strided column
    with pytest.raises(ValueError):
        tsqr._check_matrix(col, "Q", 3, 1, torch.float64, cpu)
    # input matrices: an expanded or overlapping view has a column stride below
    # m, and the kernels would read m*n elements from a smaller allocation
    assert tsqr._col_major(torch.empty((50, 1000), dtype=torch.float64).t()) == (1000, 50, 1000)
    assert tsqr._col_major(torch.empty((50, 1200), dtype=torch.float64).t()[:1000, :]) == (1000, 50, 1200)
    with pytest.raises(ValueError):
        tsqr._col_major(torch.zeros(1000, 1, dtype=torch.float64).expand(1000, 50))
    with pytest.raises(ValueError):
        tsqr._col_major(torch.zeros(2000, dtype=torch.float64).as_strided((1000, 50), (1, 10)))
    with pytest.raises(ValueError):
        tsqr._col_major(torch.empty((1000, 50), dtype=torch.float64))          # row-major
    assert tsqr._col_major(torch.zeros(1000, 1, dtype=torch.float64)) == (1000, 1, 1000)
    flat = torch.empty(100, dtype=torch.float32)
    tsqr._check_flat(flat, "A", 100, torch.float32, cpu)
    with pytest.raises(ValueError):
        tsqr._check_flat(flat, "A", 101, torch.float32, cpu)
    with pytest.raises(ValueError):
        tsqr._check_flat(flat[::2], "A", 10, torch.float32, cpu)
    with pytest.raises(TypeError):
        tsqr._check_flat(flat, "A", 10, torch.float64, cpu)


def test_noalloc_entry_point_checks_on_the_host(ph):
    """Argument codes, the scratch limit (checked from the plan, before any
    launch) and the planning-only handle, without a GPU."""
    L = tsqr.lib()
    f = L.tsqr_geqr_r_f64_noalloc
    A, R = 4096, 8192             # placeholder addresses: nothing is launched on this handle
    assert f(None, 10, 2, A, 10, R, 2, None) == -1
    assert f(ph, -1, 2, A, 10, R, 2, None) == -2
    assert f(ph, 10, -2, A, 10, R, 2, None) == -3
    assert f(ph, 10, 2, None, 10, R, 2, None) == -4
    assert f(ph, 10, 2, A, 9, R, 2, None) == -5
    assert f(ph, 10, 2, A, 10, None, 2, None) == -6
    assert f(ph, 10, 2, A, 10, R, 1, None) == -7
    assert f(ph, 10, 0, A, 10, R, 1, None) == 0
    assert f(ph, 1 << 22, 50, A, 1 << 22, R, 50, None) == tsqr.TSQR_ERR_NO_DEVICE
    assert f(ph, 10, 65, A, 10, R, 65, None) == tsqr.TSQR_ERR_UNSUPPORTED
    # every n at the largest m fits the scratch with the built-in policy ...
    for n in (1, 16, 50, 64):
        assert tsqr.tsqr_workspace_bytes(ph, 1 << 30, n, tsqr.TSQR_F64) <= tsqr.TSQR_NOALLOC_SCRATCH_BYTES, n
    # ... a tiny leaf size on a large m does not
    tsqr.tsqr_set_option(ph, tsqr.TSQR_OPT_LEAF_ROWS, 128)
    assert f(ph, 1 << 22, 50, A, 1 << 22, R, 50, None) == tsqr.TSQR_ERR_SCRATCH
    tsqr.tsqr_set_option(ph, tsqr.TSQR_OPT_LEAF_ROWS, 0)
    assert b"scratch" in L.tsqr_status_string(tsqr.TSQR_ERR_SCRATCH)


def test_rtilde_entries_argument_checks(ph):
    """tsqr_mixed_exec_rtilde (the caller's R~ is argument 3) and
    tsqr_mixed_rtilde_exec (the FP32 stage alone) on a planning handle."""
    L = tsqr.lib()
    p = tsqr.tsqr_mixed_plan_create_sampled(ph, 3, 10000, 50, 10000, 500000, 1024, 5)
    try:
        need = tsqr.tsqr_mixed_workspace_bytes(p)
        buf = ctypes.create_string_buffer(need + 512)
        ws = (ctypes.addressof(buf) + 255) // 256 * 256
        f = L.tsqr_mixed_exec_rtilde
        assert f(None, 1, 1, 1, 50, None, ws, need, None) == -1
        assert f(p, None, 1, 1, 50, None, ws, need, None) == -2
        assert f(p, 1, None, 1, 50, None, ws, need, None) == -3
        assert f(p, 1, 1, None, 50, None, ws, need, None) == -4
        assert f(p, 1, 1, 1, 49, None, ws, need, None) == -5
        assert f(p, 1, 1, 1, 50, None, None, need, None) == -7
        assert f(p, 1, 1, 1, 50, None, ws + 8, need, None) == -7
        assert f(p, 1, 1, 1, 50, None, ws, need - 1, None) == -8
        assert f(p, 1, 1, 1, 50, None, ws, need, None) == tsqr.TSQR_ERR_NO_DEVICE
        g = L.tsqr_mixed_rtilde_exec
        assert g(None, 1, ws, need, None) == -1
        assert g(p, None, ws, need, None) == -2
        assert g(p, 1, None, need, None) == -3
        assert g(p, 1, ws + 8, need, None) == -3
        assert g(p, 1, ws, need - 1, None) == -4
        assert g(p, 1, ws, need, None) == tsqr.TSQR_ERR_NO_DEVICE
    finally:
        tsqr.tsqr_mixed_plan_destroy(p)
    # an empty plan has nothing to do
    e = tsqr.tsqr_mixed_plan_create(ph, 0, 100, 8, 100, 800)
    try:
        assert L.tsqr_mixed_rtilde_exec(e, None, None, 0, None) == 0
    finally:
        tsqr.tsqr_mixed_plan_destroy(e)


def test_learned_correction_argument_checks(ph):
    """The MLP and surrogate calls: -k for the k-th argument, empty sizes are
    no-ops, a planning handle stops before any launch."""
    L = tsqr.lib()
    ND = tsqr.TSQR_ERR_NO_DEVICE
    g = L.tsqr_gemm_bf16
    assert g(None, 0, 0, 4, 4, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 4, None) == -1
    assert g(ph, 0, 0, -1, 4, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 4, None) == -4
    assert g(ph, 0, 0, 4, -1, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 4, None) == -5
    assert g(ph, 0, 0, 4, 4, -1, 1.0, 1, 4, 1, 4, 0.0, 1, 4, None) == -6
    assert g(ph, 0, 0, 4, 4, 4, 1.0, None, 4, 1, 4, 0.0, 1, 4, None) == -8
    assert g(ph, 0, 0, 5, 4, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 5, None) == -9       # lda < M
    assert g(ph, 1, 0, 4, 4, 5, 1.0, 1, 4, 1, 5, 0.0, 1, 4, None) == -9       # A stored K x M: lda < K
    assert g(ph, 0, 0, 4, 4, 4, 1.0, 1, 4, None, 4, 0.0, 1, 4, None) == -10
    assert g(ph, 0, 0, 4, 4, 5, 1.0, 1, 4, 1, 4, 0.0, 1, 4, None) == -11      # ldb < K
    assert g(ph, 0, 1, 4, 5, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 4, None) == -11      # B stored N x K: ldb < N
    assert g(ph, 0, 0, 4, 4, 4, 1.0, 1, 4, 1, 4, 0.0, None, 4, None) == -13
    assert g(ph, 0, 0, 4, 4, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 3, None) == -14
    assert g(ph, 0, 0, 0, 4, 4, 1.0, None, 1, None, 4, 0.0, None, 1, None) == 0
    assert g(ph, 0, 0, 4, 4, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 4, None) == ND
    # K = 0 writes beta C (operands unread)
    assert g(ph, 0, 0, 4, 4, 0, 1.0, None, 4, None, 1, 0.0, 1, 4, None) == ND
    b = L.tsqr_mlp_bias_act
    assert b(None, 1, 4, 4, 4, 1, 1, None) == -1
    assert b(ph, None, 4, 4, 4, 1, 1, None) == -2
    assert b(ph, 1, -1, 4, 4, 1, 1, None) == -3
    assert b(ph, 1, 4, -1, 4, 1, 1, None) == -4
    assert b(ph, 1, 4, 4, 3, 1, 1, None) == -5
    assert b(ph, 1, 4, 4, 4, None, 1, None) == -6
    assert b(ph, None, 0, 4, 1, None, 1, None) == 0
    assert b(ph, 1, 4, 4, 4, 1, 1, None) == ND
    r = L.tsqr_mlp_relu_grad
    assert r(None, 1, 1, 4, 4, 4, None) == -1
    assert r(ph, None, 1, 4, 4, 4, None) == -2
    assert r(ph, 1, None, 4, 4, 4, None) == -3
    assert r(ph, 1, 1, -1, 4, 4, None) == -4
    assert r(ph, 1, 1, 4, -1, 4, None) == -5
    assert r(ph, 1, 1, 4, 4, 3, None) == -6
    assert r(ph, 1, 1, 4, 4, 4, None) == ND
    c = L.tsqr_mlp_colsum
    assert c(None, 1, 4, 4, 4, 1, None) == -1
    assert c(ph, None, 4, 4, 4, 1, None) == -2
    assert c(ph, 1, -1, 4, 4, 1, None) == -3
    assert c(ph, 1, 4, -1, 4, 1, None) == -4
    assert c(ph, 1, 4, 4, 3, 1, None) == -5
    assert c(ph, 1, 4, 4, 4, None, None) == -6
    assert c(ph, None, 0, 4, 1, 1, None) == ND     # zero rows: s = 0 is still written
    assert c(ph, 1, 4, 4, 4, 1, None) == ND
    s = L.tsqr_mlp_mse
    assert s(None, 1, 1, 1, 4, 4, 4, 1, None) == -1
    assert s(ph, None, 1, 1, 4, 4, 4, 1, None) == -2
    assert s(ph, 1, None, 1, 4, 4, 4, 1, None) == -3
    assert s(ph, 1, 1, None, 4, 4, 4, 1, None) == -4
    assert s(ph, 1, 1, 1, 0, 4, 4, 1, None) == -5
    assert s(ph, 1, 1, 1, 4, 0, 4, 1, None) == -6
    assert s(ph, 1, 1, 1, 4, 4, 3, 1, None) == -7
    assert s(ph, 1, 1, 1, 4, 4, 4, None, None) == -8
    assert s(ph, 1, 1, 1, 4, 4, 4, 1, None) == ND
    a = L.tsqr_mlp_adam
    args = (1e-3, 0.9, 0.999, 1e-8)
    assert a(None, 1, 1, 1, 1, 4, *args, 1, None) == -1
    assert a(ph, None, 1, 1, 1, 4, *args, 1, None) == -2
    assert a(ph, 1, None, 1, 1, 4, *args, 1, None) == -3
    assert a(ph, 1, 1, None, 1, 4, *args, 1, None) == -4
    assert a(ph, 1, 1, 1, None, 4, *args, 1, None) == -5
    assert a(ph, 1, 1, 1, 1, -1, *args, 1, None) == -6
    assert a(ph, 1, 1, 1, 1, 4, *args, 0, None) == -11
    assert a(ph, None, None, None, None, 0, *args, 1, None) == 0
    assert a(ph, 1, 1, 1, 1, 4, *args, 1, None) == ND
    fe = L.tsqr_surrogate_features
    assert fe(None, 1, 4, 50, 1, None) == -1
    assert fe(ph, None, 4, 50, 1, None) == -2
    assert fe(ph, 1, -1, 50, 1, None) == -3
    assert fe(ph, 1, 4, 0, 1, None) == -4
    assert fe(ph, 1, 4, 65, 1, None) == -4
    assert fe(ph, 1, 4, 50, None, None) == -5
    assert fe(ph, None, 0, 50, None, None) == 0
    assert fe(ph, 1, 4, 50, 1, None) == ND
    t = L.tsqr_surrogate_targets
    assert t(None, 1, 50, 1, 4, 50, 1, None) == -1
    assert t(ph, None, 50, 1, 4, 50, 1, None) == -2
    assert t(ph, 1, 49, 1, 4, 50, 1, None) == -3
    assert t(ph, 1, 50, None, 4, 50, 1, None) == -4
    assert t(ph, 1, 50, 1, -1, 50, 1, None) == -5
    assert t(ph, 1, 50, 1, 4, 0, 1, None) == -6
    assert t(ph, 1, 50, 1, 4, 50, None, None) == -7
    assert t(ph, 1, 50, 1, 4, 50, 1, None) == ND
    ap = L.tsqr_surrogate_apply
    assert ap(None, 1, 1, 4, 50, 1, None) == -1
    assert ap(ph, None, 1, 4, 50, 1, None) == -2
    assert ap(ph, 1, None, 4, 50, 1, None) == -3
    assert ap(ph, 1, 1, -1, 50, 1, None) == -4
    assert ap(ph, 1, 1, 4, 0, 1, None) == -5
    assert ap(ph, 1, 1, 4, 50, None, None) == -6
    assert ap(ph, 1, 1, 4, 50, 1, None) == ND


def test_batch_exec_stamped_argument_checks(ph):
    """The stamped batch exec checks its arguments as tsqr_batch_exec does,
    then the stamps (-7); the clock query needs a device."""
    L = tsqr.lib()
    p = tsqr.tsqr_batch_plan_create(ph, 2, 50, [300, 5000], [0, 300 * 50], None, tsqr.TSQR_F64)
    try:
        need = tsqr.tsqr_batch_workspace_bytes(p)
        buf = ctypes.create_string_buffer(need + 512)
        ws = (ctypes.addressof(buf) + 255) // 256 * 256
        f = L.tsqr_batch_exec_stamped
        assert f(None, 1, 1, 50, ws, need, 1, None) == -1
        assert f(p, None, 1, 50, ws, need, 1, None) == -2
        assert f(p, 1, None, 50, ws, need, 1, None) == -3
        assert f(p, 1, 1, 49, ws, need, 1, None) == -4
        assert f(p, 1, 1, 50, None, need, 1, None) == -5
        assert f(p, 1, 1, 50, ws, need - 1, 1, None) == -6
        assert f(p, 1, 1, 50, ws, need, None, None) == -7
        assert f(p, 1, 1, 50, ws, need, 1, None) == tsqr.TSQR_ERR_NO_DEVICE
    finally:
        tsqr.tsqr_batch_plan_destroy(p)
    assert L.tsqr_device_clock_khz(None) == -1
    assert L.tsqr_device_clock_khz(ph) == -1000 - tsqr.TSQR_ERR_NO_DEVICE


def test_geqr_r_stamped_argument_checks(ph):
    """tsqr_geqr_r_f64's argument codes, then -10 for the stamps."""
    L = tsqr.lib()
    m, n = 1 << 20, 50
    need = tsqr.tsqr_workspace_bytes(ph, m, n, tsqr.TSQR_F64)
    f = L.tsqr_geqr_r_f64_stamped
    assert f(None, m, n, 1, m, 1, n, 256, need, 1, None) == -1
    assert f(ph, -1, n, 1, m, 1, n, 256, need, 1, None) == -2
    assert f(ph, m, -1, 1, m, 1, n, 256, need, 1, None) == -3
    assert f(ph, m, n, None, m, 1, n, 256, need, 1, None) == -4
    assert f(ph, m, n, 1, m - 1, 1, n, 256, need, 1, None) == -5
    assert f(ph, m, n, 1, m, None, n, 256, need, 1, None) == -6
    assert f(ph, m, n, 1, m, 1, n - 1, 256, need, 1, None) == -7
    assert f(ph, m, n, 1, m, 1, n, None, need, 1, None) == -8
    assert f(ph, m, n, 1, m, 1, n, 256, need - 1, 1, None) == -9
    assert f(ph, m, n, 1, m, 1, n, 256, need, None, None) == -10
    assert f(ph, m, n, 1, m, 1, n, 256, need, 1, None) == tsqr.TSQR_ERR_NO_DEVICE
