"""The allocation-free entry point tsqr_geqr_r_f64_noalloc, through the C ABI.

It runs the same kernels and launch geometry as tsqr_geqr_r_f64 with the
workspace taken from the library's fixed per-device scratch array, so its R
must equal the workspace entry point's bit for bit.  Two calls in a row, the
second on a smaller input (fewer leaves: the scratch still holds the first
call's triangles and counters, which the call must not depend on); a size
whose workspace exceeds the scratch is refused before any launch.
"""
import numpy as np
import pytest

import oracle
from paper_1002_4250_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1002_4250_amd import tsqr  # noqa: E402


def noalloc(h, Ad):
    m, n = Ad.shape
    R = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda").t()
    st = tsqr.tsqr_geqr_r_f64_noalloc(h, m, n, Ad.data_ptr(), Ad.stride(1), R.data_ptr(), R.stride(1),
                                      tsqr._stream_ptr(torch, Ad.device))
    return st, R


def with_workspace(h, Ad):
    m, n = Ad.shape
    return tsqr.geqr_r(Ad, ws=tsqr.workspace(m, n, torch.float64, h=h), h=h)


def device(A):
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()


def test_noalloc_equals_workspace_entry_point_twice_shrinking():
    h = tsqr.handle(0)
    for m, n, seed in [(1 << 20, 50, 41), (5000, 50, 42), (300, 17, 43)]:
        A = inputs.uniform(m, n, seed)
        Ad = device(A)
        st, R = noalloc(h, Ad)
        assert st == 0, tsqr.lib().tsqr_status_string(st)
        Rw = with_workspace(h, Ad)
        torch.cuda.synchronize()
        Rn = R.cpu().numpy()
        assert np.array_equal(Rn, Rw.cpu().numpy()), (m, n)
        if m <= 5000:
            Ro = oracle.r_factor(A)
            assert np.linalg.norm(Rn - Ro) / np.linalg.norm(Ro) < 1e-10


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    h = tsqr.tsqr_create(0)
    try:
        m, n = 1 << 22, 50
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 128)      # 32768 leaves: 334 MB of triangles
        assert tsqr.tsqr_workspace_bytes(h, m, n, tsqr.TSQR_F64) > tsqr.TSQR_NOALLOC_SCRATCH_BYTES
        A = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
        R = torch.full((n, n), 7.0, dtype=torch.float64, device="cuda").t()
        st = tsqr.tsqr_geqr_r_f64_noalloc(h, m, n, A.data_ptr(), m, R.data_ptr(), n, 0)
        assert st == tsqr.TSQR_ERR_SCRATCH
        torch.cuda.synchronize()
        assert torch.all(R == 7.0)                                    # nothing was launched
        # argument checks come first
        assert tsqr.tsqr_geqr_r_f64_noalloc(h, -1, n, A.data_ptr(), m, R.data_ptr(), n, 0) == -2
        assert tsqr.tsqr_geqr_r_f64_noalloc(h, m, n, A.data_ptr(), m - 1, R.data_ptr(), n, 0) == -5
        assert tsqr.tsqr_geqr_r_f64_noalloc(h, m, n, A.data_ptr(), m, R.data_ptr(), n - 1, 0) == -7
        assert tsqr.tsqr_geqr_r_f64_noalloc(h, m, 0, A.data_ptr(), m, R.data_ptr(), 1, 0) == 0
    finally:
        tsqr.tsqr_destroy(h)
