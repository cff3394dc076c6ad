"""Every instance of the two full-size batched workloads against the oracle.

* Ragged batch: 4096 instances, m log-uniform in [64, 65536), n = 50, one
  launch; in FP32 (the stored data) and in FP64 (the same values promoted).
* Conditioned batch: 256 instances of 65536 x 50 stored in FP32 with
  kappa_i = 10^(8 i / 255), through the mixed-precision path (FP32 TSQR
  followed by one FP64 correction).

The oracle (single-threaded C) runs over a pool of host processes
(``oracle.parallel``).  Per instance the test records kappa and the three
errors of tests/gates.py and prints a summary: the largest error of each kind,
its instance, and how many instances needed the kappa-scaled FP32 relF gate.
"""
import numpy as np
import pytest

import oracle
from gates import GRAM32, GRAM64, kappa_of, relF, row_gate64, row_scaled
from oracle import parallel
from paper_1002_4250_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1002_4250_amd import tsqr  # noqa: E402

N = 50


@pytest.fixture(scope="module")
def ragged():
    flat, sizes, offsets = inputs.batched_uniform(4096, N, 64, 65536, seed=2, dtype=np.float32)
    return flat, sizes, offsets


def summarize(label, kappas, errs):
    lines = [f"{label}: {len(kappas)} instances, kappa {np.min(kappas):.3g} .. {np.max(kappas):.3g}"]
    for name, e in errs.items():
        i = int(np.nanargmax(e))
        lines.append(f"  max {name} {e[i]:.3e} at instance {i} (kappa {kappas[i]:.3g})")
    print("\n".join(lines), flush=True)


def check_ragged(flat, sizes, offsets, dtype):
    plan = tsqr.BatchPlan(sizes, offsets, N, dtype)
    Ad = torch.from_numpy(flat).cuda()
    if dtype == torch.float64:
        Ad = Ad.double()
    Rb = plan.run(Ad).cpu().numpy()
    del Ad
    torch.cuda.empty_cache()
    Rg = [Rb[b].T for b in range(len(sizes))]
    Ro, g = parallel.check_batch(flat, [(o, m, N, m) for o, m in zip(offsets, sizes)], Rg)
    return Rg, Ro, g


def test_full_ragged_batch_fp32_every_instance(ragged):
    """FP32: backward error <= 1e-6 for every instance (kappa-free); relF <=
    1e-5 * max(1, kappa / 10) (the forward error grows with kappa; short,
    nearly square instances reach kappa in the thousands)."""
    flat, sizes, offsets = ragged
    Rg, Ro, g = check_ragged(flat, sizes, offsets, torch.float32)
    kap = np.array([kappa_of(r) for r in Ro])
    rf = np.array([relF(a.astype(np.float64), b) for a, b in zip(Rg, Ro)])
    summarize("ragged FP32", kap, {"relF": rf, "backward error": g})
    relaxed = int(np.sum(kap > 10.0))
    print(f"  instances with kappa > 10 (relF gate scaled by kappa/10): {relaxed}", flush=True)
    for b in range(len(sizes)):
        assert g[b] < GRAM32, (b, sizes[b], g[b])
        assert rf[b] < 1e-5 * max(1.0, kap[b] / 10.0), (b, sizes[b], kap[b], rf[b])
        assert np.all(np.tril(Rg[b], -1) == 0) and np.all(np.diag(Rg[b]) > 0), b


def test_full_ragged_batch_fp64_every_instance(ragged):
    """FP64 (the FP32 values promoted): relF <= 1e-10, backward error <=
    1e-14 and the row-scaled gate for every instance."""
    flat, sizes, offsets = ragged
    Rg, Ro, g = check_ragged(flat, sizes, offsets, torch.float64)
    kap = np.array([kappa_of(r) for r in Ro])
    rf = np.array([relF(a, b) for a, b in zip(Rg, Ro)])
    rs = np.array([row_scaled(a, b) for a, b in zip(Rg, Ro)])
    summarize("ragged FP64", kap, {"relF": rf, "backward error": g, "row-scaled": rs})
    for b in range(len(sizes)):
        assert rf[b] < 1e-10 and g[b] < GRAM64 and rs[b] < row_gate64(kap[b]), (b, sizes[b], rf[b], g[b], rs[b])


def test_full_conditioned_batch_mixed_every_instance():
    """256 x 65536 x 50 in FP32 storage, kappa from 1 to 1e8, mixed path:
    relF <= 1e-13 * max(1, kappa), backward error <= 1e-14 and the row-scaled
    gate for every instance; fallbacks are counted."""
    batch, m = 256, 65536
    flat, kappas = inputs.conditioned_batch(batch, m, N, log10_kappa_max=8.0, seed=3)
    plan = tsqr.MixedPlan(batch, m, N)
    R, fb = plan.run(torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    Rb = R.cpu().numpy()
    del R, plan
    torch.cuda.empty_cache()
    Rg = [Rb[b].T for b in range(batch)]
    Ro, g = parallel.check_batch(flat, [(b * m * N, m, N, m) for b in range(batch)], Rg)
    kap = np.array([kappa_of(r) for r in Ro])
    rf = np.array([relF(a, b) for a, b in zip(Rg, Ro)])
    rs = np.array([row_scaled(a, b) for a, b in zip(Rg, Ro)])
    summarize("conditioned batch, mixed", kap, {"relF": rf, "backward error": g, "row-scaled": rs})
    print(f"  fallbacks to the FP64 path: {sum(fb)}", flush=True)
    for b in range(batch):
        assert rf[b] < 1e-13 * max(1.0, kappas[b]), (b, kappas[b], rf[b])
        assert g[b] < GRAM64, (b, kappas[b], g[b])
        assert rs[b] < row_gate64(kap[b]), (b, kap[b], rs[b])
