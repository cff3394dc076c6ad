"""The C ABI from a plain C program (tests/c_client.c, no Python in the
computation): it allocates device memory with the HIP runtime, calls
tsqr_geqr_r_f64 on a stream of its own, and its R is compared with the
oracle's (FP64 gate 1e-10)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1002_4250_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client")


@pytest.mark.parametrize("m,n", [(3000, 50), (70001, 17), (1, 1)])
def test_c_client_matches_oracle(tmp_path, m, n):
    assert os.path.exists(CLIENT), "tests/c_client is missing: run __graft_entry__.build()"
    A = inputs.uniform(m, n, 12)
    a_path, r_path = tmp_path / "A.bin", tmp_path / "R.bin"
    np.asfortranarray(A).T.tofile(a_path)            # column-major bytes
    r = subprocess.run([CLIENT, str(a_path), str(m), str(n), str(r_path)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "c_client ok" in r.stdout
    R = np.fromfile(r_path, dtype=np.float64).reshape(n, n).T
    Ro = oracle.r_factor(A)
    assert np.linalg.norm(R - Ro) / np.linalg.norm(Ro) < 1e-10
    assert np.all(np.tril(R, -1) == 0) and not np.any(np.signbit(np.diag(R)))
