"""The C ABI from a plain C program (tests/abi_client.c, built by
__graft_entry__.build(): include/gmrf.h, libgmrf.so and hipMalloc for the
workspace; no Python or torch in that process): after 200 FP64 sweeps with
hyperparameter draws, its posterior mean, tau and lam match the oracle
within 1e-12 relative."""
import os
import subprocess

import numpy as np
import pytest

from paper_1702_05518_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "abi_client")
RTOL64 = 1e-12


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("rows,cols,st", [(64, 64, 4), (45, 70, 8)])
def test_c_client_matches_oracle(orc, tmp_path, rows, cols, st):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(CLIENT), "tests/abi_client is not built (__graft_entry__.build())"
    wl = inputs.lattice_workload(rows, cols, st, data_seed=3)
    yf, mf = tmp_path / "y.bin", tmp_path / "mean.bin"
    np.ascontiguousarray(wl["y"], dtype=np.float64).tofile(yf)
    r = subprocess.run([CLIENT, str(rows), str(cols), str(st), "200", "17", str(yf), str(mf)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    tau, lam, sweeps, nacc = r.stdout.split()
    mean = np.fromfile(mf, dtype=np.float64)
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=17)
    oc.sweeps(200)
    om, _ = oc.stats()
    assert int(sweeps) == 200 and int(nacc) == 200 and mean.size == rows * cols
    assert rel(mean, om) <= RTOL64
    assert rel(float(tau), oc.tau) <= RTOL64 and rel(float(lam), oc.lam) <= RTOL64
