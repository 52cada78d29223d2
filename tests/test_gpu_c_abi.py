"""GPU: the ABI called from plain C (tests/c_abi_demo.c, no Python in the
process) gives the same steady states, bit for bit, as the Python binding on
the same seeded inputs, and those pass parity against the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2503_18356_amd import build, inputs
from paper_2503_18356_amd import racipe as rp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from tests.test_gpu_parity import Case  # noqa: E402


def test_plain_c_caller_matches_the_binding():
    seed, P, n_ic = 2001, 300, 4
    exe = build.C_DEMO if os.path.exists(build.C_DEMO) else build.build_c_demo()
    print(f"[gpu] plain C caller TSSA seed={seed} P={P} n_ic={n_ic}", flush=True)
    sys.stdout.flush()
    r = subprocess.run([exe, str(seed), str(P), str(n_ic)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rows = np.array([line.split() for line in r.stdout.strip().splitlines()], dtype=np.float64)
    assert rows.shape == (P * n_ic, 3 + 2)
    assert np.array_equal(rows[:, 0], np.arange(P * n_ic))
    # The same network and seed through the Python binding (same library).
    case = Case(inputs.toggle_switch_self_activation(), seed, P, n_ic)
    opts = rp.Opts(precision=rp.FP32)
    out = case.gpu(opts)
    assert np.array_equal(rows[:, 1], out.status.cpu().numpy())
    assert np.array_equal(rows[:, 2], out.n_acc.cpu().numpy())
    # %.9g round-trips FP32 exactly.
    assert np.array_equal(rows[:, 3:].astype(np.float32), out.x.cpu().numpy())
    case.check(opts, label="plain C inputs")
