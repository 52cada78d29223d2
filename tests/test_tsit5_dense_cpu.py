"""CPU checks of the Tsit5 constants compiled into the kernels.

The kernel keeps its own copy of the Tsitouras tableau and the quartic
continuous-extension weights.  Read from the kernel source, the tableau must
equal the oracle's (which its own order-condition pins fix), and the
continuous extension must satisfy the order conditions of orders 1..4 as
polynomial identities in th, continuity with the step (b(1) = b) and
matching derivatives at both ends.  The generator beside the kernel must
reproduce the table.
"""
import importlib.util
import os
import re

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_18356_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("tsit5_dense", os.path.join(CSRC, "tsit5_dense.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _kernel_dense():
    src = open(os.path.join(CSRC, "dp5_kernel.h")).read()
    body = re.search(r"kTsDense\[7\]\[4\] = \{(.*?)\};", src, re.S).group(1)
    return np.array([float(v) for v in re.findall(r"-?\d+\.?\d*(?:e-?\d+)?", body)]).reshape(7, 4)


def test_kernel_tableau_equals_oracle():
    A = _gen().kernel_tableau()
    Ao, bo, _, _ = oracle.tableau(oracle.TSIT5)
    assert np.array_equal(A[:, :6], Ao[:, :6])


def test_continuous_extension_conditions():
    g = _gen()
    A = g.kernel_tableau()
    beta = _kernel_dense()
    M, y = g.conditions(A, A[6])
    assert np.abs(M @ beta.ravel() - y).max() < 1e-13
    # Spot-check the identities at a few th directly.
    c = A.sum(axis=1)
    for th in (0.0, 0.25, 0.5, 0.9, 1.0):
        bt = beta @ np.array([th, th**2, th**3, th**4])
        assert abs(bt.sum() - th) < 1e-14
        assert abs(bt @ c - th**2 / 2) < 1e-14
        assert abs(bt @ (A @ (A @ c)) - th**4 / 24) < 1e-14
    assert np.allclose(beta.sum(axis=1), A[6], atol=1e-14)


def test_generator_reproduces_the_table():
    g = _gen()
    beta, res = g.derive(g.kernel_tableau())
    assert res < 1e-13
    assert np.allclose(beta, _kernel_dense(), rtol=0, atol=1e-15)
