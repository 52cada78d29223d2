"""Derive the continuous extension used for Tsitouras 5(4) time series.

The interpolant is x(t + th*h) = x + h * sum_i b_i(th) k_i over the seven
stages of the step (k_7 = f at the step's end), with b_i(th) quartic in th.
Its coefficients solve, as polynomial identities in th, the Runge-Kutta order
conditions of orders 1..4 (sum_i b_i(th) Phi_i(tree) = th^r / gamma(tree)),
continuity with the step's fifth-order solution (b_i(1) = b_i) and matching
derivatives at both ends (b_i'(0) = [i == 1], b_i'(1) = [i == 7]).  That
leaves one free parameter, fixed by the minimum-norm solution.  The local
interpolation error is O(h^5).

Reads the kernel's own tableau from dp5_kernel.h and prints the C table.
"""
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEG = 4


def kernel_tableau(path=os.path.join(HERE, "dp5_kernel.h")):
    src = open(path).read()
    body = re.search(r"kTsA\[7\]\[6\] = \{(.*?)\};", src, re.S).group(1)
    nums = [float(v) for v in re.findall(r"-?\d+\.?\d*(?:e-?\d+)?", body)]
    A = np.zeros((7, 7))
    A[:, :6] = np.array(nums).reshape(7, 6)
    return A


def conditions(A, b, D=DEG):
    """Rows (over beta[7][D], row-major) and right-hand sides of the system."""
    c = A.sum(axis=1)
    one = np.ones(7)
    Ac = A @ c
    trees = [(one, 1, 1), (c, 2, 2), (c**2, 3, 3), (Ac, 3, 6), (c**3, 4, 4), (c * Ac, 4, 8),
             (A @ c**2, 4, 12), (A @ Ac, 4, 24)]
    rows, rhs = [], []
    for v, r, g in trees:
        for k in range(1, D + 1):
            m = np.zeros((7, D)); m[:, k - 1] = v
            rows.append(m.ravel()); rhs.append(1.0 / g if k == r else 0.0)
    for i in range(7):
        m = np.zeros((7, D)); m[i, :] = 1
        rows.append(m.ravel()); rhs.append(b[i])
        m = np.zeros((7, D)); m[i, 0] = 1
        rows.append(m.ravel()); rhs.append(1.0 if i == 0 else 0.0)
        m = np.zeros((7, D)); m[i, :] = np.arange(1, D + 1)
        rows.append(m.ravel()); rhs.append(1.0 if i == 6 else 0.0)
    return np.array(rows), np.array(rhs)


def derive(A):
    b = A[6].copy()
    M, y = conditions(A, b)
    # b_i'(0) is fixed exactly (the th^1 coefficients); solve for the rest.
    fixed = np.zeros((7, DEG)); fixed[0, 0] = 1.0
    free = np.ones((7, DEG), bool); free[:, 0] = False
    y2 = y - M @ fixed.ravel()
    sol = np.linalg.lstsq(M[:, free.ravel()], y2, rcond=None)[0]
    beta = fixed.copy()
    beta[free] = sol
    return beta, np.abs(M @ beta.ravel() - y).max()


if __name__ == "__main__":
    beta, res = derive(kernel_tableau())
    print(f"// residual {res:.1e}")
    print("__device__ constexpr double kTsDense[7][4] = {")
    for row in beta:
        print("    {" + ", ".join(repr(float(v)) for v in row) + "},")
    print("};")
