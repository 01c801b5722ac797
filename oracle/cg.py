"""Conjugate gradients (Hestenes and Stiefel, 1952), written from the
iteration's definition, as the checker of the library's CG calls.

TEST INFRASTRUCTURE, like the rest of this package: only the tests import it.

For symmetric positive definite A and a start x_0: r_0 = b - A x_0,
p_0 = r_0; then for k = 0, 1, ...
    alpha_k = (r_k . r_k) / (p_k . A p_k)
    x_{k+1} = x_k + alpha_k p_k
    r_{k+1} = r_k - alpha_k A p_k
    beta_k  = (r_{k+1} . r_{k+1}) / (r_k . r_k)
    p_{k+1} = r_{k+1} + beta_k p_k
A zero denominator gives a zero step (alpha or beta = 0), which happens only
once the residual is exactly zero.  The product is the oracle's row-loop
SpMV; dot products are numpy's, in double.  This is the iteration the paper's
Section 1 has in mind when it names iterative solvers as the place where CSR
is multiplied many times without a format conversion.
"""
from __future__ import annotations

import numpy as np

from . import spmv


def cg_steps(row_ptr, col, val, b, x0, iterations: int):
    """Run `iterations` steps from x0.  Returns dict(x, r, p, rr, rr_prev, bb):
    the state after the last step, rr = r.r of the last residual and rr_prev
    the one before the last step (rr_prev = rr when iterations = 0)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    r = b - spmv(row_ptr, col, val, x)
    p = r.copy()
    rr = float(r @ r)
    rr_prev = rr
    for _ in range(iterations):
        q = spmv(row_ptr, col, val, p)
        pq = float(p @ q)
        alpha = rr / pq if pq != 0.0 else 0.0
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        beta = rr_new / rr if rr != 0.0 else 0.0
        p = r + beta * p
        rr_prev, rr = rr, rr_new
    return {"x": x, "r": r, "p": p, "rr": rr, "rr_prev": rr_prev, "bb": float(b @ b)}
