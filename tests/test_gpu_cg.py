"""CG with one bound plan reused for every product: the solution of a small
2D Laplacian system against a dense direct solve."""
import numpy as np
import pytest

import csrgen
from helpers import note

pytestmark = pytest.mark.gpu


def test_cg_laplacian_matches_direct_solve():
    import torch
    from paper_1504_06474_amd import sss
    from paper_1504_06474_amd.cg import cg
    A = csrgen.laplacian2d_csr(30)
    rng = np.random.default_rng(7)
    x_true = rng.uniform(-1, 1, A.n)
    dense = np.zeros((A.m, A.n))
    for i in range(A.m):
        dense[i, A.col[A.row_ptr[i]:A.row_ptr[i + 1]]] = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
    b = dense @ x_true
    x_ref = np.linalg.solve(dense, b)
    rp, col, v = (torch.from_numpy(a).cuda() for a in (A.row_ptr, A.col, A.val))
    plan = sss.Plan(A.m, A.n, A.nnz, W=4, S=1, bind_rows=True, row_ptr=rp)
    x, it, hist = cg(plan, rp, col, v, torch.from_numpy(b).cuda(), rtol=1e-11, max_iter=2000)
    note(f"  CG: {it} iterations, final relative residual {hist[-1][1]:.2e}")
    assert hist[-1][1] <= 1e-11
    err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    assert err < 1e-8, err
