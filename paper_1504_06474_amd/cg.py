"""Conjugate gradients on the GPU with one plan reused for every product.

The paper's motivation for staying with CSR (Section 1) is the iterative
solver: the matrix arrives in CSR, is multiplied a few hundred times, and a
format conversion would cost about as much as the solve.  Here the plan's
analysis (sizes, parameters, the bound first row of every thread-bunch) is
done once, and each iteration is one speculative-segmented-sum product plus
the library's own vector and dot-product kernels (sss_cg_start,
sss_cg_iterate).  The step scalars stay on the device, so an iteration does
not wait for the host; the residual is read every `check_every` iterations.
"""
from __future__ import annotations

import math

import torch

from . import sss


def cg(plan: "sss.Plan", row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, b: torch.Tensor,
       x0: torch.Tensor | None = None, rtol: float = 1e-8, max_iter: int = 1000, check_every: int = 10):
    """Solve A x = b for symmetric positive definite A (CSR, FP64 plan).
    Returns (x, iterations, [(iteration, ||r|| / ||b||), ...]); for b = 0 the
    history holds ||r|| itself."""
    if check_every < 1:
        raise ValueError("check_every must be at least 1")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    r, p, q = torch.empty_like(b), torch.empty_like(b), torch.empty_like(b)
    work = torch.empty(sss.cg_workspace_size() // 8, dtype=torch.float64, device=b.device)
    sss.cg_start(plan, row_ptr, col, val, b, x, r, p, q, work)
    rr, bb = work[:3].tolist()[0::2]
    b_norm = math.sqrt(bb) if bb > 0 else 1.0
    hist = [(0, math.sqrt(rr) / b_norm)]
    it = 0
    while it < max_iter and hist[-1][1] > rtol:
        k = min(check_every, max_iter - it)
        sss.cg_iterate(plan, row_ptr, col, val, x, r, p, q, work, k)
        it += k
        hist.append((it, math.sqrt(float(work[0])) / b_norm))
    return x, it, hist
