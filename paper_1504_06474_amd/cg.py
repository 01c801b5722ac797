"""Conjugate gradients on the GPU with one plan reused for every product.

The paper's motivation for staying with CSR (Section 1) is the iterative
solver: the matrix arrives in CSR, is multiplied a few hundred times, and a
format conversion would cost about as much as the solve.  Here the plan's
analysis (sizes, parameters, the bound first row of every thread-bunch) is
done once, and each iteration is one speculative-segmented-sum product plus
vector updates on the device (PyTorch elementwise and dot kernels).  The step
scalars stay on the device, so an iteration does not wait for the host;
convergence is read every `check_every` iterations.
"""
from __future__ import annotations

import torch

from . import sss


def cg(plan: "sss.Plan", row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, b: torch.Tensor,
       x0: torch.Tensor | None = None, rtol: float = 1e-8, max_iter: int = 1000, check_every: int = 10):
    """Solve A x = b for symmetric positive definite A (CSR, FP64 plan).
    Returns (x, iterations, [(iteration, ||r|| / ||b||), ...])."""
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    Ap = torch.empty_like(b)
    plan.execute(row_ptr, col, val, x, Ap)
    r = b - Ap
    p = r.clone()
    rr = torch.dot(r, r)
    b_norm = float(torch.linalg.vector_norm(b))
    hist = [(0, float(torch.sqrt(rr)) / b_norm)]
    it = 0
    while it < max_iter and hist[-1][1] > rtol:
        plan.execute(row_ptr, col, val, p, Ap)
        alpha = rr / torch.dot(p, Ap)
        x.add_(p * alpha)
        r.sub_(Ap * alpha)
        rr_new = torch.dot(r, r)
        p.mul_(rr_new / rr).add_(r)
        rr = rr_new
        it += 1
        if it % check_every == 0 or it == max_iter:
            hist.append((it, float(torch.sqrt(rr)) / b_norm))
    return x, it, hist
