"""Device-side (PyTorch) generators of the selector's matrix classes.

Same classes and parameter draws as ``csrgen.selector_matrix`` (class i mod 5,
rows log-uniform in ``selector_range(i)``, class parameters from numpy PCG64
with the matrix's seed); the arrays themselves are drawn on the GPU with a seeded
``torch.Generator`` so that thousands of large matrices can be produced in
seconds.  These inputs only feed the parameter selector's timings, never a
parity check.  Holds none of the SpMV arithmetic.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import SELECTOR_CLASSES, rng_for, selector_range


def _finish(lengths: torch.Tensor, cols: torch.Tensor, n: int, gen: torch.Generator, name: str):
    m = lengths.numel()
    rp = torch.zeros(m + 1, dtype=torch.int64, device=cols.device)
    rp[1:] = torch.cumsum(lengths.to(torch.int64), 0)
    nnz = int(rp[-1])
    val = torch.rand(nnz, dtype=torch.float64, device=cols.device, generator=gen) * 2 - 1
    x = torch.rand(n, dtype=torch.float64, device=cols.device, generator=gen) * 2 - 1
    return {"row_ptr": rp.to(torch.int32), "col": cols.to(torch.int32).contiguous(), "val": val, "x": x,
            "m": m, "n": n, "nnz": nnz, "name": name}


def _stencil(N: int, dims: int, gen, device):
    m = N ** dims
    idx = torch.arange(m, dtype=torch.int64, device=device)
    if dims == 2:
        i, j = idx // N, idx % N
        offs = [(-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)]  # ascending column order
        cols, ok = [], []
        for di, dj in offs:
            ni, nj = i + di, j + dj
            ok.append((ni >= 0) & (ni < N) & (nj >= 0) & (nj < N))
            cols.append(ni * N + nj)
    else:
        i, j, k = idx // (N * N), (idx // N) % N, idx % N
        cols, ok = [], []
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for dk in (-1, 0, 1):
                    ni, nj, nk = i + di, j + dj, k + dk
                    ok.append((ni >= 0) & (ni < N) & (nj >= 0) & (nj < N) & (nk >= 0) & (nk < N))
                    cols.append((ni * N + nj) * N + nk)
    C = torch.stack(cols, 1)
    V = torch.stack(ok, 1)
    return _finish(V.sum(1), C[V], m, gen, f"stencil{dims}d_{N}")


def _fem_band(m: int, gen, device, width=50, block=10):
    w = min(width, m)
    nb = (m + block - 1) // block
    jitter = torch.randint(-2 * width, 2 * width + 1, (nb,), generator=gen, device=device)
    base = torch.clamp(torch.arange(nb, device=device) * block - width // 2 + jitter, 0, max(0, m - w))
    start = torch.repeat_interleave(base, block)[:m]
    cols = (start[:, None] + torch.arange(w, device=device)[None, :]).reshape(-1)
    return _finish(torch.full((m,), w, device=device), cols, m, gen, f"fem_band_{m}")


def _random_rows(lengths: torch.Tensor, n: int, gen, device, name):
    """Uniform random columns, duplicates within a row removed, sorted."""
    m = lengths.numel()
    rows = torch.repeat_interleave(torch.arange(m, device=device), lengths)
    cols = torch.randint(0, n, (rows.numel(),), generator=gen, device=device)
    key = torch.unique(rows * n + cols)  # sorted, unique
    r = key // n
    return _finish(torch.bincount(r, minlength=m), key % n, n, gen, name)


def _weblike(m: int, gen, device, mean=3.0, sigma=1.0):
    z = torch.randn(m, generator=gen, device=device, dtype=torch.float64)
    lengths = torch.clamp(torch.round(torch.exp(math.log(mean) - sigma * sigma / 2 + sigma * z)), 0, m).to(torch.int64)
    return _random_rows(lengths, m, gen, device, f"weblike_{m}")


def _dense_rows(m: int, gen, device, k: int, dense_len: np.ndarray, base_mean=5.0):
    lengths = torch.poisson(torch.full((m,), base_mean, dtype=torch.float64, device=device), generator=gen)
    lengths = torch.clamp(lengths, 0, m).to(torch.int64)
    which = torch.randperm(m, generator=gen, device=device)[:k]
    sparse = lengths.clone()
    sparse[which] = 0
    out = _random_rows(sparse, m, gen, device, f"dense_rows_{m}")
    # splice the dense rows (unique sorted columns) into the sparse matrix
    rp = out["row_ptr"].to(torch.int64)
    L = rp[1:] - rp[:-1]
    L[which] = torch.as_tensor(dense_len, device=device, dtype=torch.int64)
    pieces, pos = [], 0
    order = torch.sort(which).values.tolist()
    dl = dict(zip(which.tolist(), dense_len.tolist()))
    for r in order:
        pieces.append(out["col"][int(rp[pos]):int(rp[r])].to(torch.int64))
        pieces.append(torch.sort(torch.randperm(m, generator=gen, device=device)[:int(dl[r])]).values)
        pos = r
    pieces.append(out["col"][int(rp[pos]):].to(torch.int64))
    return _finish(L, torch.cat(pieces), m, gen, f"dense_rows_{m}")


def selector_matrix_gpu(i: int, seed0: int = 10000, m_lo: float | None = None, m_hi: float | None = None,
                        device="cuda"):
    """The i-th selector matrix, drawn on the GPU.  Returns a dict of device
    tensors (row_ptr, col int32; val, x float64) and sizes."""
    lo, hi = selector_range(i)
    m_lo, m_hi = (lo if m_lo is None else m_lo), (hi if m_hi is None else m_hi)
    rng = rng_for(seed0 + i)
    cls = SELECTOR_CLASSES[i % len(SELECTOR_CLASSES)]
    target = math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))
    gen = torch.Generator(device=device)
    gen.manual_seed(seed0 + i + 7_000_000)
    with torch.no_grad():
        if cls == "stencil2d":
            d = _stencil(max(2, min(int(m_hi ** 0.5), int(round(math.sqrt(target))))), 2, gen, device)
        elif cls == "stencil3d":
            d = _stencil(max(2, min(int(m_hi ** (1.0 / 3.0)), int(round(target ** (1.0 / 3.0))))), 3, gen, device)
        elif cls == "fem_band":
            d = _fem_band(max(100, int(target)), gen, device)
        elif cls == "weblike":
            d = _weblike(max(100, int(target)), gen, device)
        else:
            m = max(1000, int(target) // 2)
            k = int(rng.integers(1, 17))
            dense_len = rng.integers(max(1, m // 100), m + 1, size=k)
            d = _dense_rows(m, gen, device, k, dense_len)
    d["cls"] = cls
    return d
