"""Seeded synthetic CSR workloads shaped like the paper's benchmark families.

This module only draws inputs: it holds none of the SpMV arithmetic, and both
the CPU oracle and the GPU path take their inputs from it.  Every generator is
deterministic in its seed (numpy PCG64).

Families (the paper's suite, Section 4.2 and Table 2, mixes regular FEM-like
matrices with irregular power-law ones whose longest rows hold O(n) entries):

* ``poisson_csr``      -- short regular rows, Poisson lengths, a share of rows
                          forced empty (the empty-row case of Section 3.2).
* ``powerlaw_csr``     -- Zipf / Zipf-Mandelbrot row lengths (irregular family).
* ``stencil2d_csr`` / ``stencil3d_csr`` / ``fem_band_csr`` / ``weblike_csr`` /
  ``dense_rows_csr``  -- the classes used to train and evaluate the tile selector.
* ``batched_set``      -- many uneven power-law matrices for the batched path.

Column indices are unique and sorted within each row; values and ``x`` are
uniform on [-1, 1] unless an integer-valued copy is asked for.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSR",
    "rng_for",
    "lengths_to_csr",
    "poisson_csr",
    "zipf_mandelbrot_q",
    "zipf_lengths",
    "powerlaw_csr",
    "config1",
    "config2",
    "config5",
    "batched_set",
    "stencil2d_csr",
    "stencil3d_csr",
    "fem_band_csr",
    "weblike_csr",
    "dense_rows_csr",
    "selector_matrix",
    "SELECTOR_CLASSES",
    "SELECTOR_LARGE_BASE",
    "selector_range",
    "uniform_values",
    "integer_values",
    "lognormal_values",
    "round_to_f32",
    "round_to_bf16",
    "bf16_bits",
    "with_values",
    "quantize",
]


@dataclasses.dataclass
class CSR:
    """A CSR matrix with int32 ``row_ptr``/``col`` and float64 ``val``."""

    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.m >= 0 and len(self.row_ptr) else 0

    def stats(self) -> dict:
        lens = np.diff(self.row_ptr.astype(np.int64))
        return {
            "m": self.m,
            "n": self.n,
            "nnz": self.nnz,
            "mean": float(lens.mean()) if self.m else 0.0,
            "max": int(lens.max()) if self.m else 0,
            "empty_frac": float((lens == 0).mean()) if self.m else 0.0,
        }


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# values
# ----------------------------------------------------------------------------

def uniform_values(rng: np.random.Generator, k: int) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=k)


def integer_values(rng: np.random.Generator, k: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=k).astype(np.float64)


def lognormal_values(rng: np.random.Generator, k: int, sigma: float = 3.0) -> np.ndarray:
    mag = np.exp(rng.normal(0.0, sigma, size=k))
    sign = np.where(rng.integers(0, 2, size=k) == 0, -1.0, 1.0)
    return mag * sign


def round_to_f32(a: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even to binary32 (numpy's cast is RNE)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def bf16_bits(a32: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns of binary32 values, rounded to nearest even.

    NaN inputs are not produced by the generators and are not handled.
    """
    u = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def round_to_bf16(a: np.ndarray) -> np.ndarray:
    """Values rounded to bfloat16 (via binary32, RNE at each step), as float32."""
    b = bf16_bits(round_to_f32(a)).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32)


# ----------------------------------------------------------------------------
# structure
# ----------------------------------------------------------------------------

def _dedup_columns(rng: np.random.Generator, rows: np.ndarray, cols: np.ndarray, n: int) -> np.ndarray:
    """Redraw duplicate (row, col) pairs until every row's columns are unique.

    Returns the column array sorted within each row (rows are already in
    ascending order in ``rows``).
    """
    n64 = np.int64(n)
    key = rows.astype(np.int64) * n64 + cols.astype(np.int64)
    key.sort()
    dup = np.zeros(key.shape[0], dtype=bool)
    if key.shape[0] > 1:
        dup[1:] = key[1:] == key[:-1]
    while dup.any():
        # only the rows that hold a duplicate are redrawn and re-sorted
        bad_rows = np.unique(key[dup] // n64)
        sel = np.isin(key // n64, bad_rows)
        sub = key[sel]
        sub_dup = dup[sel]
        sub_rows = sub // n64
        redraw = rng.integers(0, n, size=int(sub_dup.sum()), dtype=np.int64)
        sub = sub.copy()
        sub[sub_dup] = sub_rows[sub_dup] * n64 + redraw
        sub.sort()
        key[sel] = sub  # rows occupy the same contiguous slots, sorted by row
        dup = np.zeros(key.shape[0], dtype=bool)
        if key.shape[0] > 1:
            dup[1:] = key[1:] == key[:-1]
    return (key % n64).astype(np.int32)


def lengths_to_csr(rng: np.random.Generator, lengths: np.ndarray, n: int,
                   values: str = "uniform", name: str = "") -> CSR:
    """Uniform unique sorted columns for the given row lengths, then values."""
    lengths = np.asarray(lengths, dtype=np.int64)
    m = lengths.shape[0]
    if (lengths > n).any():
        raise ValueError("row longer than n")
    row_ptr64 = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr64[1:])
    nnz = int(row_ptr64[-1])
    if nnz >= 2**31:
        raise ValueError("nnz must fit int32")
    dense = lengths * 4 > n
    col = np.empty(nnz, dtype=np.int32)
    sparse_rows = np.nonzero(~dense)[0]
    if sparse_rows.size:
        sl = lengths[sparse_rows]
        rows = np.repeat(sparse_rows.astype(np.int64), sl)
        draws = rng.integers(0, n, size=rows.shape[0], dtype=np.int64)
        c = _dedup_columns(rng, rows, draws, n)
        # scatter the sparse rows' columns into place
        starts = row_ptr64[sparse_rows]
        offs = np.repeat(starts - np.concatenate(([0], np.cumsum(sl)[:-1])), sl)
        col[np.arange(rows.shape[0], dtype=np.int64) + offs] = c
    for r in np.nonzero(dense)[0]:
        L = int(lengths[r])
        col[row_ptr64[r]:row_ptr64[r] + L] = np.sort(rng.choice(n, size=L, replace=False)).astype(np.int32)
    if values == "uniform":
        val = uniform_values(rng, nnz)
    elif values == "int":
        val = integer_values(rng, nnz)
    elif values == "lognormal":
        val = lognormal_values(rng, nnz)
    else:
        raise ValueError(values)
    return CSR(m, n, row_ptr64.astype(np.int32), col, val, name)


def poisson_csr(m: int, n: int, mean: float, empty_frac: float, seed: int,
                values: str = "uniform", name: str = "poisson") -> CSR:
    rng = rng_for(seed)
    lengths = np.minimum(rng.poisson(mean, size=m), n).astype(np.int64)
    n_empty = int(round(empty_frac * m))
    if n_empty:
        lengths[rng.choice(m, size=n_empty, replace=False)] = 0
    return lengths_to_csr(rng, lengths, n, values, name)


def _zm_pmf(kmax: int, a: float, q: float) -> np.ndarray:
    k = np.arange(1, kmax + 1, dtype=np.float64)
    w = (k + q) ** (-a)
    return w / w.sum()


def zipf_mandelbrot_q(kmax: int, a: float, target_mean: float) -> float:
    """Offset q so that p(k) ~ (k+q)^-a on [1, kmax] has the given mean."""
    k = np.arange(1, kmax + 1, dtype=np.float64)

    def mean(q):
        p = _zm_pmf(kmax, a, q)
        return float((k * p).sum())

    lo, hi = 0.0, 1.0
    while mean(hi) < target_mean:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if mean(mid) < target_mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def zipf_lengths(rng: np.random.Generator, m: int, kmax: int, a: float, q: float) -> np.ndarray:
    """Inverse-CDF draws from p(k) ~ (k+q)^-a on k in [1, kmax]."""
    cdf = np.cumsum(_zm_pmf(kmax, a, q))
    cdf[-1] = 1.0
    u = rng.random(m)
    return (np.searchsorted(cdf, u, side="right") + 1).astype(np.int64)


def powerlaw_csr(m: int, n: int, a: float, kmax: int, mean: float, empty_frac: float,
                 seed: int, values: str = "uniform", pure_zipf: bool = False,
                 name: str = "powerlaw") -> CSR:
    """Power-law row lengths.

    ``pure_zipf``: p(k) ~ k^-a on [1, kmax] (kmax chosen by the caller for the
    mean).  Otherwise Zipf-Mandelbrot with offset q solved so that the mean over
    non-empty rows is ``mean / (1 - empty_frac)``; then ``empty_frac`` of the
    rows are forced empty.
    """
    rng = rng_for(seed)
    kmax = min(kmax, n)
    if pure_zipf:
        q = 0.0
    else:
        q = zipf_mandelbrot_q(kmax, a, mean / (1.0 - empty_frac))
    lengths = zipf_lengths(rng, m, kmax, a, q)
    n_empty = int(round(empty_frac * m))
    if n_empty:
        lengths[rng.choice(m, size=n_empty, replace=False)] = 0
    return lengths_to_csr(rng, lengths, n, values, name)


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

def config1(int_valued: bool = False, m: int = 4096) -> tuple[CSR, np.ndarray]:
    """m=n=4096, Poisson(10) lengths, 5% forced-empty rows.  Seeds 1 / 2."""
    seed = 2 if int_valued else 1
    A = poisson_csr(m, m, 10.0, 0.05, seed, "int" if int_valued else "uniform",
                    name="poisson4096" + ("_int" if int_valued else ""))
    rng = rng_for(seed + 1000)
    x = integer_values(rng, m) if int_valued else uniform_values(rng, m)
    return A, x


# Zipf exponent 1.8 on [1, K]: K solved for mean 20 (so about 80M nnz at 4M rows)
CONFIG5_KMAX = 42207


def config2(seed: int = 1, m: int = 1_000_000, values: str = "uniform") -> tuple[CSR, np.ndarray]:
    """m=n=1e6 power law: Zipf-Mandelbrot exponent 2 on [1, 2e5], mean ~20,
    3% of rows forced empty."""
    A = powerlaw_csr(m, m, 2.0, 200_000, 20.0, 0.03, seed, values, name=f"powerlaw{m}")
    rng = rng_for(seed + 1000)
    x = integer_values(rng, m) if values == "int" else uniform_values(rng, m)
    return A, x


def config5(seed: int = 5, m: int = 4_000_000, values: str = "uniform") -> tuple[CSR, np.ndarray]:
    """m=n=4e6, pure Zipf exponent 1.8 on [1, 42207] (mean ~20, ~80M nnz)."""
    kmax = CONFIG5_KMAX if m == 4_000_000 else max(2, min(m, CONFIG5_KMAX))
    A = powerlaw_csr(m, m, 1.8, kmax, 20.0, 0.0, seed, values, pure_zipf=True,
                     name=f"zipf18_{m}_{values}")
    rng = rng_for(seed + 1000)
    x = integer_values(rng, m) if values == "int" else uniform_values(rng, m)
    return A, x


def batched_set(count: int = 512, seed0: int = 20000, m_lo: int = 1000, m_hi: int = 200_000,
                values: str = "uniform") -> list[tuple[CSR, np.ndarray]]:
    """Uneven power-law matrices: m log-uniform in [m_lo, m_hi], n = m,
    Zipf-Mandelbrot exponent 2 on [1, min(m, 2e5)] with mean 15."""
    out = []
    for i in range(count):
        rng = rng_for(seed0 + i)
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        kmax = min(m, 200_000)
        q = zipf_mandelbrot_q(kmax, 2.0, 15.0)
        lengths = zipf_lengths(rng, m, kmax, 2.0, q)
        A = lengths_to_csr(rng, lengths, m, values, name=f"batch{i}")
        x = integer_values(rng, m) if values == "int" else uniform_values(rng, m)
        out.append((A, x))
    return out


# ----------------------------------------------------------------------------
# selector classes
# ----------------------------------------------------------------------------

def _from_coo(m: int, n: int, rows: np.ndarray, cols: np.ndarray, rng, values, name) -> CSR:
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if values == "int":
        val = integer_values(rng, nnz)
    else:
        val = uniform_values(rng, nnz)
    return CSR(m, n, row_ptr.astype(np.int32), cols.astype(np.int32), val, name)


def stencil2d_csr(N: int, seed: int, values: str = "uniform") -> CSR:
    """5-point stencil on an N x N grid."""
    rng = rng_for(seed)
    idx = np.arange(N * N, dtype=np.int64)
    i, j = idx // N, idx % N
    rows, cols = [idx], [idx]
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ok = (i + di >= 0) & (i + di < N) & (j + dj >= 0) & (j + dj < N)
        rows.append(idx[ok])
        cols.append((i[ok] + di) * N + (j[ok] + dj))
    return _from_coo(N * N, N * N, np.concatenate(rows), np.concatenate(cols), rng, values, f"stencil2d_{N}")


def laplacian2d_csr(N: int) -> CSR:
    """The 5-point Laplacian on an N x N grid with Dirichlet boundaries: 4 on
    the diagonal, -1 for each grid neighbour (symmetric positive definite)."""
    idx = np.arange(N * N, dtype=np.int64)
    i, j = idx // N, idx % N
    rows, cols, vals = [idx], [idx], [np.full(N * N, 4.0)]
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ok = (i + di >= 0) & (i + di < N) & (j + dj >= 0) & (j + dj < N)
        rows.append(idx[ok])
        cols.append((i[ok] + di) * N + (j[ok] + dj))
        vals.append(np.full(int(ok.sum()), -1.0))
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    order = np.lexsort((cols, rows))
    row_ptr = np.zeros(N * N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N * N), out=row_ptr[1:])
    return CSR(N * N, N * N, row_ptr.astype(np.int32), cols[order].astype(np.int32), vals[order],
               f"laplacian2d_{N}")


def stencil3d_csr(N: int, seed: int, values: str = "uniform") -> CSR:
    """27-point stencil on an N^3 grid."""
    rng = rng_for(seed)
    idx = np.arange(N ** 3, dtype=np.int64)
    i, j, k = idx // (N * N), (idx // N) % N, idx % N
    rows, cols = [], []
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                ok = ((i + di >= 0) & (i + di < N) & (j + dj >= 0) & (j + dj < N)
                      & (k + dk >= 0) & (k + dk < N))
                rows.append(idx[ok])
                cols.append(((i[ok] + di) * N + (j[ok] + dj)) * N + (k[ok] + dk))
    return _from_coo(N ** 3, N ** 3, np.concatenate(rows), np.concatenate(cols), rng, values, f"stencil3d_{N}")


def fem_band_csr(m: int, seed: int, width: int = 50, block: int = 10, values: str = "uniform") -> CSR:
    """FEM-like: rows in blocks of ``block`` share a contiguous ``width``-wide
    column band placed near the diagonal with a random jitter."""
    rng = rng_for(seed)
    nb = (m + block - 1) // block
    jitter = rng.integers(-2 * width, 2 * width + 1, size=nb)
    base = np.clip(np.arange(nb, dtype=np.int64) * block - width // 2 + jitter, 0, max(0, m - width))
    start = np.repeat(base, block)[:m]
    lengths = np.full(m, min(width, m), dtype=np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), lengths)
    offs = np.arange(rows.shape[0], dtype=np.int64) - np.repeat(np.arange(m, dtype=np.int64) * lengths[0], lengths)
    cols = start[rows] + offs
    return _from_coo(m, m, rows, cols, rng, values, f"fem_band_{m}")


def weblike_csr(m: int, seed: int, mean: float = 3.0, sigma: float = 1.0, values: str = "uniform") -> CSR:
    """Web-graph-like: lengths round(LogNormal(ln(mean) - sigma^2/2, sigma))."""
    rng = rng_for(seed)
    lengths = np.rint(rng.lognormal(math.log(mean) - sigma * sigma / 2.0, sigma, size=m)).astype(np.int64)
    lengths = np.minimum(lengths, m)
    return lengths_to_csr(rng, lengths, m, values, f"weblike_{m}")


def dense_rows_csr(m: int, seed: int, base_mean: float = 5.0, values: str = "uniform") -> CSR:
    """Sparse rows (Poisson(base_mean)) plus 1-16 dense rows of n/100..n entries."""
    rng = rng_for(seed)
    lengths = np.minimum(rng.poisson(base_mean, size=m), m).astype(np.int64)
    k = int(rng.integers(1, 17))
    which = rng.choice(m, size=k, replace=False)
    lengths[which] = rng.integers(max(1, m // 100), m + 1, size=k)
    return lengths_to_csr(rng, lengths, m, values, f"dense_rows_{m}")


SELECTOR_CLASSES = ("stencil2d", "stencil3d", "fem_band", "weblike", "dense_rows")
# matrices 0..SELECTOR_LARGE_BASE-1 of the selector set have 1e4..2e6 rows,
# the ones from SELECTOR_LARGE_BASE on 2e6..1.6e7 (sizes past one XCD's L2 and
# past the Infinity Cache, where the best tile schedule changes again)
SELECTOR_LARGE_BASE = 2200
SELECTOR_RANGES = ((1e4, 2e6), (2e6, 1.6e7))


def selector_range(i: int):
    """Row range (m_lo, m_hi) of the i-th selector matrix."""
    return SELECTOR_RANGES[0] if i < SELECTOR_LARGE_BASE else SELECTOR_RANGES[1]


def selector_matrix(i: int, seed0: int = 10000, m_lo: float | None = None, m_hi: float | None = None,
                    values: str = "uniform") -> CSR:
    """The i-th matrix of the selector set: class i mod 5, rows log-uniform in
    selector_range(i) unless m_lo / m_hi are given; stencil sides capped at
    m_hi's square or cube root."""
    lo, hi = selector_range(i)
    m_lo, m_hi = (lo if m_lo is None else m_lo), (hi if m_hi is None else m_hi)
    rng = rng_for(seed0 + i)
    cls = SELECTOR_CLASSES[i % len(SELECTOR_CLASSES)]
    target = math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))
    seed = seed0 + i + 7_000_000
    if cls == "stencil2d":
        return stencil2d_csr(max(2, min(int(m_hi ** 0.5), int(round(math.sqrt(target))))), seed, values)
    if cls == "stencil3d":
        return stencil3d_csr(max(2, min(int(m_hi ** (1.0 / 3.0)), int(round(target ** (1.0 / 3.0))))), seed, values)
    if cls == "fem_band":
        return fem_band_csr(max(100, int(target)), seed, values=values)
    if cls == "weblike":
        return weblike_csr(max(100, int(target)), seed, values=values)
    return dense_rows_csr(max(1000, int(target) // 2), seed, values=values)


def with_values(A: CSR, kind: str, seed: int) -> CSR:
    """Same structure, new seeded values ("uniform", "int" or "lognormal")."""
    rng = rng_for(seed)
    if kind == "uniform":
        val = uniform_values(rng, A.nnz)
    elif kind == "int":
        val = integer_values(rng, A.nnz)
    elif kind == "lognormal":
        val = lognormal_values(rng, A.nnz)
    else:
        raise ValueError(kind)
    return CSR(A.m, A.n, A.row_ptr, A.col, val, A.name + "_" + kind)


def quantize(A: CSR, x: np.ndarray, kind: str):
    """Storage copies for the reduced-precision path and their exact values.

    kind "f64": unchanged.  "f32": val and x rounded to binary32.  "bf16": val
    rounded to bfloat16 (via binary32, nearest-even), x to binary32.
    Returns (val_store, x_store, val_exact, x_exact): the arrays to hand to the
    GPU (bf16 as uint16 bit patterns) and their values as float64.
    """
    if kind == "f64":
        return A.val, x, A.val, x
    x32 = round_to_f32(x)
    if kind == "f32":
        v32 = round_to_f32(A.val)
        return v32, x32, v32.astype(np.float64), x32.astype(np.float64)
    if kind == "bf16":
        bits = bf16_bits(round_to_f32(A.val))
        exact = (bits.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
        return bits, x32, exact, x32.astype(np.float64)
    raise ValueError(kind)
