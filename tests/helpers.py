"""Shared helpers for the tests: device transfer and the comparison rules.

Floating-point parity (double): per row |y_gpu - y_oracle| <= 1e-12 * (|A||x|)_i.
The scale (|A||x|)_i = sum |a_ik x_k| bounds the rounding error of any
summation order (the method sums in a different order than the oracle), and
1e-12 stays far above the FP64 bound gamma_K * (|A||x|)_i for the K <= ~1e3
additions a row sees here.  Integer-valued inputs must match exactly.
"""
import sys

import numpy as np

F64_REL_TOL = 1e-12
U32 = 2.0 ** -24


def note(msg: str):
    """Unbuffered progress line (bypasses pytest capture)."""
    sys.__stderr__.write(msg + "\n")
    sys.__stderr__.flush()


def to_dev(A, x, val_dtype=None, x_dtype=None):
    import torch
    dev = "cuda"
    rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).to(dev)
    v = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(dev)
    xx = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)
    if val_dtype is not None:
        v = v.to(val_dtype)
    if x_dtype is not None:
        xx = xx.to(x_dtype)
    return rp, col, v, xx


def assert_f64_parity(y, y_ref, scale, tol=F64_REL_TOL):
    y = np.asarray(y, dtype=np.float64)
    err = np.abs(y - y_ref)
    bad = err > tol * scale
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{int(bad.sum())} rows out of tolerance; first row {i}: got {y[i]!r} "
                             f"want {y_ref[i]!r} scale {scale[i]!r}")


def assert_exact(y, y_ref):
    y = np.asarray(y, dtype=np.float64)
    bad = y != y_ref
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{int(bad.sum())} rows differ; first row {i}: got {y[i]!r} want {y_ref[i]!r}")


def csr_from_lengths(lengths, n, seed=0, int_valued=True):
    """A CSR matrix with the given row lengths (random unique columns)."""
    import csrgen
    rng = csrgen.rng_for(seed)
    A = csrgen.lengths_to_csr(rng, np.asarray(lengths, dtype=np.int64), n, "int" if int_valued else "uniform")
    x = csrgen.integer_values(rng, n) if int_valued else csrgen.uniform_values(rng, n)
    return A, x


def to_dev_precision(A, x, kind):
    """Device tensors for dtype kind ("f64", "f32", "bf16") and the exact
    float64 values of what was stored (for the oracle)."""
    import torch
    import csrgen
    vs, xs, ve, xe = csrgen.quantize(A, x, kind)
    dev = "cuda"
    rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).to(dev)
    if kind == "bf16":
        v = torch.from_numpy(vs.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        v = torch.from_numpy(np.ascontiguousarray(vs)).to(dev)
    xx = torch.from_numpy(np.ascontiguousarray(xs)).to(dev)
    return rp, col, v, xx, ve, xe


U64 = 2.0 ** -53


def f32_path_bound(scale, row_ptr):
    """Per-row error bound of the reduced-precision path against the oracle
    on the stored values, S = (|A||x|)_i, u = 2^-24, len = the row's length:

    * products rounded once in float:            u * S
    * y rounded once to float, |sum| <= (1+u)S:   u * (1 + u) * S
    * compensated float pairs (TwoSum, the low part summed plainly) inside a
      lane and through the 64-lane scan: each of at most 40 float additions
      into a low part errs by u * (that part) <= u * u * S:   40 u^2 * S
    * double additions of tile partials, transmitters, tails and carries: at
      most one per tile the row touches (len / 256 + 2 at W >= 4) plus 32:
      (len / 256 + 34) * 2^-53 * S
    * the oracle: Dot2 (faithful, 2^-53 |y| <= 2^-53 S), and S itself summed
      plainly in double (relative error <= len * 2^-53).
    So |y - y_ref| <= S * (2u + 41 u^2 + (len/256 + 35) 2^-53) * (1 + len 2^-53)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    length = (rp[1:] - rp[:-1]).astype(np.float64)
    per_row = 2 * U32 + 41 * U32 * U32 + (length / 256.0 + 35.0) * U64
    return scale * per_row * (1.0 + length * U64)


def assert_f32_path_bound(y, y_ref, scale, row_ptr):
    """Reduced-precision path: float products, compensated segment sums,
    partials combined in double, y rounded once: the error against the
    oracle on the stored values stays within f32_path_bound (2u (|A||x|)_i
    up to second-order terms)."""
    y = np.asarray(y, dtype=np.float64)
    bound = f32_path_bound(scale, row_ptr)
    bad = np.abs(y - y_ref) > bound
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{int(bad.sum())} rows over the bound; row {i}: got {y[i]!r} want {y_ref[i]!r} "
                             f"bound {bound[i]!r}")
