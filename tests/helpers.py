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


def assert_f32_path_bound(y, y_ref, scale):
    """Reduced-precision path: float products (rounding u = 2^-24 each),
    compensated sums (O(u^2)), one final rounding of y to float: the error
    against the oracle on the stored values is at most 2u (|A||x|)_i."""
    y = np.asarray(y, dtype=np.float64)
    bound = (2 * U32) * (1 + 1e-6) * scale
    bad = np.abs(y - y_ref) > bound
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{int(bad.sum())} rows over the bound; row {i}: got {y[i]!r} want {y_ref[i]!r} "
                             f"bound {bound[i]!r}")
