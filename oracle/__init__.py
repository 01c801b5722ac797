"""CPU oracle for speculative-segmented-sum CSR SpMV.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package.  The GPU library neither imports nor
links anything here, and nothing here imports the GPU library.

Contents
* ``spmv`` -- the plain row-loop definition of y = A x (Sections 1 and 2.1),
  evaluated in FP64 with the compensated dot product Dot2 (Ogita, Rump, Oishi
  2005), in C (``csr_oracle.c``), single- or multi-threaded.
* ``spmv_naive`` / ``spmv_rowblock`` -- the paper's CPU comparators
  (Section 4.3), used only as CPU baselines.
* ``abs_spmv`` -- (|A||x|)_i, the scale of the FP error bound for tolerances.
* ``speculative`` -- a step-by-step model of the two-stage speculative method
  (Section 3.2 and the appendix algorithm), used to pin the intermediate state
  the GPU path produces: tile start rows, segment descriptors, dirty tiles,
  speculator and synchronizer.
* ``mlp`` -- FP64 forward/backward/Adam for the tile-selector network.
* ``cg`` -- conjugate gradients (Hestenes and Stiefel) on the row-loop
  product, the checker of the library's CG calls.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

# OpenMP worker threads of the oracle sleep between calls instead of spinning:
# spinning threads compete with the thread that launches GPU work and distort
# GPU timings taken in the same process.  (Read by libgomp when it loads.)
os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
            "-shared", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        for name in ("oracle_spmv_dot2", "oracle_spmv_rowblock", "oracle_abs_spmv"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_int]
            f.restype = ctypes.c_int
        lib.oracle_spmv_naive.argtypes = [ctypes.c_int64, P, P, P, P, P]
        lib.oracle_spmv_naive.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _prep(row_ptr, col, val, x):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = row_ptr.shape[0] - 1
    if m < 0:
        raise ValueError("row_ptr must hold m+1 entries")
    nnz = int(row_ptr[-1])
    if col.shape[0] < nnz or val.shape[0] < nnz:
        raise ValueError("col/val shorter than row_ptr[m]")
    return m, row_ptr, col, val, x


def _call(fn, row_ptr, col, val, x, *extra):
    m, row_ptr, col, val, x = _prep(row_ptr, col, val, x)
    y = np.empty(m, dtype=np.float64)
    rc = fn(m, row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data, x.ctypes.data,
            y.ctypes.data, *extra)
    if rc != 0:
        raise ValueError(f"oracle returned {rc}")
    return y


def spmv(row_ptr, col, val, x, threads: int = 0) -> np.ndarray:
    """y = A x by the row-loop definition, each row by Dot2 in FP64."""
    return _call(_load().oracle_spmv_dot2, row_ptr, col, val, x, int(threads))


def spmv_naive(row_ptr, col, val, x) -> np.ndarray:
    return _call(_load().oracle_spmv_naive, row_ptr, col, val, x)


def spmv_rowblock(row_ptr, col, val, x, threads: int = 0) -> np.ndarray:
    return _call(_load().oracle_spmv_rowblock, row_ptr, col, val, x, int(threads))


def abs_spmv(row_ptr, col, val, x, threads: int = 0) -> np.ndarray:
    """(|A| |x|)_i: per-row sum of |a_ik x_k|."""
    return _call(_load().oracle_abs_spmv, row_ptr, col, val, x, int(threads))


def spmv_rows(row_ptr, col, val, x, rows) -> np.ndarray:
    """Dot2 values of selected rows only (for sampled checks at full size)."""
    rows = np.asarray(rows, dtype=np.int64)
    rp = np.asarray(row_ptr, dtype=np.int64)
    lens = rp[rows + 1] - rp[rows]
    sub_rp = np.zeros(rows.shape[0] + 1, dtype=np.int64)
    np.cumsum(lens, out=sub_rp[1:])
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows]) if rows.size else np.zeros(0, np.int64)
    return spmv(sub_rp.astype(np.int32), np.asarray(col)[idx], np.asarray(val)[idx], x)


def max_threads() -> int:
    return int(_load().oracle_max_threads())
