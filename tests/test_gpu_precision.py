"""Reduced-precision paths (FP32 and BF16 values, FP32 x/y, float products,
TwoSum-compensated segment sums, double carries) against the oracle.

* Integer-valued inputs: exact (values in {-3..3} are exact in bfloat16 and
  every partial sum here is an integer below 2^24).
* General values: within 2u (|A||x|)_i of the oracle run on the stored
  (de-quantized) values, u = 2^-24, up to second-order terms
  (helpers.f32_path_bound) -- products rounded once, compensated sums,
  partials and carries combined in double, y rounded once.
* Rows built so that rounding a row's part to float before its carry is
  added (two roundings) breaks that bound: bit-exact single rounding.
"""
import numpy as np
import pytest

import csrgen
import oracle
from helpers import note, to_dev_precision, assert_exact, assert_f32_path_bound, csr_from_lengths, f32_path_bound

pytestmark = pytest.mark.gpu

DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    from paper_1504_06474_amd import sss
    sss.lib()
    return torch


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"[gpu-test] {request.node.nodeid}")
    yield


def run(torch, A, x, kind, W=0, S=0, bind=False):
    from paper_1504_06474_amd import sss
    rp, col, v, xx, ve, xe = to_dev_precision(A, x, kind)
    plan = sss.Plan(A.m, A.n, A.nnz, dtype=getattr(torch, DT[kind]), W=W, S=S, bind_rows=bind,
                    row_ptr=rp if bind else None)
    y = plan.execute(rp, col, v, xx)
    torch.cuda.synchronize()
    return y.double().cpu().numpy(), ve, xe


@pytest.mark.parametrize("kind", ["f32", "bf16"])
@pytest.mark.parametrize("WS", [(4, 1), (8, 4), (16, 2), (16, 8)])
def test_integer_valued_exact(torch_cuda, kind, WS):
    A, x = csrgen.config1(int_valued=True)
    y, ve, xe = run(torch_cuda, A, x, kind, *WS)
    assert_exact(y, oracle.spmv(A.row_ptr, A.col, ve, xe))


@pytest.mark.parametrize("kind", ["f32", "bf16"])
@pytest.mark.parametrize("values", ["uniform", "lognormal"])
def test_config1_error_bound(torch_cuda, kind, values):
    A, x = csrgen.config1()
    A = csrgen.with_values(A, values, 77)
    y, ve, xe = run(torch_cuda, A, x, kind)
    ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
    assert_f32_path_bound(y, ref, oracle.abs_spmv(A.row_ptr, A.col, ve, xe), A.row_ptr)


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_edge_shapes(torch_cuda, kind):
    for lengths, n in (([2] * 50 + [150_000] + [1] * 3000 + [0] * 10 + [40_000], 200_000),
                       ([5] * 10 + [0] * 100_000 + [7] * 10, 100),
                       ([0] * 700 + [3, 5, 1] * 200 + [0] * 900, 400)):
        A, x = csr_from_lengths(lengths, n, seed=len(lengths), int_valued=False)
        for WS in ((4, 1), (16, 2)):
            y, ve, xe = run(torch_cuda, A, x, kind, *WS)
            ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
            assert_f32_path_bound(y, ref, oracle.abs_spmv(A.row_ptr, A.col, ve, xe), A.row_ptr)


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_config2_full_size(torch_cuda, kind):
    A, x = csrgen.config2()
    note(f"  powerlaw1e6 {kind}")
    y, ve, xe = run(torch_cuda, A, x, kind)
    ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
    assert_f32_path_bound(y, ref, oracle.abs_spmv(A.row_ptr, A.col, ve, xe), A.row_ptr)


_C5 = {}


@pytest.mark.parametrize("kind,values", [("f64", "uniform"), ("f32", "uniform"), ("bf16", "uniform"),
                                         ("f64", "lognormal"), ("f32", "lognormal"), ("bf16", "lognormal")])
def test_config5_full_size(torch_cuda, kind, values):
    """The 4M-row Zipf 1.8 matrix (80.3M nnz) in the benchmark's launch
    configuration (the type's default W and S, rows bound at plan time):
    every row against the oracle on the stored values, for uniform values and
    for the lognormal-magnitude values (sigma 3, the benchmark's seed)."""
    from helpers import assert_f64_parity
    if not _C5:
        _C5["A"], _C5["x"] = csrgen.config5()
    A, x = _C5["A"], _C5["x"]
    if values == "lognormal":
        if "L" not in _C5:
            _C5["L"] = csrgen.with_values(A, "lognormal", 55)
        A = _C5["L"]
    note(f"  zipf18_4M nnz={A.nnz} {kind} {values}")
    y, ve, xe = run(torch_cuda, A, x, kind, bind=True)
    ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
    scale = oracle.abs_spmv(A.row_ptr, A.col, ve, xe)
    if kind == "f64":
        assert_f64_parity(y, ref, scale)
    else:
        assert_f32_path_bound(y, ref, scale, A.row_ptr)


# Three terms of one row: two at the end of a tile (p1 dominant, its product
# rounded down by exactly half an ulp; p2 putting p1 + p2 just below a
# rounding midpoint) and one, c, at the start of the next tile.  The exact sum
# p1 + p2 + c needs ONE rounding to float; rounding p1 + p2 to float first and
# then adding c (two roundings) errs by about 3u |y|, beyond the 2u bound.
# Values are exact in the storage type (bf16 values, float x).
_STRADDLE = {
    "f32": ([1 + 2.0 ** -12, 2.0 ** -24 - 2.0 ** -40, 3 * 2.0 ** -24 - 2.0 ** -40], [1 + 2.0 ** -12, 1.0, 1.0]),
    "bf16": ([1 + 2.0 ** -7, 2.0 ** -24, 2.0 ** -22], [1 + 2.0 ** -17, 1 - 2.0 ** -16, 0.75 - 2.0 ** -18]),
}


def _straddle_matrix(kind, W, n_tiles, seed=3):
    """A CSR matrix with one such row across every tile boundary (so across
    every thread-bunch boundary too, whatever S), filler rows of 0..12
    entries (about 10% empty, so many tiles are dirty) between them."""
    WT = W * 64
    n = 1000
    rng = csrgen.rng_for(seed)
    v3, x3 = _STRADDLE[kind]
    lengths, cols, vals, straddle_rows = [], [], [], []

    def filler(count):
        while count > 0:
            L = int(min(count, rng.integers(0, 13)))
            lengths.append(L)
            if L:
                cols.extend(np.sort(rng.choice(np.arange(3, n), L, replace=False)).tolist())
                vals.extend(rng.uniform(-1.0, 1.0, L).tolist())
            count -= L

    for j in range(1, n_tiles):
        filler(WT - 2 if j == 1 else WT - 3)
        straddle_rows.append(len(lengths))
        lengths.append(3)
        cols.extend([0, 1, 2])
        vals.extend(v3)
    filler(WT // 2 + 5)
    rp = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=rp[1:])
    A = csrgen.CSR(len(lengths), n, rp.astype(np.int32), np.asarray(cols, dtype=np.int32),
                   np.asarray(vals, dtype=np.float64), f"straddle_{kind}_{W}")
    x = rng.uniform(-1.0, 1.0, n)
    x[:3] = x3
    return A, x, np.asarray(straddle_rows)


@pytest.mark.parametrize("kind", ["f32", "bf16"])
@pytest.mark.parametrize("WS", [(4, 1), (8, 4), (16, 2)])
def test_rows_across_bunches_rounded_once(torch_cuda, kind, WS):
    W, S = WS
    A, x, rows = _straddle_matrix(kind, W, n_tiles=40)
    y, ve, xe = run(torch_cuda, A, x, kind, W=W, S=S)
    ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
    scale = oracle.abs_spmv(A.row_ptr, A.col, ve, xe)
    bound = f32_path_bound(scale, A.row_ptr)
    # the three products, each exact or rounded once in float, as the kernel forms them
    v3, x3 = (np.asarray(a, dtype=np.float32) for a in _STRADDLE[kind])
    p = (v3 * x3).astype(np.float64)
    t = p[0] + p[1]  # exact in double
    once = np.float32(t + p[2])
    twice = np.float32(np.float64(np.float32(t)) + p[2])
    r = rows[0]
    # the construction discriminates: two roundings break the bound, one does not
    assert abs(float(twice) - ref[r]) > bound[r]
    assert abs(float(once) - ref[r]) <= bound[r]
    assert np.all(y[rows] == float(once)), (y[rows][:4], float(once), float(twice))
    assert_f32_path_bound(y, ref, scale, A.row_ptr)
