"""Reduced-precision paths (FP32 and BF16 values, FP32 x/y, float products,
TwoSum-compensated segment sums, double carries) against the oracle.

* Integer-valued inputs: exact (values in {-3..3} are exact in bfloat16 and
  every partial sum here is an integer below 2^24).
* General values: within 2u (|A||x|)_i of the oracle run on the stored
  (de-quantized) values, u = 2^-24 -- products rounded once, compensated sums,
  y rounded once.
"""
import numpy as np
import pytest

import csrgen
import oracle
from helpers import note, to_dev_precision, assert_exact, assert_f32_path_bound, csr_from_lengths

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
    assert_f32_path_bound(y, ref, oracle.abs_spmv(A.row_ptr, A.col, ve, xe))


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_edge_shapes(torch_cuda, kind):
    for lengths, n in (([2] * 50 + [150_000] + [1] * 3000 + [0] * 10 + [40_000], 200_000),
                       ([5] * 10 + [0] * 100_000 + [7] * 10, 100),
                       ([0] * 700 + [3, 5, 1] * 200 + [0] * 900, 400)):
        A, x = csr_from_lengths(lengths, n, seed=len(lengths), int_valued=False)
        for WS in ((4, 1), (16, 2)):
            y, ve, xe = run(torch_cuda, A, x, kind, *WS)
            ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
            assert_f32_path_bound(y, ref, oracle.abs_spmv(A.row_ptr, A.col, ve, xe))


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_config2_full_size(torch_cuda, kind):
    A, x = csrgen.config2()
    note(f"  powerlaw1e6 {kind}")
    y, ve, xe = run(torch_cuda, A, x, kind)
    ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
    assert_f32_path_bound(y, ref, oracle.abs_spmv(A.row_ptr, A.col, ve, xe))


_C5 = {}


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16"])
def test_config5_full_size(torch_cuda, kind):
    """The 4M-row Zipf 1.8 matrix (80.3M nnz) in the benchmark's launch
    configuration (the type's default W and S, rows bound at plan time):
    every row against the oracle on the stored values."""
    from helpers import assert_f64_parity
    if not _C5:
        _C5["A"], _C5["x"] = csrgen.config5()
    A, x = _C5["A"], _C5["x"]
    note(f"  zipf18_4M nnz={A.nnz} {kind}")
    y, ve, xe = run(torch_cuda, A, x, kind, bind=True)
    ref = oracle.spmv(A.row_ptr, A.col, ve, xe)
    scale = oracle.abs_spmv(A.row_ptr, A.col, ve, xe)
    if kind == "f64":
        assert_f64_parity(y, ref, scale)
    else:
        assert_f32_path_bound(y, ref, scale)
