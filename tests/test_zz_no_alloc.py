"""The allocation-free one-call form (sss_csr_spmv_noalloc) through the C
ABI against the one-call form with its cached plan (sss_csr_spmv): the same
kernels and parameters, so bitwise the same y, within the double-precision
tolerance of the oracle and exact on integer-valued inputs.  Two calls in a
row, the second on a smaller matrix (the static scratch keeps the first
call's contents)."""

import numpy as np
import pytest

import csrgen
import oracle
from helpers import note, to_dev, assert_exact, assert_f64_parity

pytestmark = pytest.mark.gpu

MAX_NNZ = 412_956_160  # the largest nnz whose plan arrays fit the 16 MiB scratch (default W = 8, S = 5)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1504_06474_amd import sss
    sss.lib()
    return torch


def _calls(torch, A, x):
    from paper_1504_06474_amd import sss
    L = sss.lib()
    rp, col, v, xx = to_dev(A, x)
    y_na = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
    y_ref = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    args = (A.m, A.n, A.nnz, rp.data_ptr(), col.data_ptr(), v.data_ptr(), xx.data_ptr())
    assert L.sss_csr_spmv_noalloc(*args, y_na.data_ptr(), s) == 0
    assert L.sss_csr_spmv(*args, y_ref.data_ptr(), s) == 0
    torch.cuda.synchronize()
    return y_na.cpu().numpy(), y_ref.cpu().numpy()


def test_noalloc_matches_one_call_form(torch_cuda):
    torch = torch_cuda
    big, xb = csrgen.config2(seed=3, m=300_000)
    small, xs = csrgen.config1(int_valued=True)
    for A, x, exact in ((big, xb, False), (small, xs, True)):
        note(f"[gpu-test] noalloc m={A.m} nnz={A.nnz}")
        y_na, y_ref = _calls(torch, A, x)
        assert np.array_equal(y_na.view(np.int64), y_ref.view(np.int64))
        want = oracle.spmv(A.row_ptr, A.col, A.val, x)
        if exact:
            assert_exact(y_na, want)
        else:
            assert_f64_parity(y_na, want, oracle.abs_spmv(A.row_ptr, A.col, A.val, x))
    from paper_1504_06474_amd import sss
    sss.csr_spmv_cache_clear()


def test_noalloc_size_limit(torch_cuda):
    """Beyond the scratch: SSS_ERR_TOO_LARGE before any device work (no
    pointer is read); m = 0 is a no-op."""
    from paper_1504_06474_amd import sss
    L = sss.lib()
    assert L.sss_csr_spmv_noalloc(10, 10, MAX_NNZ + 1, None, None, None, None, None, None) == -6
    assert L.sss_csr_spmv_noalloc(0, 10, 0, None, None, None, None, None, None) == 0
    assert L.sss_csr_spmv_noalloc(-1, 10, 0, None, None, None, None, None, None) == -1
