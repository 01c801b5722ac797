"""The row-wise comparators (CSR-scalar, sub-wavefront groups, CSR-vector)
against the oracle: exact on integer-valued inputs for every lane count and
value type, within the FP64 tolerance on general values, on the edge shapes
where row-wise kernels break (long rows, runs of empty rows, tiny m)."""
import numpy as np
import pytest

import csrgen
import oracle
from helpers import note, to_dev, assert_exact, assert_f64_parity, csr_from_lengths

pytestmark = pytest.mark.gpu

LANES = [1, 2, 4, 8, 16, 32, 64]


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


def run(torch, A, x, lanes, vdt=None, xdt=None):
    from paper_1504_06474_amd import sss
    vdt = vdt or torch.float64
    xdt = xdt or (torch.float64 if vdt == torch.float64 else torch.float32)
    rp, col, v, xx = to_dev(A, x, val_dtype=vdt, x_dtype=xdt)
    y = torch.full((A.m,), float("nan"), dtype=xdt, device="cuda")
    sss.csr_rowwise(rp, col, v, xx, y, A.n, lanes)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("lanes", LANES)
@pytest.mark.parametrize("kind", ["f64", "f32", "bf16"])
def test_integer_exact(torch_cuda, lanes, kind):
    torch = torch_cuda
    vdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[kind]
    A, x = csrgen.config1(int_valued=True)
    assert_exact(run(torch, A, x, lanes, vdt), oracle.spmv(A.row_ptr, A.col, A.val, x))


EDGE = {
    "long_row": ([2] * 50 + [150_000] + [1] * 3000 + [0] * 10 + [40_000], 200_000),
    "empty_runs": ([5] * 10 + [0] * 100_000 + [7] * 10, 100),
    "single_row": ([1000], 1000),
    "all_empty": ([0] * 300, 50),
    "odd_m": ([3] * 77, 10),
}


@pytest.mark.parametrize("name", sorted(EDGE))
@pytest.mark.parametrize("lanes", [1, 8, 64])
def test_edge_integer_exact(torch_cuda, name, lanes):
    lengths, n = EDGE[name]
    A, x = csr_from_lengths(lengths, n, seed=len(lengths))
    note(f"  {name} m={A.m} nnz={A.nnz} lanes={lanes}")
    assert_exact(run(torch_cuda, A, x, lanes), oracle.spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("lanes", [1, 64])
def test_general_values_f64(torch_cuda, lanes):
    A, x = csrgen.config1()
    assert_f64_parity(run(torch_cuda, A, x, lanes), oracle.spmv(A.row_ptr, A.col, A.val, x),
                      oracle.abs_spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("matrix", ["powerlaw_1M", "zipf18_4M"])
@pytest.mark.parametrize("lanes", [1, 64])
def test_benchmark_matrix_every_row(torch_cuda, lanes, matrix):
    """The 1M-row power-law matrix (19.2M nonzeros, a 197,189-entry row) and
    the 4M-row Zipf 1.8 matrix (80.3M nonzeros), on which the benchmark times
    the comparators: every row against the oracle within
    the bound of plain summation in any order, gamma_k (|A||x|)_i with
    gamma_k = k u / (1 - k u), k the row's length and u = 2^-53, plus the
    oracle's own error (compensated: u |y_i| + gamma_k^2 (|A||x|)_i)."""
    A, x = csrgen.config2() if matrix == "powerlaw_1M" else csrgen.config5()
    got = run(torch_cuda, A, x, lanes)
    want = oracle.spmv(A.row_ptr, A.col, A.val, x)
    scale = oracle.abs_spmv(A.row_ptr, A.col, A.val, x)
    k = np.diff(A.row_ptr).astype(np.float64)
    u = 2.0 ** -53
    gamma = k * u / (1.0 - k * u)
    bound = gamma * scale + u * np.abs(want) + gamma * gamma * scale
    err = np.abs(got - want)
    ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), 0.0)
    i = int(np.argmax(ratio))
    note(f"  lanes={lanes}: max err / bound {ratio[i]:.3f} (row length {int(k[i])})")
    assert np.all(err <= bound), int(np.sum(err > bound))
    assert np.all(got[k == 0] == 0.0)
