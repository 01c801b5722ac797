"""Maximum sizes on the device: nnz at the library's index limit
(SSS_MAX_INDEX = 2^31 - 4097, ~26 GB of FP64 values and int32 columns), m at
that limit (2^31 - 4097 rows, mostly empty), and one batch whose total nnz
passes 2^31 (its global bunch index space is 64-bit).

The matrices are generated on the device with col[k] = k mod n and
val[k] = 1 + (k mod 2), and x is integer-valued, so every partial sum is an
integer below 2^53 and y is exact whatever the order of the additions.  The
expected y comes from the definition of the product (Section 2.1: y_r is the
sum of val[k] x[col[k]] over the row's entries) in closed form: with
P(K) = sum_{k<K} (1 + k mod 2) x[k mod n], which repeats with period 2n,
y_r = P(row_ptr[r+1]) - P(row_ptr[r]).  Those prefix sums are computed on
the host in exact integer arithmetic; nothing expected comes from the
kernels.
"""
import numpy as np
import pytest

from helpers import note, assert_f32_path_bound

MAX_INDEX = 2147479551  # SSS_MAX_INDEX
CHUNK = 1 << 27


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


class Prefix:
    """P(K) = sum_{k<K} (1 + k mod 2) x[k mod n] for integer-valued x, exactly."""

    def __init__(self, x: np.ndarray):
        n = x.size
        self.T = 2 * n
        k = np.arange(self.T, dtype=np.int64)
        w = (1 + (k & 1)) * x[k % n].astype(np.int64)
        self.pre = np.concatenate([[0], np.cumsum(w)])
        self.per_period = int(self.pre[-1])

    def __call__(self, K) -> np.ndarray:
        K = np.asarray(K, dtype=np.int64)
        return (K // self.T) * self.per_period + self.pre[K % self.T]


def expected_y(rp: np.ndarray, P: Prefix) -> np.ndarray:
    rp = rp.astype(np.int64)
    return (P(rp[1:]) - P(rp[:-1])).astype(np.float64)


def fill_entries(torch, col, val, n: int):
    """col[k] = k mod n, val[k] = 1 + (k mod 2), on the device in chunks."""
    nnz = col.numel()
    for s in range(0, nnz, CHUNK):
        e = min(nnz, s + CHUNK)
        k = torch.arange(s, e, dtype=torch.int64, device="cuda")
        col[s:e] = (k % n).to(torch.int32)
        val[s:e] = (1 + (k & 1)).to(val.dtype)
        del k


def ragged_row_ptr(m: int, nnz: int, seed: int) -> np.ndarray:
    """Row lengths around nnz / m with 5% empty rows, empty leading and
    trailing rows, and one long row that takes the remainder (it spans many
    thread-bunches, so its carries form a long synchronizer run)."""
    rng = np.random.default_rng(seed)
    base = nnz // m
    lengths = rng.integers(0, 2 * base, size=m).astype(np.int64)
    lengths[rng.random(m) < 0.05] = 0
    lengths[:3] = 0
    lengths[-100:] = 0
    lengths[7] = 0
    lengths[7] = nnz - lengths.sum()
    assert lengths[7] > 100 * base
    rp = np.concatenate([[0], np.cumsum(lengths)])
    assert rp[-1] == nnz
    return rp.astype(np.int32)


def int_x(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(-8, 9, size=n).astype(np.float64)


def test_closed_form_matches_the_oracle():
    """The closed form against the oracle's product on small matrices of the
    same structure (ragged rows, empty leading, trailing and inner rows, a
    long row; n odd and even, so the period 2n and the parity interact)."""
    import oracle
    for m, n, nnz, seed in ((1_001, 97, 60_000, 1), (777, 64, 50_000, 2), (300, 1, 40_000, 3)):
        rp = ragged_row_ptr(m, nnz, seed)
        x = int_x(n, seed)
        k = np.arange(nnz, dtype=np.int64)
        col = (k % n).astype(np.int32)
        val = (1 + (k & 1)).astype(np.float64)
        want = oracle.spmv(rp, col, val, x)
        assert np.array_equal(expected_y(rp, Prefix(x)), want)
        # and P itself at K past several periods, by direct summation
        P = Prefix(x)
        for K in (0, 1, 2 * n - 1, 2 * n, 5 * n + 3, nnz):
            kk = np.arange(K, dtype=np.int64)
            assert int(P(K)) == int(np.sum((1 + (kk & 1)) * x[kk % n].astype(np.int64)))


@pytest.mark.gpu
def test_nnz_at_index_limit(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    m, n, nnz = 1_048_573, 1_000_003, MAX_INDEX
    rp = ragged_row_ptr(m, nnz, 31)
    x = int_x(n, 32)
    want = expected_y(rp, Prefix(x))
    rp_d, x_d = torch.from_numpy(rp).cuda(), torch.from_numpy(x).cuda()
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz, dtype=torch.float64, device="cuda")
    fill_entries(torch, col, val, n)
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    for kw in ({}, {"W": 4, "S": 1, "B": 1}, {"W": 16, "S": 8, "B": 2}):
        for bind in (False, True):
            note(f"[gpu-test]   plan {kw} bind_rows={bind}")
            plan = sss.Plan(m, n, nnz, bind_rows=bind, row_ptr=rp_d if bind else None, **kw)
            y.fill_(float("nan"))
            plan.execute(rp_d, col, val, x_d, y)
            torch.cuda.synchronize()
            got = y.cpu().numpy()
            assert np.array_equal(got, want), (kw, bind, int(np.sum(got != want)))
            plan.close()
    del col, val, y
    torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_nnz_at_index_limit_reduced_precision(torch_cuda, kind):
    """The same matrix with FP32 or BF16 values (1 and 2 are exact in both)
    and an FP32 x: rows whose sums stay below 2^24 come out exact, and every
    row, the 108M-entry one included, within the reduced-precision path's
    bound of 2u (|A||x|)_i against the exact product, (|A||x|)_i being the
    same closed form over |x|."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    m, n, nnz = 1_048_573, 1_000_003, MAX_INDEX
    rp = ragged_row_ptr(m, nnz, 31)
    x = int_x(n, 32)
    want = expected_y(rp, Prefix(x))
    scale = expected_y(rp, Prefix(np.abs(x)))
    vt = torch.float32 if kind == "f32" else torch.bfloat16
    rp_d, x_d = torch.from_numpy(rp).cuda(), torch.from_numpy(x).float().cuda()
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz, dtype=vt, device="cuda")
    fill_entries(torch, col, val, n)
    y = torch.empty(m, dtype=torch.float32, device="cuda")
    for kw in ({}, {"W": 4, "S": 1, "B": 1}, {"W": 16, "S": 8, "B": 2}):
        note(f"[gpu-test]   {kind} plan {kw}")
        plan = sss.Plan(m, n, nnz, dtype=vt, bind_rows=True, row_ptr=rp_d, **kw)
        y.fill_(float("nan"))
        plan.execute(rp_d, col, val, x_d, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy().astype(np.float64)
        small = np.abs(scale) < 2 ** 24
        assert np.array_equal(got[small], want[small]), (kind, kw)
        assert_f32_path_bound(got, want, scale, rp)
        plan.close()
    del col, val, y
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_rows_at_index_limit(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    m, n, nnz = MAX_INDEX, 1_000_003, 150_000_007
    x = int_x(n, 33)
    P = Prefix(x)
    # row_ptr[r] = floor(r nnz / m): rows of 0 or 1 entries, ~93% empty
    rp_d = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    for s in range(0, m + 1, CHUNK):
        e = min(m + 1, s + CHUNK)
        r = torch.arange(s, e, dtype=torch.int64, device="cuda")
        rp_d[s:e] = (r * nnz // m).to(torch.int32)
        del r
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz, dtype=torch.float64, device="cuda")
    fill_entries(torch, col, val, n)
    x_d = torch.from_numpy(x).cuda()
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    total = float(P(nnz))
    windows = [0, 5_000_003, m // 3, m // 2 + 12_345, m - 1_000_000]
    for bind in (True, False):
        note(f"[gpu-test]   default plan, bind_rows={bind}")
        plan = sss.Plan(m, n, nnz, bind_rows=bind, row_ptr=rp_d if bind else None)
        y.fill_(float("nan"))
        plan.execute(rp_d, col, val, x_d, y)
        torch.cuda.synchronize()
        # every row: the integer-valued total is exact in any order (|y| < 2^36)
        assert float(y.sum()) == total
        for s in windows:
            e = min(m, s + 1_000_000)
            r = np.arange(s, e + 1, dtype=np.int64)
            want = expected_y(r * nnz // m, P)
            assert np.array_equal(y[s:e].cpu().numpy(), want), (bind, s)
        plan.close()
    del rp_d, col, val, y
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_batch_total_nnz_past_int32(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    shapes = [(600_001, 700_001, 1_200_000_000, 41), (400_003, 300_007, 1_000_000_003, 42)]
    assert sum(s[2] for s in shapes) > 2 ** 31
    mats, wants = [], []
    for m, n, nnz, seed in shapes:
        rp = ragged_row_ptr(m, nnz, seed)
        x = int_x(n, seed + 100)
        wants.append(expected_y(rp, Prefix(x)))
        col = torch.empty(nnz, dtype=torch.int32, device="cuda")
        val = torch.empty(nnz, dtype=torch.float64, device="cuda")
        fill_entries(torch, col, val, n)
        mats.append({"row_ptr": torch.from_numpy(rp).cuda(), "col": col, "val": val,
                     "x": torch.from_numpy(x).cuda(), "y": torch.empty(m, dtype=torch.float64, device="cuda"),
                     "n": n})
    for kw in ({}, {"W": 4, "S": 1}, {"persistent": True}):
        note(f"[gpu-test]   batch plan {kw}")
        bp = sss.BatchPlan(mats, dtype=torch.float64, **kw)
        for d in mats:
            d["y"].fill_(float("nan"))
        bp.execute()
        torch.cuda.synchronize()
        for i, d in enumerate(mats):
            got = d["y"].cpu().numpy()
            assert np.array_equal(got, wants[i]), (kw, i, int(np.sum(got != wants[i])))
        bp.close()
    del mats
    torch.cuda.empty_cache()
