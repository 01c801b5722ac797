"""CG through the library (sss_cg_start, sss_cg_iterate), one bound plan
reused for every product: the state after k steps against the CG oracle
(oracle/cg.py) on a 2D Laplacian, a Laplacian larger than one pass of the
vector kernels' grid with a ragged tail, an irregular SPD matrix with
power-law rows, and the benchmark's 1M-row Laplacian in the selector's plan;
the solution against a dense direct solve; a run repeated
bit for bit; a zero right-hand side; and the calls' argument checks."""
import ctypes

import numpy as np
import pytest

import csrgen
from helpers import note
from oracle import cg as ocg

pytestmark = pytest.mark.gpu

# Two FP64 runs of the iteration that differ only in rounding order (the
# oracle's compensated row sums and numpy's dots against the kernels' sums)
# stay within ~1e-14 of each other over these step counts on these matrices;
# a wrong term, sign or step size is off by far more.
REL_TOL = 1e-11


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


def irregular_spd(m, seed):
    """B + B^T plus a diagonal that dominates every row: symmetric positive
    definite, with power-law row lengths (up to a few thousand entries)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    lens = np.minimum((rng.pareto(1.2, m) * 2).astype(np.int64), 3000)
    rows = np.repeat(np.arange(m), lens)
    cols = rng.integers(0, m, int(lens.sum()))
    B = sp.csr_matrix((rng.uniform(-1, 1, rows.size), (rows, cols)), shape=(m, m))
    S = (B + B.T).tocsr()
    d = np.asarray(abs(S).sum(axis=1)).ravel() + 1.0
    A = (S + sp.diags(d)).tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)


def matrix(name):
    if name == "irregular_spd_40k":
        return irregular_spd(40_013, 11)
    # 600^2 = 360,000 rows: the vector kernels' workgroups take more than one
    # grid stride, with a ragged tail; 1024^2 is the benchmark's solver workload
    L = csrgen.laplacian2d_csr(int(name.split("_")[1]))
    return L.row_ptr, L.col, L.val


class State:
    def __init__(self, torch, sss, rp, col, val, b, x0, **plan_kw):
        self.torch, self.sss = torch, sss
        m = rp.size - 1
        self.rp, self.col, self.val = (torch.from_numpy(a).cuda() for a in (rp, col, val))
        self.plan = sss.Plan(m, m, val.size, bind_rows=True, row_ptr=self.rp, **plan_kw)
        self.b = torch.from_numpy(b).cuda()
        self.x = torch.from_numpy(x0).cuda()
        self.r, self.p, self.q = (torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
                                  for _ in range(3))
        self.work = torch.full((sss.cg_workspace_size() // 8,), float("nan"), dtype=torch.float64, device="cuda")
        sss.cg_start(self.plan, self.rp, self.col, self.val, self.b, self.x, self.r, self.p, self.q, self.work)

    def iterate(self, k):
        self.sss.cg_iterate(self.plan, self.rp, self.col, self.val, self.x, self.r, self.p, self.q, self.work, k)

    def host(self):
        self.torch.cuda.synchronize()
        w = self.work[:3].cpu().numpy()
        return {"x": self.x.cpu().numpy(), "r": self.r.cpu().numpy(), "p": self.p.cpu().numpy(),
                "rr": w[0], "rr_prev": w[1], "bb": w[2]}


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


@pytest.mark.parametrize("name", ["laplacian_30", "laplacian_600", "irregular_spd_40k", "laplacian_1024"])
def test_cg_steps_match_the_oracle(torch_cuda, name):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    rp, col, val = matrix(name)
    m = rp.size - 1
    rng = np.random.default_rng(21)
    b = rng.uniform(-1, 1, m)
    x0 = rng.uniform(-1, 1, m) if name in ("laplacian_30", "irregular_spd_40k") else np.zeros(m)
    # the benchmark's launch configuration for its solver workload: the selector's plan
    kw = {"mode": sss.MODE_SELECTOR} if name == "laplacian_1024" else {}
    st = State(torch, sss, rp, col, val, b, x0, **kw)
    done = 0
    for k in (0, 1, 2, 5, 20):
        st.iterate(k - done)
        done = k
        got = st.host()
        want = ocg.cg_steps(rp, col, val, b, x0, k)
        errs = {key: rel(got[key], want[key]) for key in ("x", "r", "p")}
        errs.update({key: abs(got[key] - want[key]) / want[key] for key in ("rr", "rr_prev", "bb")})
        note(f"  {name} k={k}: " + " ".join(f"{key} {e:.1e}" for key, e in errs.items()))
        assert all(np.isfinite(list(errs.values())))
        assert max(errs.values()) <= REL_TOL, (k, errs)


@pytest.mark.parametrize("m", [1, 2, 3, 257, 1025, 262_145])
def test_cg_edge_sizes(torch_cuda, m):
    """Sizes where the vector kernels have one workgroup, a partial
    workgroup, or a grid stride one element past a whole number of strides
    (262,145 = 256 threads x 4 elements x 256 workgroups + 1).  The small
    systems are solved within the three steps, so r and p are compared
    against the size of the starting residual and x against the solution."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    rp, col, val = irregular_spd(m, 100 + m)
    rng = np.random.default_rng(m)
    b = rng.uniform(-1, 1, m)
    x0 = rng.uniform(-1, 1, m)
    st = State(torch, sss, rp, col, val, b, x0)
    st.iterate(3)
    got = st.host()
    want = ocg.cg_steps(rp, col, val, b, x0, 3)
    rr0 = ocg.cg_steps(rp, col, val, b, x0, 0)["rr"]
    errs = {"x": rel(got["x"], want["x"])}
    errs.update({key: np.linalg.norm(got[key] - want[key]) / np.sqrt(rr0) for key in ("r", "p")})
    errs.update({key: abs(got[key] - want[key]) / rr0 for key in ("rr", "rr_prev")})
    errs["bb"] = abs(got["bb"] - want["bb"]) / want["bb"]
    note(f"  m={m}: " + " ".join(f"{key} {e:.1e}" for key, e in errs.items()))
    assert all(np.isfinite(list(errs.values())))
    assert max(errs.values()) <= REL_TOL, errs


def test_cg_empty_system(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    plan = sss.Plan(0, 0, 0)
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    val = torch.zeros(0, dtype=torch.float64, device="cuda")
    vec = [torch.zeros(0, dtype=torch.float64, device="cuda") for _ in range(5)]
    work = torch.full((sss.cg_workspace_size() // 8,), float("nan"), dtype=torch.float64, device="cuda")
    sss.cg_start(plan, rp, col, val, *vec, work)
    sss.cg_iterate(plan, rp, col, val, *vec[1:], work, 3)
    torch.cuda.synchronize()
    assert work[:3].tolist() == [0.0, 0.0, 0.0]


def test_cg_solution_matches_direct_solve(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    from paper_1504_06474_amd.cg import cg
    A = csrgen.laplacian2d_csr(30)
    rng = np.random.default_rng(7)
    x_true = rng.uniform(-1, 1, A.n)
    dense = np.zeros((A.m, A.n))
    for i in range(A.m):
        dense[i, A.col[A.row_ptr[i]:A.row_ptr[i + 1]]] = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
    b = dense @ x_true
    x_ref = np.linalg.solve(dense, b)
    rp, col, v = (torch.from_numpy(a).cuda() for a in (A.row_ptr, A.col, A.val))
    plan = sss.Plan(A.m, A.n, A.nnz, W=4, S=1, bind_rows=True, row_ptr=rp)
    x, it, hist = cg(plan, rp, col, v, torch.from_numpy(b).cuda(), rtol=1e-11, max_iter=2000)
    note(f"  CG: {it} iterations, final relative residual {hist[-1][1]:.2e}")
    assert hist[-1][1] <= 1e-11
    assert all(h[0] % 10 == 0 for h in hist) and hist[-1][0] == it
    err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    assert err < 1e-8, err


def test_cg_repeats_bit_for_bit(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    rp, col, val = irregular_spd(40_013, 12)
    b = np.random.default_rng(3).uniform(-1, 1, rp.size - 1)
    runs = []
    for _ in range(2):
        st = State(torch, sss, rp, col, val, b, np.zeros(rp.size - 1), W=8, S=2)
        st.iterate(15)
        runs.append(st.host())
    for key in ("x", "r", "p"):
        assert np.array_equal(runs[0][key], runs[1][key]), key
    assert runs[0]["rr"] == runs[1]["rr"]


def test_cg_zero_rhs_stays_at_zero(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    L = csrgen.laplacian2d_csr(20)
    st = State(torch, sss, L.row_ptr, L.col, L.val, np.zeros(L.m), np.zeros(L.m))
    st.iterate(4)
    got = st.host()
    for key in ("x", "r", "p"):
        assert np.all(got[key] == 0.0), key
    assert got["rr"] == 0.0 and got["rr_prev"] == 0.0 and got["bb"] == 0.0


def test_cg_argument_checks(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    L = csrgen.laplacian2d_csr(10)
    rp, col, v = (torch.from_numpy(a).cuda() for a in (L.row_ptr, L.col, L.val))
    vec = [torch.zeros(L.m, dtype=torch.float64, device="cuda") for _ in range(5)]
    work = torch.zeros(sss.cg_workspace_size() // 8 + 1, dtype=torch.float64, device="cuda")
    lib = sss.lib()
    P = [t.data_ptr() for t in vec]
    f64 = sss.Plan(L.m, L.n, L.nnz, bind_rows=True, row_ptr=rp)
    h = f64.handle
    # misaligned work, negative iterations, NULL work, NULL plan
    assert lib.sss_cg_start(h, rp.data_ptr(), col.data_ptr(), v.data_ptr(), *P, work.data_ptr() + 4, None) == -1
    assert lib.sss_cg_iterate(h, rp.data_ptr(), col.data_ptr(), v.data_ptr(), *P[1:], work.data_ptr(), -1,
                              None) == -1
    assert lib.sss_cg_iterate(h, rp.data_ptr(), col.data_ptr(), v.data_ptr(), *P[1:], None, 1, None) == -1
    assert lib.sss_cg_start(None, rp.data_ptr(), col.data_ptr(), v.data_ptr(), *P, work.data_ptr(), None) == -1
    # another row_ptr than the bound plan's: the product's own check
    rp2 = rp.clone()
    assert lib.sss_cg_iterate(h, rp2.data_ptr(), col.data_ptr(), v.data_ptr(), *P[1:], work.data_ptr(), 1,
                              None) == -3
    # an FP32 plan, and a non-square one
    f32 = sss.Plan(L.m, L.n, L.nnz, dtype=torch.float32)
    assert lib.sss_cg_start(f32.handle, rp.data_ptr(), col.data_ptr(), v.data_ptr(), *P, work.data_ptr(),
                            None) == -2
    rect = sss.Plan(L.m, L.n + 1, L.nnz)
    assert lib.sss_cg_iterate(rect.handle, rp.data_ptr(), col.data_ptr(), v.data_ptr(), *P[1:], work.data_ptr(),
                              1, None) == -1
    size = ctypes.c_size_t()
    assert lib.sss_cg_workspace_size(None) == -1
    assert lib.sss_cg_workspace_size(ctypes.byref(size)) == 0 and size.value >= 24
    with pytest.raises(ValueError):
        sss.cg_iterate(f32, rp, col, v, *vec[1:], work, 1)
    torch.cuda.synchronize()
