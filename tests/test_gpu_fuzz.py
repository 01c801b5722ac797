"""Seeded random matrices against the oracle, bit-exact (integer values and x
in {-3..3}): row-length mixes that stress the method's corner cases -- runs of
empty rows, rows spanning many thread-bunches, rows ending exactly on tile
boundaries -- under random (W, S, B), searched or bound first rows, FP64,
FP32 or BF16 values, and random batches with per-matrix S in either stage-1
form.  Integer values and x in {-3..3} are exact in BF16, and every partial
sum (|s| <= 9 * 40 * 1024 < 2^24) is exact in FP32, so every type is
compared bit for bit."""
import numpy as np
import pytest

import csrgen
import oracle
from helpers import note, to_dev, to_dev_precision, assert_exact

pytestmark = pytest.mark.gpu


def random_lengths(rng, W):
    """A row-length sequence mixing the structures the method treats
    specially; W*64 (one tile) is used to place rows on tile boundaries."""
    WT = W * 64
    parts = []
    for _ in range(int(rng.integers(1, 12))):
        kind = int(rng.integers(0, 6))
        k = int(rng.integers(1, 400))
        if kind == 0:
            parts.append(np.zeros(k, np.int64))                       # a run of empty rows
        elif kind == 1:
            parts.append(rng.integers(0, 12, k))                      # short rows, some empty
        elif kind == 2:
            parts.append(np.full(int(rng.integers(1, 4)), int(rng.integers(WT, 40 * WT))))  # rows over many tiles
        elif kind == 3:
            parts.append(np.full(int(rng.integers(1, 20)), WT))       # rows that are exactly one tile
        elif kind == 4:
            parts.append(np.full(k, int(rng.integers(1, 3))))         # many tiny rows
        else:
            L = rng.integers(0, 30, k)
            L[rng.random(k) < 0.5] = 0                                 # half empty
            parts.append(L)
    return np.concatenate(parts)


def random_matrix(seed, W):
    rng = np.random.default_rng(seed)
    lengths = random_lengths(rng, W)
    n = int(rng.integers(1, 3000)) if rng.random() < 0.5 else int(rng.integers(50_000, 200_000))
    lengths = np.minimum(lengths, n)  # unique columns per row
    A = csrgen.lengths_to_csr(rng, lengths, n, "int")
    x = csrgen.integer_values(rng, n)
    return A, x


@pytest.mark.parametrize("seed", range(400))
def test_fuzz_single(seed):
    import torch
    from paper_1504_06474_amd import sss
    rng = np.random.default_rng(1000 + seed)
    W = int(rng.choice([4, 8, 16]))
    S = int(rng.integers(1, 17))
    B = int(rng.integers(1, 5))
    bind = bool(rng.integers(0, 2))
    kind = ("f64", "f32", "bf16")[int(rng.integers(0, 3))]
    A, x = random_matrix(seed, W)
    note(f"  seed={seed} m={A.m} n={A.n} nnz={A.nnz} W={W} S={S} B={B} bind={bind} {kind}")
    rp, col, v, xx, ve, xe = to_dev_precision(A, x, kind)
    plan = sss.Plan(A.m, A.n, A.nnz, dtype=v.dtype, W=W, S=S, B=B, bind_rows=bind, row_ptr=rp if bind else None)
    y = torch.full((A.m,), float("nan"), dtype=xx.dtype, device="cuda")
    plan.execute(rp, col, v, xx, y)
    torch.cuda.synchronize()
    assert_exact(y.double().cpu().numpy(), oracle.spmv(A.row_ptr, A.col, ve, xe))


@pytest.mark.parametrize("seed", range(40))
def test_fuzz_batched(seed):
    import torch
    from paper_1504_06474_amd import sss
    rng = np.random.default_rng(5000 + seed)
    W = int(rng.choice([4, 8, 16]))
    mats = [random_matrix(10_000 * (seed + 1) + i, W) for i in range(int(rng.integers(1, 24)))]
    descs, refs = [], []
    for A, x in mats:
        rp, col, v, xx = to_dev(A, x)
        y = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
        descs.append({"row_ptr": rp, "col": col, "val": v, "x": xx, "y": y, "n": A.n, "S": int(rng.integers(1, 17))})
        refs.append(oracle.spmv(A.row_ptr, A.col, A.val, x))
    persistent = bool(rng.integers(0, 2))
    note(f"  seed={seed} matrices={len(mats)} W={W} nnz={sum(A.nnz for A, _ in mats)} persistent={persistent}")
    plan = sss.BatchPlan(descs, W=W, persistent=persistent)
    plan.execute()
    torch.cuda.synchronize()
    for d, ref in zip(descs, refs):
        assert_exact(d["y"].cpu().numpy(), ref)


@pytest.mark.parametrize("seed", range(60))
def test_fuzz_stage2_on_host(seed):
    """The paper's split on random matrices: stage 1 on the device, then the
    carries, the re-arrangement and the leading rows on a host core
    (sss_csr_spmv_stage2_host), bit-exact against the oracle in FP64 and in
    FP32."""
    import torch
    from paper_1504_06474_amd import sss
    rng = np.random.default_rng(9000 + seed)
    W = int(rng.choice([4, 8, 16]))
    S = int(rng.integers(1, 17))
    bind = bool(rng.integers(0, 2))
    kind = ("f64", "f32")[int(rng.integers(0, 2))]
    A, x = random_matrix(20_000 + seed, W)
    note(f"  seed={seed} m={A.m} nnz={A.nnz} W={W} S={S} bind={bind} {kind}")
    rp, col, v, xx, ve, xe = to_dev_precision(A, x, kind)
    plan = sss.Plan(A.m, A.n, A.nnz, dtype=v.dtype, W=W, S=S, bind_rows=bind, row_ptr=rp if bind else None)
    y = torch.full((A.m,), float("nan"), dtype=xx.dtype, device="cuda")
    plan.stage1(rp, col, v, xx, y)
    torch.cuda.synchronize()
    y_host = y.cpu()
    plan.stage2_host(A.row_ptr, y_host)
    assert_exact(y_host.double().numpy(), oracle.spmv(A.row_ptr, A.col, ve, xe))


@pytest.mark.parametrize("seed", range(40))
def test_fuzz_bound_plan_row_ptr_rewritten(seed):
    """A plan bound to a row_ptr array whose contents are then replaced in
    place by another structure with the same m and nnz (the row lengths
    shuffled): stage 1 finds the stored first rows stale and searches again,
    stage 2 takes the unlisted dirty bunches too; y stays exact, on two calls
    in a row."""
    import torch
    from paper_1504_06474_amd import sss
    rng = np.random.default_rng(12_000 + seed)
    W = int(rng.choice([4, 8, 16]))
    S = int(rng.integers(1, 17))
    A, x = random_matrix(30_000 + seed, W)
    lengths = np.diff(A.row_ptr.astype(np.int64))
    A2 = csrgen.lengths_to_csr(rng, rng.permutation(lengths), A.n, "int")
    note(f"  seed={seed} m={A.m} nnz={A.nnz} W={W} S={S}")
    rp, col, v, xx = to_dev(A, x)
    plan = sss.Plan(A.m, A.n, A.nnz, W=W, S=S, bind_rows=True, row_ptr=rp)
    rp.copy_(torch.from_numpy(A2.row_ptr.astype(np.int32)).cuda())
    col2 = torch.from_numpy(A2.col).cuda()
    v2 = torch.from_numpy(A2.val).cuda()
    want = oracle.spmv(A2.row_ptr, A2.col, A2.val, x)
    for _ in range(2):
        y = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
        plan.execute(rp, col2, v2, xx, y)
        torch.cuda.synchronize()
        assert_exact(y.cpu().numpy(), want)


@pytest.mark.parametrize("seed", range(24))
def test_fuzz_execute_replayed_from_a_graph(seed):
    """execute captured once into a graph on random matrices and types, then
    replayed three times with a new x and y clobbered by the program's own
    eager work in between: every replay is exact."""
    import torch
    from paper_1504_06474_amd import sss
    rng = np.random.default_rng(15_000 + seed)
    W = int(rng.choice([4, 8, 16]))
    S = int(rng.integers(1, 17))
    bind = bool(rng.integers(0, 2))
    kind = ("f64", "f32", "bf16")[int(rng.integers(0, 3))]
    A, x = random_matrix(40_000 + seed, W)
    note(f"  seed={seed} m={A.m} nnz={A.nnz} W={W} S={S} bind={bind} {kind}")
    rp, col, v, xx, ve, xe = to_dev_precision(A, x, kind)
    plan = sss.Plan(A.m, A.n, A.nnz, dtype=v.dtype, W=W, S=S, bind_rows=bind, row_ptr=rp if bind else None)
    y = torch.empty(A.m, dtype=xx.dtype, device="cuda")
    plan.execute(rp, col, v, xx, y)  # first call outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(rp, col, v, xx, y)
    for rep in range(3):
        xh = csrgen.integer_values(rng, A.n)  # exact in every type
        xx.copy_(torch.from_numpy(xh).to(xx.dtype))
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_exact(y.double().cpu().numpy(), oracle.spmv(A.row_ptr, A.col, ve, xh))
        plan.execute(rp, col, v, xx, y)  # eager work between replays
        torch.cuda.synchronize()
    del g


@pytest.mark.parametrize("seed", range(12))
def test_fuzz_batched_graph_replays(seed):
    """Random batches run from the plan's own graph (sss_batch_graph_launch,
    captured on the first call) three times, with every x rewritten and every
    y clobbered by eager work in between: exact each time."""
    import torch
    from paper_1504_06474_amd import sss
    rng = np.random.default_rng(18_000 + seed)
    W = int(rng.choice([4, 8, 16]))
    mats = [random_matrix(50_000 * (seed + 1) + i, W) for i in range(int(rng.integers(1, 16)))]
    descs = []
    for A, x in mats:
        rp, col, v, xx = to_dev(A, x)
        y = torch.empty(A.m, dtype=torch.float64, device="cuda")
        descs.append({"row_ptr": rp, "col": col, "val": v, "x": xx, "y": y, "n": A.n, "S": int(rng.integers(1, 17))})
    persistent = bool(rng.integers(0, 2))
    note(f"  seed={seed} matrices={len(mats)} W={W} persistent={persistent}")
    plan = sss.BatchPlan(descs, W=W, persistent=persistent)
    for rep in range(3):
        xs = [csrgen.integer_values(rng, A.n) for A, _ in mats]
        for d, xh in zip(descs, xs):
            d["x"].copy_(torch.from_numpy(xh))
            d["y"].fill_(float("nan"))
        torch.cuda.synchronize()
        plan.graph_launch()
        torch.cuda.synchronize()
        for d, (A, _), xh in zip(descs, mats, xs):
            assert_exact(d["y"].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, xh))
        plan.execute()  # eager work between replays
        torch.cuda.synchronize()
