"""Batched path: many uneven matrices in one launch per stage (stage 1 as
one wavefront per thread-bunch, or as a persistent grid), eager and replayed
from a HIP graph, each y_i against the oracle."""
import numpy as np
import pytest

import csrgen
import oracle
from helpers import note, assert_exact, assert_f64_parity, csr_from_lengths

pytestmark = pytest.mark.gpu


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


def batch_set(int_valued):
    """Uneven power-law matrices plus edge shapes: an all-empty matrix, a
    matrix with nnz = 0, a single long row, leading/trailing empty rows."""
    mats = csrgen.batched_set(count=24, m_lo=200, m_hi=6000, values="int" if int_valued else "uniform")
    extra = [([0] * 50, 7), ([1], 1), ([30_000], 40_000), ([0] * 300 + [4, 0, 6] * 100 + [0] * 200, 50),
             ([3, 1, 0, 0, 2] * 500, 900)]
    for k, (lengths, n) in enumerate(extra):
        mats.append(csr_from_lengths(lengths, n, seed=500 + k, int_valued=int_valued))
    return mats


def to_dev(torch, mats, dtype):
    out = []
    for A, x in mats:
        out.append((torch.from_numpy(A.row_ptr).cuda(), torch.from_numpy(A.col).cuda(),
                    torch.from_numpy(A.val).cuda().to(dtype), torch.from_numpy(x).cuda().to(dtype),
                    torch.full((A.m,), float("nan"), dtype=dtype, device="cuda"), A.n))
    return out


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("WS", [(4, 1), (8, 5), (16, 2)])
def test_batched_integer_exact(torch_cuda, WS, persistent):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    mats = batch_set(True)
    dev = to_dev(torch, mats, torch.float64)
    plan = sss.BatchPlan(dev, W=WS[0], S=WS[1], persistent=persistent)
    plan.execute()
    torch.cuda.synchronize()
    for (A, x), d in zip(mats, dev):
        assert_exact(d[4].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_row_ptr_rewritten_in_place(torch_cuda, persistent):
    """A batch plan lists its dirty bunches at plan time.  One matrix's
    row_ptr rewritten in place with empty rows (same m and nnz) makes tiles
    dirty outside the list: stage 1 marks the plan stale and stage 2's carry
    items then re-arrange those bunches too, so every y stays exact, call
    after call, and again once the first structure is written back."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    lens = np.full(4000, 9, dtype=np.int64)
    A0, x0 = csr_from_lengths(lens, 600, seed=61, int_valued=True)
    mats = [(A0, x0), csr_from_lengths([3, 1, 0, 0, 2] * 500, 900, seed=62, int_valued=True),
            csr_from_lengths([7] * 3000, 500, seed=63, int_valued=True)]
    pick = csrgen.rng_for(64).choice(4000, size=400, replace=False)
    lens2 = lens.copy()
    lens2[pick[:200]] = 0
    lens2[pick[200:]] += 9
    rp2 = np.zeros(A0.m + 1, dtype=np.int64)
    np.cumsum(lens2, out=rp2[1:])
    A0b = csrgen.CSR(A0.m, A0.n, rp2.astype(np.int32), A0.col, A0.val, "rows_emptied")
    dev = to_dev(torch, mats, torch.float64)
    plan = sss.BatchPlan(dev, W=8, S=2, persistent=persistent)

    def check(first):
        plan.execute()
        torch.cuda.synchronize()
        for k, ((A, x), d) in enumerate(zip(mats, dev)):
            A = first if k == 0 else A
            assert_exact(d[4].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x))

    check(A0)
    dev[0][0].copy_(torch.from_numpy(A0b.row_ptr).cuda())
    check(A0b)
    check(A0b)
    dev[0][0].copy_(torch.from_numpy(A0.row_ptr).cuda())
    check(A0)


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("bunches", [1, 3, 17, 33])
def test_batched_small_grids(torch_cuda, bunches, persistent):
    """Batches of 1, 3, 17 and 33 thread-bunches (W = 8, S = 5, B = 2): stage
    1's grid below 8 workgroups, and rounded up to a multiple of 8 with idle
    wavefronts in the last workgroups; the last bunch is ragged."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    nnz = 2560 * bunches - 7
    lengths = [10] * (nnz // 10) + ([nnz % 10] if nnz % 10 else [])
    mats = [csr_from_lengths(lengths, 64, seed=700 + bunches, int_valued=True),
            csr_from_lengths([0] * 5 + [3, 0, 2], 9, seed=800 + bunches, int_valued=True)]
    dev = to_dev(torch, mats, torch.float64)
    plan = sss.BatchPlan(dev, W=8, S=5, B=2, persistent=persistent)
    assert plan.info()["n_bunches"] == bunches + 1
    plan.execute()
    torch.cuda.synchronize()
    for (A, x), d in zip(mats, dev):
        assert_exact(d[4].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x))


def test_batched_per_matrix_S_and_tolerance(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    mats = batch_set(False)
    dev = to_dev(torch, mats, torch.float64)
    descs = [{"row_ptr": d[0], "col": d[1], "val": d[2], "x": d[3], "y": d[4], "n": d[5], "S": 1 + (i % 7)}
             for i, d in enumerate(dev)]
    plan = sss.BatchPlan(descs, W=8)
    plan.execute()
    torch.cuda.synchronize()
    for (A, x), d in zip(mats, dev):
        assert_f64_parity(d[4].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x),
                          oracle.abs_spmv(A.row_ptr, A.col, A.val, x))


def test_batched_graph_replays(torch_cuda):
    """Replay the captured graph several times; between replays the program
    does its own eager work (new x values, a clobbered y) and synchronises;
    every replay must equal the eager result for the current x."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    mats = batch_set(True)
    dev = to_dev(torch, mats, torch.float64)
    plan = sss.BatchPlan(dev, W=8, S=2)
    rng = np.random.default_rng(3)
    for rep in range(4):
        for (A, x), d in zip(mats, dev):
            d[3].copy_(torch.from_numpy(rng.integers(-3, 4, A.n).astype(np.float64)))
            d[4].fill_(float("nan"))
        torch.cuda.synchronize()
        plan.graph_launch()
        torch.cuda.synchronize()
        for (A, x), d in zip(mats, dev):
            xh = d[3].cpu().numpy()
            assert_exact(d[4].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, xh))
        # eager run in between must agree too
        plan.execute()
        torch.cuda.synchronize()


def test_batched_f32(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    mats = batch_set(True)
    dev = to_dev(torch, mats, torch.float32)
    plan = sss.BatchPlan(dev, dtype=torch.float32, W=16, S=2)
    plan.execute()
    torch.cuda.synchronize()
    for (A, x), d in zip(mats, dev):
        assert_exact(d[4].double().cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_bf16(torch_cuda, persistent):
    """BF16 values (x and y FP32): integer values and x in {-3..3} are exact in
    BF16 and every partial sum is exact in FP32, so each y_i is bit-exact;
    both stage-1 forms, eager and replayed."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    from helpers import to_dev_precision
    mats = batch_set(True)
    dev, refs = [], []
    for A, x in mats:
        rp, col, v, xx, ve, xe = to_dev_precision(A, x, "bf16")
        dev.append((rp, col, v, xx, torch.full((A.m,), float("nan"), dtype=torch.float32, device="cuda"), A.n))
        refs.append(oracle.spmv(A.row_ptr, A.col, ve, xe))
    plan = sss.BatchPlan(dev, dtype=torch.bfloat16, persistent=persistent)
    for launch in (plan.execute, plan.graph_launch):
        for d in dev:
            d[4].fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        for d, ref in zip(dev, refs):
            assert_exact(d[4].double().cpu().numpy(), ref)
    plan.close()


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_batched_floor_probe_reads_every_nonzero_once(torch_cuda, kind):
    """The batched measurement kernel streams exactly every matrix once: on
    integer-valued data the sum of its outputs is the sum over all matrices of
    sum_k val[k] * x[col[k]] (gather) and of sum_k (val[k] + col[k]) (stream
    only), exactly; a persistent plan is refused."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    tdt = torch.float64 if kind == "f64" else torch.float32
    mats = batch_set(True)
    dev = to_dev(torch, mats, tdt)
    plan = sss.BatchPlan(dev, dtype=tdt)
    out = torch.full((plan.info()["n_bunches"] * 64,), float("nan"), dtype=tdt, device="cuda")
    plan.floor_probe(out, gather=True)
    torch.cuda.synchronize()
    assert float(out.double().sum()) == float(sum(np.sum(A.val * x[A.col]) for A, x in mats))
    plan.floor_probe(out, gather=False)
    torch.cuda.synchronize()
    assert float(out.double().sum()) == float(sum(np.sum(A.val + A.col) for A, x in mats))
    with pytest.raises(sss.SSSError):
        sss.BatchPlan(dev, dtype=tdt, persistent=True).floor_probe(out)


def test_batched_rejects_bad_descriptors(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1()
    rp = torch.from_numpy(A.row_ptr).cuda()
    col = torch.from_numpy(A.col).cuda()
    v = torch.from_numpy(A.val).cuda()
    xx = torch.from_numpy(x).cuda()
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    colx = torch.empty(A.nnz + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(sss.SSSError):
        sss.BatchPlan([(rp, colx[1:], v, xx, y, A.n)])
    with pytest.raises(sss.SSSError):
        sss.BatchPlan([{"row_ptr": rp, "col": col, "val": v, "x": xx, "y": y, "n": A.n, "S": 99}])


_FULL = {}


def _full_set():
    """The 512-matrix batched workload (seeds 20000..20511, sum nnz ~2.8e8)
    with integer values and x in {-3..3}: every row sum is exact in FP64 and
    in FP32 (|partial| <= 9 * 2e5 < 2^24), so any order of addition gives the
    oracle's value."""
    if not _FULL:
        note("  generating the 512-matrix integer-valued batch")
        _FULL["mats"] = csrgen.batched_set(512, values="int")
        note("  oracle on 512 matrices")
        _FULL["refs"] = [oracle.spmv(A.row_ptr, A.col, A.val, x) for A, x in _FULL["mats"]]
    return _FULL["mats"], _FULL["refs"]


@pytest.mark.parametrize("kind,persistent", [("f64", False), ("f32", False), ("f64", True)])
def test_batched_full_size_exact(torch_cuda, kind, persistent):
    """All 512 matrices in the launch configuration the benchmark times (the
    per-dtype default W, S; also the persistent stage 1 in FP64), eager and
    then replayed from the captured graph with y clobbered in between: every
    row of every matrix bit-exact."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    tdt = torch.float64 if kind == "f64" else torch.float32
    mats, refs = _full_set()
    dev = to_dev(torch, mats, tdt)
    plan = sss.BatchPlan(dev, dtype=tdt, persistent=persistent)
    note(f"  {kind} batch plan {plan.info()}")
    plan.execute()
    torch.cuda.synchronize()
    for (A, _), d, ref in zip(mats, dev, refs):
        assert_exact(d[4].double().cpu().numpy(), ref)
    for d in dev:
        d[4].fill_(float("nan"))
    torch.cuda.synchronize()
    plan.graph_launch()
    torch.cuda.synchronize()
    for (A, _), d, ref in zip(mats, dev, refs):
        assert_exact(d[4].double().cpu().numpy(), ref)
    plan.close()
    del dev
    torch.cuda.empty_cache()


def test_batched_grid_schedule(torch_cuda):
    """The batch autotuner keeps the fastest class of its own timings, applies
    that S to every matrix, and its plan computes every y exactly, eager and
    replayed (integer-valued batch with edge shapes; per-matrix S ignored)."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    mats = batch_set(True)
    dev = to_dev(torch, mats, torch.float64)
    descs = [{"row_ptr": d[0], "col": d[1], "val": d[2], "x": d[3], "y": d[4], "n": d[5], "S": 3} for d in dev]
    plan, us, best = sss.BatchPlan.grid(descs, reps=2)
    assert us.shape == (12,) and np.all(us > 0)
    assert best == int(np.argmin(us))
    info = plan.info()
    assert (info["W"], info["S"]) == sss.class_params(best)
    for launch in (plan.execute, plan.graph_launch):
        for d in dev:
            d[4].fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        for (A, x), d in zip(mats, dev):
            assert_exact(d[4].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x))
    plan.close()


def _selector_schedule(sss, dev, kind_dtype, W_given=0):
    """The schedule the selector mode must produce, recomputed here from the
    library's features (size features replaced by the batch's totals) and
    class scores: W by nonzero-weighted vote of each matrix's best class
    (unless given), then each matrix's best S with that W."""
    classes = [sss.class_params(c) for c in range(12)]
    scores, votes = [], {4: 0, 8: 0, 16: 0}
    tot = [sum(d[0].numel() - 1 for d in dev), sum(d[5] for d in dev), sum(d[2].numel() for d in dev)]
    for d in dev:
        m, nnz = d[0].numel() - 1, d[2].numel()
        if m == 0 or nnz == 0:
            scores.append(None)
            continue
        f = sss.features(d[0], d[5], nnz, kind_dtype)
        f[:3] = np.log2(np.asarray(tot, dtype=np.float64) + 1.0).astype(np.float32)
        z = sss.selector_scores(f)
        scores.append(z)
        votes[classes[int(np.argmax(z))][0]] += nnz
    W = W_given or (4 if votes[4] > votes[8] and votes[4] > votes[16] else (16 if votes[16] > votes[8] else 8))
    S = []
    for z in scores:
        if z is None:
            S.append(None)
            continue
        best = max((c for c in range(12) if classes[c][0] == W), key=lambda c: z[c])
        S.append(classes[best][1])
    return W, S


@pytest.mark.parametrize("W_given", [0, 4])
def test_batched_selector_schedule(torch_cuda, W_given):
    """SELECTOR batch plans: each matrix's S is its best-scored class with the
    batch's W (chosen by the selector's votes, or given); every y exact,
    eager and replayed (integer-valued batch with edge shapes)."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    assert sss.load_selector()
    mats = batch_set(True)
    dev = to_dev(torch, mats, torch.float64)
    plan = sss.BatchPlan(dev, mode=sss.MODE_SELECTOR, W=W_given)
    W, S = plan.schedule()
    W_want, S_want = _selector_schedule(sss, dev, torch.float64, W_given)
    assert W == W_want
    for s, s_want in zip(S, S_want):
        if s_want is not None:
            assert s == s_want
    for launch in (plan.execute, plan.graph_launch):
        for d in dev:
            d[4].fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        for (A, x), d in zip(mats, dev):
            assert_exact(d[4].cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x))
    plan.close()


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_batched_selector_full_size_exact(torch_cuda, kind):
    """The 512-matrix workload with the selector's per-matrix schedule (the
    benchmark's selector-scheduled batch): every row of every matrix
    bit-exact, eager and replayed."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    assert sss.load_selector()
    tdt = torch.float64 if kind == "f64" else torch.float32
    mats, refs = _full_set()
    dev = to_dev(torch, mats, tdt)
    plan = sss.BatchPlan(dev, dtype=tdt, mode=sss.MODE_SELECTOR)
    W, S = plan.schedule()
    note(f"  {kind} selector schedule W={W} S counts {np.bincount(S, minlength=9)[[1, 2, 4, 8]].tolist()}")
    for launch in (plan.execute, plan.graph_launch):
        for d in dev:
            d[4].fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        for (A, _), d, ref in zip(mats, dev, refs):
            assert_exact(d[4].double().cpu().numpy(), ref)
    plan.close()
    del dev
    torch.cuda.empty_cache()
