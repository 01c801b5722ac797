"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Double precision: per-row tolerance 1e-12 * (|A||x|)_i; integer-valued inputs
bit-exact.  The debug dump of stage 1 (tile start rows, segment descriptors,
dirty tiles, speculator, synchronizer) must equal the oracle's definitions
exactly, at T = 64.
"""
import math

import numpy as np
import pytest

import csrgen
import oracle
from oracle import speculative as sp
from helpers import note, to_dev, assert_f64_parity, assert_exact, csr_from_lengths

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1504_06474_amd import sss
    sss.lib()  # fails loudly if the library is not built
    return torch


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"[gpu-test] {request.node.nodeid}")
    yield


def run_plan(torch, A, x, W=0, S=0, B=0, debug=False, dtype=None, bind_rows=False):
    from paper_1504_06474_amd import sss
    dtype = dtype or torch.float64
    xdt = torch.float64 if dtype == torch.float64 else torch.float32
    rp, col, v, xx = to_dev(A, x, val_dtype=dtype, x_dtype=xdt)
    plan = sss.Plan(A.m, A.n, A.nnz, dtype=dtype, W=W, S=S, B=B, debug=debug, bind_rows=bind_rows,
                    row_ptr=rp if bind_rows else None)
    y = plan.execute(rp, col, v, xx)
    torch.cuda.synchronize()
    return y.double().cpu().numpy(), plan


def test_config1_f64_default(torch_cuda):
    A, x = csrgen.config1()
    note(f"  poisson4096 nnz={A.nnz}")
    y, _ = run_plan(torch_cuda, A, x)
    ref = oracle.spmv(A.row_ptr, A.col, A.val, x)
    assert_f64_parity(y, ref, oracle.abs_spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("W", [4, 8, 16])
@pytest.mark.parametrize("S", [1, 2, 5, 8])
@pytest.mark.parametrize("B", [1, 4])
def test_config1_integer_exact_all_params(torch_cuda, W, S, B):
    A, x = csrgen.config1(int_valued=True)
    y, _ = run_plan(torch_cuda, A, x, W=W, S=S, B=B)
    assert_exact(y, oracle.spmv(A.row_ptr, A.col, A.val, x))


EDGE = {
    "single_entry": ([1], 1),
    "identity_1000": ([1] * 1000, 1000),
    "all_empty": ([0] * 300, 50),
    "leading_trailing_empty": ([0] * 700 + [3, 5, 1] * 200 + [0] * 900, 400),
    "long_row_many_bunches": ([2] * 50 + [150_000] + [1] * 3000 + [0] * 10 + [40_000], 200_000),
    "empty_run_100k_inside_tile": ([5] * 10 + [0] * 100_000 + [7] * 10, 100),
    "rows_of_one_tile": ([512] * 30 + [0] + [512] * 30, 1024),
    "rows_of_two_tiles_with_empties": ([1024, 0, 0, 1024, 0, 1024] * 10, 2048),
    "alternating_empty": ([1, 0] * 20_000, 64),
    "dense_rows": ([4096] * 64, 4096),
}


@pytest.mark.parametrize("name", sorted(EDGE))
@pytest.mark.parametrize("WS", [(4, 1), (8, 5), (16, 2)])
def test_edge_matrices_integer_exact(torch_cuda, name, WS):
    lengths, n = EDGE[name]
    A, x = csr_from_lengths(lengths, n, seed=len(lengths))
    note(f"  {name} m={A.m} nnz={A.nnz} W,S={WS}")
    y, _ = run_plan(torch_cuda, A, x, W=WS[0], S=WS[1])
    assert_exact(y, oracle.spmv(A.row_ptr, A.col, A.val, x))


def test_m_zero_and_nnz_zero(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    p = sss.Plan(0, 5, 0)
    y = torch.empty(0, dtype=torch.float64, device="cuda")
    p.execute(torch.zeros(1, dtype=torch.int32, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
              torch.zeros(0, dtype=torch.float64, device="cuda"), torch.ones(5, dtype=torch.float64, device="cuda"), y)
    p2 = sss.Plan(7, 5, 0)
    y2 = torch.full((7,), 3.0, dtype=torch.float64, device="cuda")
    p2.execute(torch.zeros(8, dtype=torch.int32, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
               torch.zeros(0, dtype=torch.float64, device="cuda"), torch.ones(5, dtype=torch.float64, device="cuda"),
               y2)
    torch.cuda.synchronize()
    assert y2.cpu().numpy().tolist() == [0.0] * 7


def _check_dump(d, A, W, S, x):
    T = 64
    rp = A.row_ptr.astype(np.int64)
    n_tiles = math.ceil(A.nnz / (W * T))
    assert d["n_tiles"] == n_tiles
    assert d["n_bunches"] == math.ceil(A.nnz / (S * W * T))
    starts = sp.tile_starts_vec(rp, T, W)
    assert np.array_equal(d["tile_start"], starts[:-1])
    dirty = sp.dirty_tiles_vec(rp, T, W)
    assert np.array_equal(d["tile_dirty"].astype(bool), dirty)
    flags = sp.head_flags_vec(rp, T, W).reshape(n_tiles, W * T // 32, 32)
    words = (flags.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=2).astype(np.uint32)
    assert np.array_equal(d["heads"], words)
    assert d["dirty_count"] == int(dirty.sum())
    spec = {tuple(r[:3]) for r in d["speculator"]}
    want = {(int(starts[t]), int(starts[t + 1]), t) for t in np.nonzero(dirty)[0]}
    assert spec == want
    assert np.array_equal(d["sync_idx"], starts[:-1][::S])
    tails = d["tail_val"]
    for tb, v in _expected_tails(A, x, W, S).items():
        assert tails[tb] == v, (tb, tails[tb], v)


def _expected_tails(A, x, W, S):
    """Bunch tb's tail, where it has one: the products of the row holding
    the bunch's last nonzero, from that row's head to the bunch's end, when
    the row continues into the next bunch and is not the bunch's first row
    (exact on integer-valued inputs)."""
    SWT = S * W * 64
    rp = A.row_ptr.astype(np.int64)
    out = {}
    for tb in range(math.ceil(A.nnz / SWT) - 1):
        b0, e = tb * SWT, (tb + 1) * SWT
        r0 = int(np.searchsorted(rp, b0, side="right")) - 1
        r = int(np.searchsorted(rp, e - 1, side="right")) - 1  # the row holding nonzero e - 1
        if rp[r + 1] > e and r != r0:
            k = np.arange(rp[r], e)
            out[tb] = float(np.sum(A.val[k] * x[A.col[k]]))
    return out


def test_debug_dump_matches_oracle_definitions(torch_cuda):
    A, x = csrgen.config1(int_valued=True)
    for W, S in ((8, 5), (4, 1), (16, 2)):
        note(f"  dump W={W} S={S}")
        y, plan = run_plan(torch_cuda, A, x, W=W, S=S, debug=True)
        assert_exact(y, oracle.spmv(A.row_ptr, A.col, A.val, x))
        _check_dump(plan.debug_dump(), A, W, S, x)


def test_debug_dump_synchronizer_matches_loop_model(torch_cuda):
    """Synchronizer values against the step-by-step model at T = 64."""
    A, x = csr_from_lengths([3, 0, 700, 1, 1, 0, 0, 2000, 5] * 8 + [9] * 300, 3000, seed=4)
    W, S = 4, 2
    y, plan = run_plan(torch_cuda, A, x, W=W, S=S, debug=True)
    d = plan.debug_dump()
    r1 = sp.stage_one(A.row_ptr, A.col, A.val, x, 64, W, S)
    assert [s[0] for s in r1.synchronizer] == list(d["sync_idx"])
    assert [s[1] for s in r1.synchronizer] == list(d["sync_val"])
    assert d["dirty_count"] == r1.dirty_counter
    assert {tuple(r[:3]) for r in d["speculator"]} == set(r1.speculator)
    assert_exact(y, sp.stage_two(r1, A.row_ptr))


def test_repeat_and_determinism(torch_cuda):
    """The dirty counter is reset between calls; results are bitwise stable."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1()
    rp, col, v, xx = to_dev(A, x)
    plan = sss.Plan(A.m, A.n, A.nnz, debug=True)
    ys = []
    for _ in range(5):
        ys.append(plan.execute(rp, col, v, xx).cpu().numpy())
        d = plan.debug_dump()
        assert d["dirty_count"] == int(sp.dirty_tiles_vec(A.row_ptr, 64, 8).sum())
    for y in ys[1:]:
        assert np.array_equal(y, ys[0])


def test_plans_on_two_streams(torch_cuda):
    """Two plans on two streams (default priority), launches interleaved, and
    the one-call form of one size on both streams (a cached plan per
    stream): no hidden state is shared, every result exact."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A1, x1 = csrgen.config1(int_valued=True)
    A2, x2 = csrgen.config1(int_valued=True, m=3000)
    d1, d2 = to_dev(A1, x1), to_dev(A2, x2)
    p1 = sss.Plan(A1.m, A1.n, A1.nnz, bind_rows=True, row_ptr=d1[0])
    p2 = sss.Plan(A2.m, A2.n, A2.nnz, W=4, S=3)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    y1 = torch.empty(A1.m, dtype=torch.float64, device="cuda")
    y2 = torch.empty(A2.m, dtype=torch.float64, device="cuda")
    ya = torch.empty(A1.m, dtype=torch.float64, device="cuda")
    yb = torch.empty(A1.m, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for _ in range(20):
        p1.execute(*d1, y1, stream=s1)
        p2.execute(*d2, y2, stream=s2)
        sss.csr_spmv(*d1, y=ya, stream=s1)
        sss.csr_spmv(*d1, y=yb, stream=s2)
    torch.cuda.synchronize()
    ref1 = oracle.spmv(A1.row_ptr, A1.col, A1.val, x1)
    assert_exact(y1.cpu().numpy(), ref1)
    assert_exact(y2.cpu().numpy(), oracle.spmv(A2.row_ptr, A2.col, A2.val, x2))
    assert_exact(ya.cpu().numpy(), ref1)
    assert_exact(yb.cpu().numpy(), ref1)
    p1.close()
    p2.close()


def test_one_call_form_and_validate(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1(int_valued=True)
    rp, col, v, xx = to_dev(A, x)
    y = sss.csr_spmv(rp, col, v, xx)
    y2 = sss.csr_spmv(rp, col, v, xx)  # cached plan
    assert_exact(y.cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x))
    assert torch.equal(y, y2)
    # a second size, then the cache freed and both sizes planned again
    A2, x2 = csrgen.config1(int_valued=True, m=700)
    d2 = to_dev(A2, x2)
    y3 = sss.csr_spmv(*d2)
    sss.csr_spmv_cache_clear()
    sss.csr_spmv_cache_clear()  # an empty cache is fine
    assert torch.equal(sss.csr_spmv(rp, col, v, xx), y)
    assert torch.equal(sss.csr_spmv(*d2), y3)
    assert_exact(y3.cpu().numpy(), oracle.spmv(A2.row_ptr, A2.col, A2.val, x2))
    assert sss.validate_csr(rp, col, A.n)
    bad_col = col.clone()
    bad_col[5] = A.n
    assert not sss.validate_csr(rp, bad_col, A.n)
    bad_rp = rp.clone()
    bad_rp[10] = bad_rp[11] + 1
    assert not sss.validate_csr(bad_rp, col, A.n)


def test_misaligned_pointers_rejected(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1()
    rp, col, v, xx = to_dev(A, x)
    colx = torch.empty(A.nnz + 1, dtype=torch.int32, device="cuda")
    colx[1:] = col
    plan = sss.Plan(A.m, A.n, A.nnz)
    with pytest.raises(sss.SSSError):
        plan.execute(rp, colx[1:], v, xx)


def test_binding_checks_arrays_before_any_launch(torch_cuda):
    """The C entry points take bare pointers; the binding refuses host
    tensors, strided views, and arrays shorter or of another type than the
    plan was made for, in execute and in each stage, before calling them."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1()
    rp, col, v, xx = to_dev(A, x)
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    plan = sss.Plan(A.m, A.n, A.nnz)
    bad_calls = [
        lambda: plan.execute(rp, col[:-1], v, xx, y),
        lambda: plan.execute(rp, col, v, xx, y.cpu()),
        lambda: plan.execute(rp, col, v, xx[:-1], y),
        lambda: plan.stage1(rp, col, v[:-1], xx, y),
        lambda: plan.stage1(rp, col, v.float(), xx, y),
        lambda: plan.stage1(rp, col, v, xx, y[:-1]),
        lambda: plan.stage2(rp[:-1], y),
        lambda: plan.stage2(rp, y[:-1]),
        lambda: plan.stage2(rp, torch.empty(2 * A.m, dtype=torch.float64, device="cuda")[::2]),
    ]
    for call in bad_calls:
        with pytest.raises((ValueError, TypeError)):
            call()
    plan.execute(rp, col, v, xx, y)
    torch.cuda.synchronize()
    assert_f64_parity(y.cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x),
                      oracle.abs_spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("WS,bind", [((8, 5), True), ((8, 5), False), ((4, 8), False), ((16, 2), True)])
def test_config2_full_size_f64(torch_cuda, WS, bind):
    """The 1M-row power-law matrix: every row against the oracle; W=8, S=5
    with bound rows is the benchmark's launch configuration."""
    A, x = _config2_cached()
    note(f"  powerlaw1e6 nnz={A.nnz} W,S={WS} bind={bind}")
    y, _ = run_plan(torch_cuda, A, x, W=WS[0], S=WS[1], bind_rows=bind)
    ref, scale = _config2_ref()
    assert_f64_parity(y, ref, scale)


_C2 = {}


def _config2_cached():
    if "A" not in _C2:
        _C2["A"], _C2["x"] = csrgen.config2()
    return _C2["A"], _C2["x"]


def _config2_ref():
    A, x = _config2_cached()
    if "ref" not in _C2:
        _C2["ref"] = oracle.spmv(A.row_ptr, A.col, A.val, x)
        _C2["scale"] = oracle.abs_spmv(A.row_ptr, A.col, A.val, x)
    return _C2["ref"], _C2["scale"]


@pytest.mark.parametrize("k", [15, 16, 17, 63, 64, 65, 130])
@pytest.mark.parametrize("delta", [-1, 0, 1])
def test_synchronizer_runs(torch_cuda, k, delta):
    """Rows spanning k thread-bunches: short and long carry runs, a long row
    first and last, and two long rows back to back."""
    W, S = 4, 1
    swt = S * W * 64
    L = k * swt + delta
    lengths = [L, 3, 0, L + 7, L, 5, 0, 0, 2, L]
    A, x = csr_from_lengths(lengths, L + 8, seed=k * 3 + delta)
    y, _ = run_plan(torch_cuda, A, x, W=W, S=S)
    assert_exact(y, oracle.spmv(A.row_ptr, A.col, A.val, x))
    y2, _ = run_plan(torch_cuda, A, x, W=8, S=2)
    assert_exact(y2, oracle.spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("WS", [(8, 5), (4, 1), (16, 3)])
def test_floor_probe_reads_every_nonzero_once(torch_cuda, WS):
    """The measurement kernel streams exactly the matrix: on integer-valued
    data the sum of its per-lane outputs is sum_k val[k] * x[col[k]] (gather)
    and sum_k (val[k] + col[k]) (stream only), exactly."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1(int_valued=True)
    plan = sss.Plan(A.m, A.n, A.nnz, W=WS[0], S=WS[1])
    rp, col, v, xx = to_dev(A, x)
    out = torch.full((plan.info()["n_bunches"] * 64,), float("nan"), dtype=torch.float64, device="cuda")
    plan.floor_probe(col, v, xx, out, gather=True)
    torch.cuda.synchronize()
    assert float(out.sum()) == float(np.sum(A.val * x[A.col]))
    plan.floor_probe(col, v, None, out, gather=False)
    torch.cuda.synchronize()
    assert float(out.sum()) == float(np.sum(A.val + A.col))


@pytest.mark.parametrize("mode_u_w", [(0, 4, 4), (0, 16, 8), (4, 16, 2), (2, 8, 1)])
def test_gather_probe_reads_every_nonzero_and_row_once(torch_cuda, mode_u_w):
    """The design-independent probe reads the matrix exactly once: on
    integer-valued data its per-thread sums add up to sum_k val[k] x[col[k]];
    with the row part they add row_ptr[m] too, and y holds row_ptr[0..m-1]."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    mode, U, wps = mode_u_w
    # config 1, and 5M short or empty rows: more rows than one batch of 8 per
    # thread covers, so several row batches are spread over the gather loop
    for A, x in (csrgen.config1(int_valued=True),
                 csr_from_lengths(np.random.default_rng(4).integers(0, 3, size=5_000_000), 50_000, seed=4)):
        _check_gather_probe(torch, sss, A, x, mode, U, wps)


def _check_gather_probe(torch, sss, A, x, mode, U, wps):
    rp, col, v, xx = to_dev(A, x)
    out = torch.full((1 << 20,), float("nan"), dtype=torch.float64, device="cuda")
    th, _ = sss.gather_probe(col, xx, out, v, mode, U, wps)
    torch.cuda.synchronize()
    assert float(out[:th].sum()) == float(np.sum(A.val * x[A.col]))
    for after in (0, 8):  # rows spread over the gathers, or after them
        y = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
        th, _ = sss.gather_probe(col, xx, out, v, mode | after, U, wps, row_ptr=rp, y=y)
        torch.cuda.synchronize()
        assert float(out[:th].sum()) == float(np.sum(A.val * x[A.col])) + float(A.row_ptr[-1])
        assert np.array_equal(y.cpu().numpy(), A.row_ptr[:-1].astype(np.float64))


@pytest.mark.parametrize("name", sorted(EDGE) + ["config1"])
@pytest.mark.parametrize("WS", [(4, 1), (8, 5), (16, 2)])
def test_bound_rows_plan(torch_cuda, name, WS):
    """A plan that found every thread-bunch's first row at plan time: the
    same tile start rows, descriptors, dirty tiles and synchronizer as the
    searching plan (debug dump), bitwise the same y, exact on integers."""
    if name == "config1":
        A, x = csrgen.config1(int_valued=True)
    else:
        lengths, n = EDGE[name]
        A, x = csr_from_lengths(lengths, n, seed=len(lengths))
    note(f"  {name} m={A.m} nnz={A.nnz} W,S={WS}")
    y_b, p_b = run_plan(torch_cuda, A, x, W=WS[0], S=WS[1], debug=True, bind_rows=True)
    y_s, p_s = run_plan(torch_cuda, A, x, W=WS[0], S=WS[1], debug=True)
    assert_exact(y_b, oracle.spmv(A.row_ptr, A.col, A.val, x))
    assert np.array_equal(y_b.view(np.int64), y_s.view(np.int64))
    d_b, d_s = p_b.debug_dump(), p_s.debug_dump()
    for key in ("tile_start", "tile_dirty", "heads", "sync_idx"):
        assert np.array_equal(d_b[key], d_s[key]), key
    assert d_b["dirty_count"] == d_s["dirty_count"]


def test_bound_rows_needs_row_ptr(torch_cuda):
    from paper_1504_06474_amd import sss
    with pytest.raises(sss.SSSError):
        sss.Plan(10, 10, 10, bind_rows=True)


def test_bound_plan_rejects_another_row_ptr(torch_cuda):
    """A plan bound to one row_ptr array returns PLAN_MISMATCH for another
    (execute, stage 1 and stage 2 alike); an unbound plan takes any."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1(int_valued=True)
    rp, col, v, xx = to_dev(A, x)
    other = rp.clone()
    plan = sss.Plan(A.m, A.n, A.nnz, bind_rows=True, row_ptr=rp)
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    for call in (lambda: plan.execute(other, col, v, xx, y), lambda: plan.stage1(other, col, v, xx, y),
                 lambda: plan.stage2(other, y)):
        with pytest.raises(sss.SSSError) as e:
            call()
        assert e.value.status == -3
    plan.execute(rp, col, v, xx, y)
    free = sss.Plan(A.m, A.n, A.nnz)
    y2 = free.execute(other, col, v, xx)
    torch.cuda.synchronize()
    want = oracle.spmv(A.row_ptr, A.col, A.val, x)
    assert_exact(y.cpu().numpy(), want)
    assert_exact(y2.cpu().numpy(), want)


@pytest.mark.parametrize("WS", [(4, 1), (8, 5), (16, 2)])
def test_bound_plan_row_ptr_rewritten_in_place(torch_cuda, WS):
    """The same row_ptr array rewritten in place with another structure of
    the same m and nnz: stage 1 finds its stored first rows no longer hold
    and searches, so y is still exact (and matches a fresh plan's)."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1(int_valued=True)
    lens = np.diff(A.row_ptr.astype(np.int64))
    lens2 = csrgen.rng_for(11).permutation(lens)
    rp2 = np.zeros(A.m + 1, dtype=np.int64)
    np.cumsum(lens2, out=rp2[1:])
    A2 = csrgen.CSR(A.m, A.n, rp2.astype(np.int32), A.col, A.val, "config1_rows_permuted")
    rp, col, v, xx = to_dev(A, x)
    plan = sss.Plan(A.m, A.n, A.nnz, W=WS[0], S=WS[1], bind_rows=True, row_ptr=rp)
    y1 = plan.execute(rp, col, v, xx).cpu().numpy()
    rp.copy_(torch.from_numpy(A2.row_ptr).to("cuda"))
    y2 = plan.execute(rp, col, v, xx).cpu().numpy()
    assert_exact(y1, oracle.spmv(A.row_ptr, A.col, A.val, x))
    assert_exact(y2, oracle.spmv(A2.row_ptr, A2.col, A2.val, x))


def _dirty_bunches(row_ptr, W, S):
    """Thread-bunches holding a dirty tile, by the oracle's definition of a
    dirty tile (Section 3.2: an empty row inside the tile's row range)."""
    return np.unique(np.nonzero(sp.dirty_tiles_vec(row_ptr, 64, W))[0] // S).astype(np.int32)


@pytest.mark.parametrize("name", sorted(EDGE) + ["config1", "no_empty_rows"])
@pytest.mark.parametrize("WS", [(4, 1), (8, 5), (16, 2)])
def test_bound_plan_dirty_list(torch_cuda, name, WS):
    """A bound plan lists at plan time exactly the thread-bunches that the
    oracle's dirty-tile definition marks, stage 1's dirty flags fall in the
    same bunches, and y is exact (stage 2 re-arranges only listed bunches)."""
    if name == "config1":
        A, x = csrgen.config1(int_valued=True)
    elif name == "no_empty_rows":
        A, x = csr_from_lengths([27] * 5000, 5000, seed=27)
    else:
        lengths, n = EDGE[name]
        A, x = csr_from_lengths(lengths, n, seed=len(lengths))
    note(f"  {name} m={A.m} nnz={A.nnz} W,S={WS}")
    y, p = run_plan(torch_cuda, A, x, W=WS[0], S=WS[1], debug=True, bind_rows=True)
    listed = p.dirty_list()
    assert np.array_equal(listed, _dirty_bunches(A.row_ptr, *WS))
    d = p.debug_dump()
    assert np.array_equal(np.unique(np.nonzero(d["tile_dirty"])[0] // WS[1]), listed)
    assert_exact(y, oracle.spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("WS", [(4, 1), (8, 5), (16, 2)])
def test_bound_plan_without_dirty_bunches_rewritten_with_empty_rows(torch_cuda, WS):
    """A bound plan made for a matrix with no empty row lists no bunch.  Its
    row_ptr rewritten in place with empty rows (same m and nnz) makes tiles
    dirty outside the list: stage 1 marks the plan stale and stage 2 then
    re-arranges those bunches itself, so y stays exact call after call, and
    again once the first structure is written back."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    lens = np.full(4000, 9, dtype=np.int64)
    A, x = csr_from_lengths(lens, 600, seed=5)
    pick = csrgen.rng_for(6).choice(4000, size=400, replace=False)
    lens2 = lens.copy()
    lens2[pick[:200]] = 0
    lens2[pick[200:]] += 9
    rp2 = np.zeros(A.m + 1, dtype=np.int64)
    np.cumsum(lens2, out=rp2[1:])
    A2 = csrgen.CSR(A.m, A.n, rp2.astype(np.int32), A.col, A.val, "rows_emptied")
    rp, col, v, xx = to_dev(A, x)
    plan = sss.Plan(A.m, A.n, A.nnz, W=WS[0], S=WS[1], bind_rows=True, row_ptr=rp)
    assert plan.dirty_list().size == 0
    want1 = oracle.spmv(A.row_ptr, A.col, A.val, x)
    want2 = oracle.spmv(A2.row_ptr, A2.col, A2.val, x)
    assert_exact(plan.execute(rp, col, v, xx).cpu().numpy(), want1)
    rp.copy_(torch.from_numpy(A2.row_ptr).to("cuda"))
    for _ in range(2):
        assert_exact(plan.execute(rp, col, v, xx).cpu().numpy(), want2)
    rp.copy_(torch.from_numpy(A.row_ptr).to("cuda"))
    assert_exact(plan.execute(rp, col, v, xx).cpu().numpy(), want1)


def test_plan_workspace(torch_cuda):
    """A plan in a caller's workspace (as the binding makes them, from
    PyTorch's allocator) and a plan with its own allocation give bitwise the
    same y; a workspace that is too small or misaligned is rejected."""
    import ctypes
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1()
    rp, col, v, xx = to_dev(A, x)
    L = sss.lib()
    need = sss.workspace_size(A.m, A.n, A.nnz, W=8, S=5)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    for ptr, size in ((ws.data_ptr(), need - 1), (ws.data_ptr() + 16, need)):
        o = sss.PlanOpts(sss.MODE_FIXED, 8, 5, 0, 0, 0, 0, ptr, size)
        assert L.sss_csr_spmv_plan_create(A.m, A.n, A.nnz, None, 0, ctypes.byref(o), None, ctypes.byref(h)) == -1
        assert h.value is None
    o = sss.PlanOpts(sss.MODE_FIXED, 8, 5, 0, 0, 0, 0, None, 0)
    assert L.sss_csr_spmv_plan_create(A.m, A.n, A.nnz, None, 0, ctypes.byref(o), None, ctypes.byref(h)) == 0
    y_own = torch.empty(A.m, dtype=torch.float64, device="cuda")
    assert L.sss_csr_spmv_execute(h, rp.data_ptr(), col.data_ptr(), v.data_ptr(), xx.data_ptr(), y_own.data_ptr(),
                                  None) == 0
    torch.cuda.synchronize()
    assert L.sss_plan_destroy(h) == 0
    y_ws = sss.Plan(A.m, A.n, A.nnz, W=8, S=5).execute(rp, col, v, xx)
    torch.cuda.synchronize()
    assert np.array_equal(y_own.cpu().numpy().view(np.int64), y_ws.cpu().numpy().view(np.int64))
    assert_f64_parity(y_ws.cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x),
                      oracle.abs_spmv(A.row_ptr, A.col, A.val, x))


@pytest.mark.parametrize("bind", [False, True])
def test_execute_captured_in_a_graph(torch_cuda, bind):
    """execute allocates nothing and syncs nothing, so it can be captured:
    replay the graph several times with new x (and y clobbered) written by
    the program's own eager work in between; every replay is exact."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config1(int_valued=True)
    rp, col, v, xx = to_dev(A, x)
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    plan = sss.Plan(A.m, A.n, A.nnz, W=8, S=3, bind_rows=bind, row_ptr=rp if bind else None)
    plan.execute(rp, col, v, xx, y)  # first call outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(rp, col, v, xx, y)
    rng = np.random.default_rng(5)
    for rep in range(4):
        xh = rng.integers(-3, 4, A.n).astype(np.float64)
        xx.copy_(torch.from_numpy(xh))
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_exact(y.cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, xh))
        plan.execute(rp, col, v, xx, y)  # eager work between replays
        torch.cuda.synchronize()
    del g


@pytest.mark.parametrize("name", ["config1", "leading_trailing_empty", "long_row_many_bunches",
                                  "empty_run_100k_inside_tile", "rows_of_two_tiles_with_empties"])
@pytest.mark.parametrize("WS", [(4, 1), (8, 5), (16, 2)])
def test_stage2_on_host(torch_cuda, name, WS):
    """The paper's split (stage 1 on the GPU, stage 2 on a host core) gives
    the same exact result on integer-valued inputs."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    if name == "config1":
        A, x = csrgen.config1(int_valued=True)
    else:
        lengths, n = EDGE[name]
        A, x = csr_from_lengths(lengths, n, seed=len(lengths))
    rp, col, v, xx = to_dev(A, x)
    y = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
    plan = sss.Plan(A.m, A.n, A.nnz, W=WS[0], S=WS[1])
    plan.stage1(rp, col, v, xx, y)
    torch.cuda.synchronize()
    yh = y.cpu().numpy().copy()
    plan.stage2_host(A.row_ptr, yh)
    assert_exact(yh, oracle.spmv(A.row_ptr, A.col, A.val, x))


def test_stage2_on_host_benchmark_matrix(torch_cuda):
    """The paper's split at full size, as the benchmark times it: the 1M-row
    power-law matrix with the rows bound at plan time (stage 1 on the device,
    stage 2 on a host core); every row within 1e-12 (|A||x|)_i of the oracle.
    The host adds a row's carries in bunch order and the device adds runs of
    more than 16 bunches by a tree, so the two agree bit for bit except on
    the rows that such runs end in."""
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    A, x = csrgen.config2()
    rp, col, v, xx = to_dev(A, x)
    plan = sss.Plan(A.m, A.n, A.nnz, bind_rows=True, row_ptr=rp)
    y_dev = plan.execute(rp, col, v, xx)
    y = torch.full((A.m,), float("nan"), dtype=torch.float64, device="cuda")
    plan.stage1(rp, col, v, xx, y)
    torch.cuda.synchronize()
    yh = y.cpu().numpy().copy()
    plan.stage2_host(A.row_ptr, yh)
    assert_f64_parity(yh, oracle.spmv(A.row_ptr, A.col, A.val, x), oracle.abs_spmv(A.row_ptr, A.col, A.val, x))
    # rows shorter than 16 bunches' worth of nonzeros get no tree-summed run
    short = np.diff(A.row_ptr) < 16 * plan.info()["W"] * 64 * plan.info()["S"]
    assert np.array_equal(yh[short], y_dev.cpu().numpy()[short])
