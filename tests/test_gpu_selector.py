"""The trained selector in use: SELECTOR-mode plans compute the same y (parity
against the oracle) with the class the network picks, and on held-out
matrices the picked parameters beat the method's default parameters
(W = 8, S = 5) and stay close to the autotuned grid's best."""
import numpy as np
import pytest

import csrgen
import oracle
from helpers import note, assert_f64_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sel():
    import torch
    assert torch.cuda.is_available()
    from paper_1504_06474_amd import sss
    assert sss.load_selector(), "the trained selector parameters are missing"
    return torch, sss


@pytest.fixture(autouse=True)
def _announce(request):
    note(f"[gpu-test] {request.node.nodeid}")
    yield


def test_selector_plan_parity(sel):
    torch, sss = sel
    for A, x in (csrgen.config1(), (csrgen.stencil3d_csr(40, 3), np.random.default_rng(1).uniform(-1, 1, 64000))):
        rp = torch.from_numpy(A.row_ptr).cuda()
        plan = sss.Plan(A.m, A.n, A.nnz, mode=sss.MODE_SELECTOR, row_ptr=rp)
        f = sss.features(rp, A.n, A.nnz)
        W, S = sss.class_params(sss.selector_predict(f))
        info = plan.info()
        assert (info["W"], info["S"]) == (W, S)
        y = plan.execute(rp, torch.from_numpy(A.col).cuda(), torch.from_numpy(A.val).cuda(),
                         torch.from_numpy(x).cuda())
        assert_f64_parity(y.cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x),
                          oracle.abs_spmv(A.row_ptr, A.col, A.val, x))


def _time(torch, plan, args, reps=7):
    from paper_1504_06474_amd.selector_train import time_plan
    return time_plan(plan, args, reps) * 1e-3


def _held_out_gain_and_regret(torch, sss, kind, indices):
    from csrgen.torch_gen import selector_matrix_gpu
    from paper_1504_06474_amd.selector_train import VALUE_TYPES
    vt, xt = VALUE_TYPES[kind]
    gains, regrets = [], []
    for i in indices:
        d = selector_matrix_gpu(i)
        args = (d["row_ptr"], d["col"], d["val"].to(vt), d["x"].to(xt), torch.empty(d["m"], dtype=xt, device="cuda"))
        # gain: selected vs default plan, both timed the same way
        p_sel = sss.Plan(d["m"], d["n"], d["nnz"], dtype=vt, mode=sss.MODE_SELECTOR, row_ptr=d["row_ptr"],
                         bind_rows=True)
        p_def = sss.Plan(d["m"], d["n"], d["nnz"], dtype=vt, bind_rows=True, row_ptr=d["row_ptr"])
        t_sel, t_def = _time(torch, p_sel, args), _time(torch, p_def, args)
        gains.append(t_def / t_sel)
        # regret: the picked class against the best class of one grid timing
        grid, _ = sss.autotune(*args, n=d["n"], reps=7)
        W, S = p_sel.info()["W"], p_sel.info()["S"]
        cls = [sss.class_params(c) for c in range(12)].index((W, S))
        regrets.append(grid[cls] / grid.min())
        note(f"  {i} {d['name']}: sel {t_sel * 1e3:.1f}us default {t_def * 1e3:.1f}us | grid picked "
             f"{grid[cls]:.1f}us best {grid.min():.1f}us")
    g = float(np.exp(np.mean(np.log(gains))))
    r = float(np.exp(np.mean(np.log(regrets)))) - 1
    note(f"  geomean gain over default {g:.3f}, regret vs grid {r:.4f}")
    return g, r


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16"])
def test_selector_gain_on_held_out(sel, kind):
    """Held-out selector matrices (indices 2000.., never trained on), stored
    as `kind`; the default plan is the library's default for that type."""
    torch, sss = sel
    g, r = _held_out_gain_and_regret(torch, sss, kind, range(2000, 2015))
    assert g > 1.1
    assert r <= 0.05  # the selector's target: within 5% of the autotuned grid


def test_selector_on_held_out_large_matrices(sel):
    """Held-out matrices of the selector set's large part (2e6..1.6e7 rows,
    indices 2360.., never trained on; one of each class), FP64: within 5% of
    the grid, and no slower than the default plan (whose S suits large
    matrices, so there is little to gain there)."""
    torch, sss = sel
    import csrgen
    from paper_1504_06474_amd.selector_train import LARGE_TRAIN
    first = csrgen.SELECTOR_LARGE_BASE + LARGE_TRAIN
    g, r = _held_out_gain_and_regret(torch, sss, "f64", range(first, first + 5))
    assert r <= 0.05
    assert g > 0.98


def test_grid_plan(sel):
    """GRID mode: the plan carries a class of the grid, computes y like any
    other plan, and an m = 0 / nnz = 0 matrix gets a plan without timing."""
    torch, sss = sel
    A, x = csrgen.config1()
    rp, col = torch.from_numpy(A.row_ptr).cuda(), torch.from_numpy(A.col).cuda()
    v, xx = torch.from_numpy(A.val).cuda(), torch.from_numpy(x).cuda()
    y = torch.empty(A.m, dtype=torch.float64, device="cuda")
    plan = sss.plan_grid(rp, col, v, xx, y, n=A.n, reps=3)
    info = plan.info()
    assert (info["W"], info["S"]) in [sss.class_params(c) for c in range(12)]
    y.fill_(float("nan"))
    plan.execute(rp, col, v, xx, y)
    torch.cuda.synchronize()
    assert_f64_parity(y.cpu().numpy(), oracle.spmv(A.row_ptr, A.col, A.val, x),
                      oracle.abs_spmv(A.row_ptr, A.col, A.val, x))
    plan.close()
    rp0 = torch.zeros(6, dtype=torch.int32, device="cuda")
    e = torch.empty(0, device="cuda")
    p0 = sss.plan_grid(rp0, e.int(), e.double(), torch.zeros(3, dtype=torch.float64, device="cuda"),
                       torch.empty(5, dtype=torch.float64, device="cuda"), n=3)
    assert p0.info()["n_tiles"] == 0
    p0.close()
