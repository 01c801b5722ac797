"""The selector's native pieces against the oracle: the feature kernel
(integer statistics exact, variance within FP64 rounding) and the FP32
network kernels (forward, gradients, Adam) against the FP64 oracle network."""
import numpy as np
import pytest

import csrgen
from oracle import mlp
from helpers import note, csr_from_lengths

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


def expected_features(A, bytes_per_value):
    L = np.diff(A.row_ptr.astype(np.int64))
    mean = L.mean()
    var = (L.astype(np.float64) ** 2).mean() - mean * mean
    return np.array([np.log2(A.m + 1), np.log2(A.n + 1), np.log2(A.nnz + 1), np.log2(1 + mean),
                     np.log2(1 + max(var, 0)), np.log2(1 + L.max()), (L == 0).mean(), bytes_per_value])


@pytest.mark.parametrize("which", ["config1", "config2", "dense_rows", "empty_rows"])
def test_features(torch_cuda, which):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    if which == "config1":
        A, _ = csrgen.config1()
    elif which == "config2":
        A, _ = csrgen.config2()
    elif which == "dense_rows":
        A = csrgen.dense_rows_csr(20_000, 5)
    else:
        A, _ = csr_from_lengths([0] * 1000 + [3] * 10 + [0] * 5, 20, seed=1)
    rp = torch.from_numpy(A.row_ptr).cuda()
    for dt, bpv in ((torch.float64, 8), (torch.float32, 4), (torch.bfloat16, 2)):
        f = sss.features(rp, A.n, A.nnz, dt)
        want = expected_features(A, bpv)
        assert np.allclose(f, want.astype(np.float32), rtol=1e-6, atol=1e-6), (f, want)


def test_mlp_forward_backward_adam(torch_cuda):
    torch = torch_cuda
    from paper_1504_06474_amd import sss
    rng = np.random.default_rng(1)
    N = 257
    X = rng.normal(size=(N, 8))
    Q = rng.random(size=(N, 12))
    Q /= Q.sum(axis=1, keepdims=True)
    p = mlp.init_params(2) * 0.7
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    P, Xd, Qd = d(p), d(X), d(Q)
    H1 = torch.empty(N, 64, device="cuda")
    H2 = torch.empty(N, 64, device="cuda")
    Z = torch.empty(N, 12, device="cuda")
    sss.mlp_forward(P, Xd, H1, H2, Z)
    # the oracle on the same float32-rounded inputs
    p32 = p.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    Q32 = Q.astype(np.float32).astype(np.float64)
    h1, h2, z = mlp.forward(p32, X32)
    torch.cuda.synchronize()
    assert np.allclose(Z.cpu().numpy(), z, rtol=1e-4, atol=1e-4)
    assert np.allclose(H1.cpu().numpy(), h1, rtol=1e-4, atol=1e-5)
    grad = torch.empty(mlp.N_PARAMS, device="cuda")
    loss = torch.empty(N, device="cuda")
    work = torch.empty(N * 140, device="cuda")
    sss.mlp_backward(P, Xd, H1, H2, Z, Qd, grad, loss, work)
    g = mlp.backward(p32, X32, Q32)
    torch.cuda.synchronize()
    gg = grad.cpu().numpy()
    assert np.abs(gg - g).max() <= 1e-4 * np.abs(g).max() + 1e-7
    assert abs(float(loss.mean()) - mlp.loss(p32, X32, Q32)) < 1e-4
    # Adam: two steps against the oracle
    m1 = torch.zeros(mlp.N_PARAMS, device="cuda")
    m2 = torch.zeros(mlp.N_PARAMS, device="cuda")
    pr, mr, vr = p32.copy(), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    gr = gg.astype(np.float64)
    for step in (1, 2):
        sss.mlp_adam(P, grad, m1, m2, step, 1e-3)
        pr, mr, vr = mlp.adam_step(pr, gr, mr, vr, step, 1e-3)
    torch.cuda.synchronize()
    assert np.abs(P.cpu().numpy() - pr).max() < 1e-6


def test_class_table_and_selector_roundtrip(torch_cuda):
    from paper_1504_06474_amd import sss
    assert [sss.class_params(c) for c in range(12)] == [(w, s) for w in (4, 8, 16) for s in (1, 2, 4, 8)]
    # a network whose last bias favours class 9 and whose weights are zero
    p = np.zeros(mlp.N_PARAMS)
    p[-12 + 9] = 5.0
    sss.selector_set(p, np.zeros(8), np.ones(8))
    assert sss.selector_predict(np.ones(8)) == 9
