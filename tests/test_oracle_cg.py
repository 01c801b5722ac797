"""Pins of the CG oracle (oracle/cg.py) against what the mathematics fixes:
termination in at most n steps (one per distinct eigenvalue), the residual
recurrence r_k = b - A x_k, orthogonal residuals and A-conjugate directions,
a zero right-hand side, and planted mistakes that the termination pin
catches."""
import numpy as np
import pytest

import csrgen
from oracle import cg as ocg
from oracle import spmv


def dense_to_csr(A):
    rows, cols = np.nonzero(A)
    row_ptr = np.zeros(A.shape[0] + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), A[rows, cols].astype(np.float64)


def spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(n, n))
    return M @ M.T + n * np.eye(n)


def test_terminates_in_n_steps():
    n = 10
    A = spd(n, 1)
    b = np.random.default_rng(2).normal(size=n)
    rp, col, val = dense_to_csr(A)
    want = np.linalg.solve(A, b)
    got = ocg.cg_steps(rp, col, val, b, np.zeros(n), n)
    assert np.linalg.norm(got["x"] - want) <= 1e-10 * np.linalg.norm(want)
    assert np.sqrt(got["rr"]) <= 1e-9 * np.linalg.norm(b)
    assert got["bb"] == pytest.approx(float(b @ b), rel=1e-15)


def test_one_step_per_distinct_eigenvalue():
    rng = np.random.default_rng(3)
    b = rng.normal(size=12)
    # A = 3 I: one step, alpha = 1/3
    rp, col, val = dense_to_csr(3.0 * np.eye(12))
    one = ocg.cg_steps(rp, col, val, b, np.zeros(12), 1)
    assert np.allclose(one["x"], b / 3.0, rtol=1e-15, atol=0)
    # two distinct eigenvalues: exact after two steps, not after one
    d = np.where(np.arange(12) % 2 == 0, 2.0, 5.0)
    rp, col, val = dense_to_csr(np.diag(d))
    want = b / d
    after1 = ocg.cg_steps(rp, col, val, b, np.zeros(12), 1)["x"]
    after2 = ocg.cg_steps(rp, col, val, b, np.zeros(12), 2)["x"]
    assert np.linalg.norm(after1 - want) > 1e-2 * np.linalg.norm(want)
    assert np.linalg.norm(after2 - want) <= 1e-14 * np.linalg.norm(want)


def test_residual_recurrence_orthogonality_and_conjugacy():
    L = csrgen.laplacian2d_csr(8)
    rng = np.random.default_rng(4)
    b = rng.uniform(-1, 1, L.m)
    x0 = rng.uniform(-1, 1, L.m)
    states = [ocg.cg_steps(L.row_ptr, L.col, L.val, b, x0, k) for k in range(7)]
    for s in states:
        true_r = b - spmv(L.row_ptr, L.col, L.val, s["x"])
        assert np.linalg.norm(s["r"] - true_r) <= 1e-12 * np.linalg.norm(b)
        assert s["rr"] == pytest.approx(float(s["r"] @ s["r"]), rel=1e-15)
    for i in range(7):
        for j in range(i):
            ri, rj = states[i]["r"], states[j]["r"]
            assert abs(ri @ rj) <= 1e-9 * np.linalg.norm(ri) * np.linalg.norm(rj)
            pi, pj = states[i]["p"], states[j]["p"]
            Apj = spmv(L.row_ptr, L.col, L.val, pj)
            assert abs(pi @ Apj) <= 1e-9 * np.linalg.norm(pi) * np.linalg.norm(Apj)
    # rr_prev of k steps is rr of k - 1 steps
    for k in range(1, 7):
        assert states[k]["rr_prev"] == states[k - 1]["rr"]


def test_zero_right_hand_side():
    L = csrgen.laplacian2d_csr(5)
    got = ocg.cg_steps(L.row_ptr, L.col, L.val, np.zeros(L.m), np.zeros(L.m), 3)
    for key in ("x", "r", "p"):
        assert np.all(got[key] == 0.0)
    assert got["rr"] == 0.0 and got["bb"] == 0.0


def _mistaken_cg(A, b, steps, mistake):
    x = np.zeros_like(b)
    r = b - A @ x
    p = r.copy()
    rr = r @ r
    for _ in range(steps):
        q = A @ p
        alpha = rr / (p @ q) if mistake != "alpha_over_pp" else rr / (p @ p)
        x = x + alpha * p if mistake != "x_minus" else x - alpha * p
        r = r - alpha * q
        rr_new = r @ r
        beta = rr_new / rr if mistake != "beta_inverted" else rr / rr_new
        p = r + beta * p if mistake != "p_from_old_direction_only" else r + beta * (r - p)
        rr = rr_new
    return x


@pytest.mark.parametrize("mistake", ["alpha_over_pp", "x_minus", "beta_inverted", "p_from_old_direction_only"])
def test_planted_mistakes_miss_termination(mistake):
    n = 10
    A = spd(n, 1)
    b = np.random.default_rng(2).normal(size=n)
    want = np.linalg.solve(A, b)
    assert np.linalg.norm(_mistaken_cg(A, b, n, "none") - want) <= 1e-10 * np.linalg.norm(want)
    assert np.linalg.norm(_mistaken_cg(A, b, n, mistake) - want) > 1e-6 * np.linalg.norm(want)
