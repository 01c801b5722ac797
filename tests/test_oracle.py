"""Pins of the CPU oracle's plain SpMV (y = A x, Sections 1 and 2.1) against
facts fixed by the mathematics and the paper, independent of the oracle's code:
exact rational brute force, special matrices, the paper's 6x6 example, and the
accuracy the compensated dot product guarantees."""
import json
import os
from fractions import Fraction

import numpy as np

import oracle
import csrgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_exact(row_ptr, col, val, x, m):
    """Exact y = A x with rational arithmetic over a dense copy of A."""
    n = len(x)
    A = [[Fraction(0)] * n for _ in range(m)]
    for i in range(m):
        for k in range(row_ptr[i], row_ptr[i + 1]):
            A[i][col[k]] += Fraction(float(val[k]))
    return [sum((A[i][j] * Fraction(float(x[j])) for j in range(n)), Fraction(0)) for i in range(m)]


def random_tiny(rng, m, n, dyadic=True):
    lengths = rng.integers(0, n + 1, size=m)
    lengths[rng.random(m) < 0.3] = 0
    rp = np.zeros(m + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lengths)
    col = np.concatenate([np.sort(rng.choice(n, size=L, replace=False)) for L in lengths]).astype(np.int32) \
        if lengths.sum() else np.zeros(0, np.int32)
    if dyadic:
        val = rng.integers(-64, 65, size=int(rp[-1])) / 16.0
        x = rng.integers(-64, 65, size=n) / 8.0
    else:
        val = rng.uniform(-1, 1, size=int(rp[-1]))
        x = rng.uniform(-1, 1, size=n)
    return rp, col, val, x


def test_dense_brute_force_exact():
    rng = np.random.default_rng(11)
    for _ in range(200):
        m, n = int(rng.integers(0, 13)), int(rng.integers(1, 13))
        rp, col, val, x = random_tiny(rng, m, n)
        y = oracle.spmv(rp, col, val, x)
        ex = dense_exact(rp, col, val, x, m)
        assert [Fraction(float(v)) for v in y] == ex


def test_dense_brute_force_general_values_error_bound():
    # Dot2 bound (Ogita-Rump-Oishi, Prop. 5.5 form): |res - s| <= u|s| + gamma_n^2 sum|a b|
    rng = np.random.default_rng(12)
    u = 2.0 ** -53
    for _ in range(200):
        m, n = int(rng.integers(1, 13)), int(rng.integers(1, 13))
        rp, col, val, x = random_tiny(rng, m, n, dyadic=False)
        y = oracle.spmv(rp, col, val, x)
        ex = dense_exact(rp, col, val, x, m)
        ab = oracle.abs_spmv(rp, col, val, x)
        for i in range(m):
            k = rp[i + 1] - rp[i]
            g = k * u / (1 - k * u)
            err = abs(Fraction(float(y[i])) - ex[i])
            assert err <= Fraction(u) * abs(ex[i]) + Fraction(2 * g * g * float(ab[i]) + 1e-300)


def test_compensation_recovers_cancelled_term():
    # 1e16 + 1 - 1e16 = 1: a plain sum loses the 1, Dot2 keeps it
    rp = np.array([0, 3], dtype=np.int32)
    col = np.array([0, 1, 2], dtype=np.int32)
    val = np.array([1e16, 1.0, -1e16])
    x = np.ones(3)
    assert oracle.spmv(rp, col, val, x)[0] == 1.0
    assert oracle.spmv_naive(rp, col, val, x)[0] == 0.0


def test_identity_and_permutation():
    rng = np.random.default_rng(3)
    n = 1000
    x = rng.uniform(-1, 1, n)
    rp = np.arange(n + 1, dtype=np.int32)
    eye = np.arange(n, dtype=np.int32)
    assert np.array_equal(oracle.spmv(rp, eye, np.ones(n), x), x)
    perm = rng.permutation(n).astype(np.int32)
    assert np.array_equal(oracle.spmv(rp, perm, np.ones(n), x), x[perm])
    d = rng.uniform(-2, 2, n)
    assert np.array_equal(oracle.spmv(rp, eye, d, x), d * x)


def test_empty_matrix_and_empty_rows():
    assert oracle.spmv(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(5)).shape == (0,)
    rp = np.zeros(8, dtype=np.int32)
    y = oracle.spmv(rp, np.zeros(0, np.int32), np.zeros(0), np.ones(4))
    assert np.array_equal(y, np.zeros(7))


def test_row_sums_with_unit_x_integer_exact():
    A, _ = csrgen.config1(int_valued=True)
    y = oracle.spmv(A.row_ptr, A.col, A.val, np.ones(A.n))
    rp = A.row_ptr.astype(np.int64)
    for i in range(0, A.m, 7):
        assert y[i] == sum(int(v) for v in A.val[rp[i]:rp[i + 1]])


def test_single_dense_row_is_a_dot_product():
    rng = np.random.default_rng(5)
    n = 3000
    v = rng.integers(-1000, 1001, n) / 64.0
    x = rng.integers(-1000, 1001, n) / 32.0
    rp = np.array([0, n], dtype=np.int32)
    y = oracle.spmv(rp, np.arange(n, dtype=np.int32), v, x)
    assert Fraction(float(y[0])) == sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(v, x))


def test_paper_6x6_example():
    g = json.load(open(os.path.join(GOLDEN, "e8_csr_6x6.json")))
    letters = {L: float(i + 2) * (1 if i % 2 else -1) for i, L in enumerate(g["letters"])}
    val = np.array([letters[L] for L in g["letters"]])
    y = oracle.spmv(np.array(g["row_ptr"], np.int32), np.array(g["col"], np.int32), val,
                    np.array(g["x"], float))
    expect = [eval(f, {}, letters) for f in g["y_formula"]]
    assert list(y) == expect


def test_comparators_agree_on_integer_inputs():
    A, x = csrgen.config1(int_valued=True)
    y = oracle.spmv(A.row_ptr, A.col, A.val, x)
    assert np.array_equal(oracle.spmv_naive(A.row_ptr, A.col, A.val, x), y)
    assert np.array_equal(oracle.spmv_rowblock(A.row_ptr, A.col, A.val, x, 4), y)
    assert np.array_equal(oracle.spmv(A.row_ptr, A.col, A.val, x, 1), y)


def test_rows_subset_matches_full():
    A, x = csrgen.config1()
    y = oracle.spmv(A.row_ptr, A.col, A.val, x)
    rows = np.array([0, 5, 17, 4095, 100])
    assert np.array_equal(oracle.spmv_rows(A.row_ptr, A.col, A.val, x, rows), y[rows])


def test_abs_spmv_bounds_y():
    A, x = csrgen.config1()
    y = oracle.spmv(A.row_ptr, A.col, A.val, x)
    assert np.all(np.abs(y) <= oracle.abs_spmv(A.row_ptr, A.col, A.val, x) * (1 + 1e-15))


def test_abs_spmv_exact_closed_form():
    """(|A||x|)_i = sum_k |a_ik x_k| exactly (dyadic inputs: every product and
    partial sum is representable), including a row whose terms cancel: there
    |y_i| = 0 while (|A||x|)_i = 2, so taking |sum| instead of sum|.| fails."""
    rng = np.random.default_rng(41)
    for _ in range(40):
        m, n = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        rp, col, val, x = random_tiny(rng, m, n)
        want = [sum((abs(Fraction(float(val[k])) * Fraction(float(x[col[k]]))) for k in range(rp[i], rp[i + 1])),
                    Fraction(0)) for i in range(m)]
        got = oracle.abs_spmv(rp, col, val, x)
        assert [Fraction(float(v)) for v in got] == want
    rp = np.array([0, 2], np.int32)
    col = np.array([0, 1], np.int32)
    val = np.array([1.0, -1.0])
    x = np.array([1.0, 1.0])
    assert oracle.spmv(rp, col, val, x)[0] == 0.0
    assert oracle.abs_spmv(rp, col, val, x)[0] == 2.0
