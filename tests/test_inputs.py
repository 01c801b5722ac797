"""The seeded input generators: determinism, the workload statistics they
promise, and the storage rounding used by the reduced-precision paths."""
import numpy as np

import csrgen


def test_bf16_round_to_nearest_even():
    # 1 + 2^-8 lies halfway between bf16 1 and 1 + 2^-7: ties go to the even one (1)
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0, 1e-3], dtype=np.float32)
    b = csrgen.round_to_bf16(vals)
    assert b[0] == 1.0
    assert b[1] == 1.0
    assert b[2] == np.float32(1 + 2 ** -6)  # halfway 1+2^-7 / 1+2^-6 -> even mantissa 1+2^-6
    assert b[3] == np.float32(1 + 2 ** -7)
    assert b[4] == -2.5 and b[5] == 3.0
    assert abs(b[6] - 1e-3) <= 2 ** -9 * 1e-3


def test_small_integers_exact_in_all_storage_types():
    A, x = csrgen.config1(int_valued=True)
    for kind in ("f32", "bf16"):
        vs, xs, ve, xe = csrgen.quantize(A, x, kind)
        assert np.array_equal(ve, A.val) and np.array_equal(xe, x)


def test_generators_are_deterministic():
    a1, x1 = csrgen.config1()
    a2, x2 = csrgen.config1()
    assert np.array_equal(a1.col, a2.col) and np.array_equal(a1.val, a2.val) and np.array_equal(x1, x2)


def test_config1_shape_and_columns():
    A, _ = csrgen.config1()
    st = A.stats()
    assert st["m"] == 4096 and abs(st["empty_frac"] - 0.05) < 1e-3
    assert 9.0 < st["mean"] < 10.0
    rp = A.row_ptr.astype(np.int64)
    for i in range(0, A.m, 37):
        c = A.col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and (c.size == 0 or (c.min() >= 0 and c.max() < A.n))


def test_zipf_mandelbrot_offset_hits_mean():
    q = csrgen.zipf_mandelbrot_q(200_000, 2.0, 20.0 / 0.97)
    k = np.arange(1, 200_001, dtype=np.float64)
    p = (k + q) ** -2.0
    p /= p.sum()
    assert abs((k * p).sum() - 20.0 / 0.97) < 1e-6


def test_selector_classes_small():
    for i in range(5):
        A = csrgen.selector_matrix(i, m_lo=2e3, m_hi=5e3)
        assert A.nnz > 0 and A.row_ptr[-1] == A.nnz
        assert A.col.max() < A.n


def test_laplacian2d_structure():
    """5-point Laplacian: symmetric, 4 on the diagonal, interior rows sum to
    zero, boundary rows to the number of missing neighbours."""
    N = 6
    A = csrgen.laplacian2d_csr(N)
    dense = np.zeros((A.m, A.n))
    for i in range(A.m):
        dense[i, A.col[A.row_ptr[i]:A.row_ptr[i + 1]]] = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
    assert np.array_equal(dense, dense.T)
    assert np.all(np.diag(dense) == 4.0)
    i, j = np.divmod(np.arange(N * N), N)
    missing = (i == 0).astype(int) + (i == N - 1) + (j == 0) + (j == N - 1)
    assert np.array_equal(dense.sum(axis=1), missing.astype(float))
