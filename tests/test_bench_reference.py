"""bench.py on the CPU.  Its error figures use its own reference (`row_sums`:
products and row sums in long double), checked here against the oracle:
ragged rows, runs of empty rows at both ends, a long row, all-empty and
nnz = 0 matrices.  Also: it refuses more than one GPU, and its JSON line
holds no NaN or infinity."""
import numpy as np

import bench
import csrgen
import oracle


def _check(rp, col, val, x):
    y, sc = bench.row_sums(rp, col, val, x)
    yo = oracle.spmv(rp, col, val, x)
    so = oracle.abs_spmv(rp, col, val, x)
    s = np.where(so > 0, so, 1.0)
    assert np.all(np.abs(y - yo) <= 1e-15 * s)
    assert np.all(np.abs(sc - so) <= 1e-14 * s)
    assert np.all(y[so == 0] == 0)


def test_row_sums_matches_oracle_on_ragged_rows():
    rng = np.random.default_rng(7)
    lengths = np.concatenate([np.zeros(5, np.int64), rng.integers(0, 30, 400), [20_000], np.zeros(7, np.int64)])
    A = csrgen.lengths_to_csr(rng, lengths, 50_000, "uniform")
    x = rng.uniform(-1, 1, 50_000)
    _check(A.row_ptr, A.col, A.val, x)


def test_row_sums_benchmark_generator_small():
    A, x = csrgen.config1()
    _check(A.row_ptr, A.col, A.val, x)


def test_row_sums_degenerate():
    x = np.array([1.0, -2.0, 3.0])
    y, sc = bench.row_sums(np.zeros(4, np.int32), np.zeros(0, np.int32), np.zeros(0), x)
    assert y.shape == (3,) and not y.any() and not sc.any()
    y, sc = bench.row_sums(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), x)
    assert y.shape == (0,)
    rp = np.array([0, 0, 2, 2, 3], np.int32)
    y, sc = bench.row_sums(rp, np.array([0, 2, 1], np.int32), np.array([2.0, -1.0, 4.0]), x)
    assert list(y) == [0.0, -1.0, 0.0, -8.0] and list(sc) == [0.0, 5.0, 0.0, 8.0]


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so,
    before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_bench_json_has_no_non_finite_numbers():
    import json
    line = json.dumps(bench._finite({"a": float("nan"), "b": [1.5, float("-inf")], "c": {"d": float("inf")}}),
                      allow_nan=False)
    assert json.loads(line) == {"a": None, "b": [1.5, None], "c": {"d": None}}


def test_algorithmic_bytes_of_the_benchmark_matrix():
    """The roofline's bytes per product: each of the 19,189,716 entries once
    (8-byte value, 4-byte column), row_ptr's 1,000,001 int32 offsets, x and
    y once each (1,000,000 doubles each); the FP32 form halves values and
    vectors."""
    assert bench.alg_bytes(1_000_000, 1_000_000, 19_189_716, 8, 8) == 250_276_596
    assert bench.alg_bytes(1_000_000, 1_000_000, 19_189_716, 4, 4) == 19_189_716 * 8 + 4_000_004 + 8_000_000
    # rectangular: x has n entries, y has m
    assert bench.alg_bytes(3, 5, 7, 8, 8) == 7 * 12 + 4 * 4 + 5 * 8 + 3 * 8
