"""Pins of the oracle's step-by-step model of the speculative method.

The model must reproduce every intermediate value the paper prints for its
worked example (Section 3.2, Fig. 3), the 6x6 segment descriptor (Section 2.1),
the auxiliary-array sizes (Section 3.3), brute-force definitions of tile start
rows and dirty tiles, and -- for its final y -- exact rational brute force.
Mutation tests plant plausible mistakes in the model and check the pins catch
each one.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import speculative as sp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_e9():
    g = json.load(open(os.path.join(GOLDEN, "e9_two_tile_example.json")))
    rp = g["row_ptr"]
    m = len(rp) - 1
    letter = g["row_letter_values"]
    val, col = [], []
    for r in range(m):
        for k in range(rp[r + 1] - rp[r]):
            val.append(float(letter[r]))
            col.append(k)
    return g, np.array(rp), np.array(col), np.array(val), np.ones(48)


def tok(s, letters):
    """'5e' -> 5 * value(e)."""
    k, L = int(s[:-1]), s[-1]
    return k * letters[L]


LETTERS = {L: i + 1 for i, L in enumerate("abcdefghij")}


def brute_y(rp, col, val, x):
    m = len(rp) - 1
    return [sum((Fraction(float(val[k])) * Fraction(float(x[col[k]])) for k in range(rp[i], rp[i + 1])),
                Fraction(0)) for i in range(m)]


def brute_tile_start(rp, b):
    """Linear scan: the last r with row_ptr[r] <= b."""
    r = 0
    for i in range(len(rp)):
        if rp[i] <= b:
            r = i
    return r


# ---------------------------------------------------------------- worked example

def test_e9_tile_offsets_and_descriptor():
    g, rp, col, val, x = load_e9()
    pr = g["printed"]
    T, W, S = g["T"], g["W"], g["S"]
    assert sp.tile_boundaries(48, T, W, S, 0) == pr["tile_boundaries"]
    assert [sp.rightmost_match(rp, b) for b in pr["tile_boundaries"]] == pr["tile_offset"]
    start, stop = pr["tile_offset"][1], pr["tile_offset"][2]
    assert list(rp[start:stop + 1]) == pr["second_tile_row_ptr"]
    assert [int(v) - 24 for v in rp[start:stop + 1]] == pr["second_tile_offsets"]
    d, dirty = sp.segment_descriptor(list(rp), start, stop, 24, W * T)
    assert list(np.nonzero(d)[0]) == pr["second_tile_effective_heads"]
    assert dirty
    r1 = sp.stage_one(rp, col, val, x, T, W, S)
    assert list(np.nonzero(r1.descriptors[1])[0]) == pr["second_tile_heads_with_forced_first"]


def test_e9_speculation_state():
    g, rp, col, val, x = load_e9()
    pr = g["printed"]
    r1 = sp.stage_one(rp, col, val, x, g["T"], g["W"], g["S"])
    assert r1.dirty_counter == pr["dirty_counter"]
    assert [(a, b) for a, b, _ in r1.speculator] == [tuple(p) for p in pr["speculator"]]
    assert r1.transmitted[0] == tok(pr["first_tile_transmitted"], LETTERS)
    idx, v = pr["synchronizer_0"]
    assert r1.synchronizer[0] == (idx, tok(v, LETTERS))
    wrong = [tok(s, LETTERS) for s in pr["wrong_slot_rows_4_to_9_before_rearrangement"]]
    assert list(r1.y[4:10]) == wrong


def test_e9_rearrangement_and_final():
    g, rp, col, val, x = load_e9()
    pr = g["printed"]
    y, _ = sp.speculative_spmv(rp, col, val, x, g["T"], g["W"], g["S"])
    for s, row in pr["moved_entries_final_rows"].items():
        assert y[row] == tok(s, LETTERS)
    assert y[6] == 0 and y[9] == 0
    assert [Fraction(v) for v in y] == brute_y(rp, col, val, x)


def test_e8_descriptor_one_tile():
    g = json.load(open(os.path.join(GOLDEN, "e8_csr_6x6.json")))
    # one tile of W*T = 12 entries covers the whole matrix
    r1 = sp.stage_one(g["row_ptr"], g["col"], np.ones(12), np.ones(6), T=4, W=3, S=1)
    assert [int(b) for b in r1.descriptors[0]] == g["segment_descriptor"]
    assert r1.dirty == [True]  # row 3 is empty


# ---------------------------------------------------------------- random pins

@st.composite
def csr_case(draw):
    m = draw(st.integers(0, 30))
    n = draw(st.integers(1, 12))
    kinds = st.sampled_from(["empty", "short", "long", "any"])
    lengths = []
    for _ in range(m):
        k = draw(kinds)
        if k == "empty":
            lengths.append(0)
        elif k == "short":
            lengths.append(draw(st.integers(1, 3)))
        elif k == "long":
            lengths.append(draw(st.integers(8, 40)))
        else:
            lengths.append(draw(st.integers(0, 12)))
    rp = [0]
    for L in lengths:
        rp.append(rp[-1] + L)
    nnz = rp[-1]
    col = [draw(st.integers(0, n - 1)) for _ in range(nnz)]
    val = [float(draw(st.integers(-3, 3))) for _ in range(nnz)]
    x = [float(draw(st.integers(-3, 3))) for _ in range(n)]
    T = draw(st.sampled_from([1, 2, 3, 4, 8]))
    W = draw(st.integers(1, 6))
    S = draw(st.integers(1, 4))
    return np.array(rp), np.array(col, dtype=np.int64), np.array(val), np.array(x), T, W, S


@settings(max_examples=1500, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(csr_case())
def test_model_matches_brute_force(case):
    rp, col, val, x, T, W, S = case
    y, r1 = sp.speculative_spmv(rp, col, val, x, T, W, S)
    assert [Fraction(v) for v in y] == brute_y(rp, col, val, x)
    nnz = int(rp[-1])
    WT = W * T
    # aux sizes (Section 3.3)
    assert r1.n_bunches == (math.ceil(nnz / (S * WT)) if nnz else 0)
    assert len(r1.synchronizer) == r1.n_bunches
    n_tiles = math.ceil(nnz / WT) if nnz else 0
    assert len(r1.tile_start) == n_tiles and r1.dirty_counter <= n_tiles
    # tile start rows by linear scan; dirty by its definition
    for t in range(n_tiles):
        b, e = t * WT, min(t * WT + WT, nnz)
        start, stop = brute_tile_start(rp, b), brute_tile_start(rp, e)
        assert (r1.tile_start[t], r1.tile_stop[t]) == (start, stop)
        assert r1.dirty[t] == any(rp[r] == rp[r + 1] for r in range(start, stop))
    # vectorised definitions used at scale agree with the loop model
    if n_tiles:
        ts = sp.tile_starts_vec(rp, T, W)
        assert list(ts[:-1]) == r1.tile_start
        assert list(sp.dirty_tiles_vec(rp, T, W)) == r1.dirty
        hf = sp.head_flags_vec(rp, T, W)
        assert np.array_equal(hf, np.concatenate(r1.descriptors))
    # every bunch's synchronizer row is its first tile's start row
    for tb in range(r1.n_bunches):
        assert r1.synchronizer[tb][0] == r1.tile_start[tb * S]


FORCED = {
    "no_empty_rows": [3, 1, 4, 1, 5, 9, 2, 6, 5, 3],
    "all_tiles_dirty": [1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0],
    "leading_trailing_empties": [0, 0, 0, 2, 3, 0, 4, 0, 0, 0],
    "nnz_zero": [0, 0, 0, 0],
    "boundary_aligned_rows": [4, 4, 4, 4, 0, 4, 4],
    "one_row_many_bunches": [1, 200, 1, 0, 2],
    "long_empty_run_in_tile": [2] + [0] * 1000 + [3, 1],
    "m_zero": [],
}


@pytest.mark.parametrize("name", sorted(FORCED))
@pytest.mark.parametrize("TWS", [(4, 1, 1), (2, 2, 2), (4, 3, 2), (1, 4, 3)])
def test_model_forced_cases(name, TWS):
    lengths = FORCED[name]
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64) if lengths else np.array([0])
    nnz = int(rp[-1])
    rng = np.random.default_rng(len(lengths))
    col = rng.integers(0, 5, nnz)
    val = rng.integers(-3, 4, nnz).astype(float)
    x = rng.integers(-3, 4, 5).astype(float)
    T, W, S = TWS
    y, r1 = sp.speculative_spmv(rp, col, val, x, T, W, S)
    assert [Fraction(v) for v in y] == brute_y(rp, col, val, x)
    if name == "no_empty_rows":
        assert r1.dirty_counter == 0
    if name == "all_tiles_dirty" and T * W <= 2:
        assert r1.dirty_counter == len(r1.tile_start)


# ---------------------------------------------------------------- planted mistakes

def _pins_fail(monkeypatch_ctx) -> bool:
    """True when at least one of the example pins fails under a mutation."""
    checks = [test_e9_tile_offsets_and_descriptor, test_e9_speculation_state,
              test_e9_rearrangement_and_final, test_e8_descriptor_one_tile]
    for c in checks:
        try:
            c()
        except Exception:
            return True
    # random cases
    rng = np.random.default_rng(99)
    for _ in range(300):
        m = int(rng.integers(1, 20))
        lengths = rng.integers(0, 9, m)
        lengths[rng.random(m) < 0.3] = 0
        rp = np.concatenate([[0], np.cumsum(lengths)])
        nnz = int(rp[-1])
        col = rng.integers(0, 6, nnz)
        val = rng.integers(-3, 4, nnz).astype(float)
        x = rng.integers(-3, 4, 6).astype(float)
        T, W, S = int(rng.integers(1, 5)), int(rng.integers(1, 5)), int(rng.integers(1, 4))
        try:
            y, _ = sp.speculative_spmv(rp, col, val, x, T, W, S)
        except Exception:
            return True
        if [Fraction(v) for v in y] != brute_y(rp, col, val, x):
            return True
    return False


def leftmost_match(row_ptr, b):
    lo, hi = 0, len(row_ptr) - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if row_ptr[mid] < b:
            lo = mid + 1
        else:
            hi = mid
    return lo if row_ptr[lo] <= b else lo - 1


def descriptor_literal_bound(row_ptr, start, stop, b, WT):
    """Rows start..stop-1 only (drops the head of row stop)."""
    m = len(row_ptr) - 1
    d = np.zeros(WT, dtype=bool)
    dirty = False
    for j in range(start, stop):
        if j >= m:
            break
        if row_ptr[j] != row_ptr[j + 1]:
            off = row_ptr[j] - b
            if 0 <= off < WT:
                d[off] = True
        else:
            dirty = True
    return d, dirty


_ORIG_DESCRIPTOR = sp.segment_descriptor
_ORIG_SEGMENT_SUMS = sp._segment_sums


def descriptor_no_dirty(row_ptr, start, stop, b, WT):
    d, _ = _ORIG_DESCRIPTOR(row_ptr, start, stop, b, WT)
    return d, False


def segment_sums_drop_last(product, descriptor, T, W):
    per, tc = _ORIG_SEGMENT_SUMS(product, descriptor, T, W)
    # lose the last entry of every segment
    heads = list(np.nonzero(descriptor)[0]) + [W * T]
    sums = [sum(product[heads[q]:heads[q + 1] - 1]) for q in range(len(heads) - 1)]
    out, it = [], iter(sums)
    for j in range(T):
        out.append([next(it) for _ in range(tc[j])])
    return out, tc


def exclusive_as_inclusive(a):
    out, acc = [], 0
    for v in a:
        acc += v
        out.append(acc)
    return out


@pytest.mark.parametrize("mutant", [
    ("rightmost_match", leftmost_match),
    ("segment_descriptor", descriptor_literal_bound),
    ("segment_descriptor", descriptor_no_dirty),
    ("_segment_sums", segment_sums_drop_last),
    ("exclusive_scan", exclusive_as_inclusive),
])
def test_planted_mistakes_are_caught(monkeypatch, mutant):
    name, fn = mutant
    monkeypatch.setattr(sp, name, fn)
    assert _pins_fail(monkeypatch)
