"""Step-by-step CPU model of the two-stage speculative segmented sum.

TEST INFRASTRUCTURE (part of the oracle).  It follows the method's steps in the
paper's order and names (Section 3.1 data decomposition; Section 3.2 algorithm
description; the appendix algorithm for the first stage), written as plain
Python loops for small inputs.  Its purpose is to pin the intermediate state
that the GPU path exposes in its debug dump: tile start rows (``tile_offset``),
segment descriptors, the dirty tiles with ``dirty_counter`` and
``speculator``, and the ``synchronizer``.  The final ``y`` it produces must
equal the plain row-loop definition; the tests check that against exact dense
brute force.

Readings of the paper taken here (where it is silent or inconsistent):

* rightmost match: ``tile_offset`` = largest r in [0, m] with row_ptr[r] <= b.
* the last thread-bunch's boundaries are clamped to nnz; tiles whose left
  boundary is nnz or beyond do nothing; products past nnz are zero.
* the descriptor loop visits rows start..stop inclusive (rows < m) to set heads,
  and tests emptiness (the dirty condition) for rows start..stop-1.  Visiting
  only start..stop-1 would drop the head of row ``stop`` when that row begins
  inside the tile, which contradicts the worked example of Section 3.2.
* the transmitter is 0 at the start of every thread-bunch.
* y is zero before the first stage, so the synchronizer's additions and the
  re-arrangement's additions land on defined values.
* re-arrangement of a dirty tile: its partial 0 (row ``start``) is already in
  place; partials 1.. go, in order, to the non-empty rows strictly between
  ``start`` and ``stop``; the other rows strictly between get 0; when the tile
  ends inside row ``stop`` its last partial is added to y[stop] (the next tile
  wrote y[stop] without it, because the transmitter is cleared after a dirty
  tile).
* the speculator records the tile index beside <start, stop>, so the
  re-arrangement knows the tile's boundaries.
* rows before the first tile's start row (leading empty rows) are covered by
  no tile and keep the zero they started with; nnz = 0 gives y = 0.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np


def rightmost_match(row_ptr, b: int) -> int:
    """Binary search: the largest r in [0, m] with row_ptr[r] <= b.

    Section 3.2 requires the rightmost slot when several hold the same value
    (runs of empty rows).  row_ptr[0] = 0 <= b for every b >= 0.
    """
    lo, hi = 0, len(row_ptr) - 1
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if row_ptr[mid] <= b:
            lo = mid
        else:
            hi = mid - 1
    return lo


def segment_descriptor(row_ptr, start: int, stop: int, b: int, WT: int):
    """Head flags of the tile whose left boundary is b, and its dirty flag.

    Section 3.2: each row r of start..stop that is non-empty puts a head at
    offset row_ptr[r] - b when that offset falls inside the tile; two equal
    neighbouring row_ptr entries (an empty row) among rows start..stop-1 mark
    the tile dirty.
    """
    m = len(row_ptr) - 1
    descriptor = np.zeros(WT, dtype=bool)
    dirty = False
    for j in range(start, stop + 1):
        if j >= m:
            break
        if row_ptr[j] != row_ptr[j + 1]:
            off = row_ptr[j] - b
            if 0 <= off < WT:
                descriptor[off] = True
        elif j < stop:
            dirty = True
    return descriptor, dirty


def tile_boundaries(nnz: int, T: int, W: int, S: int, tb: int) -> List[int]:
    """Left boundaries of the S tiles of thread-bunch tb plus the right end.

    Section 3.1: a tile holds W*T nonzeros, a thread-bunch S contiguous tiles.
    Boundaries beyond nnz are clamped to nnz.
    """
    return [min(nnz, tb * S * W * T + i * W * T) for i in range(S + 1)]


@dataclasses.dataclass
class StageOneResult:
    T: int
    W: int
    S: int
    n_bunches: int
    tile_start: List[int]  # start row of every tile (tile_offset), per tile
    tile_stop: List[int]  # stop row of every tile
    descriptors: List[np.ndarray]  # W*T head flags per tile, after the forced first bit
    dirty: List[bool]  # per tile
    dirty_counter: int
    speculator: List[Tuple[int, int, int]]  # <start, stop, tile>
    synchronizer: List[Tuple[int, float]]  # <idx, val> per thread-bunch
    transmitted: List[float]  # transmitter value after each tile
    partials: List[List[float]]  # compact partial sums of each tile, in order
    y: np.ndarray  # y after the first stage


def _segment_sums(product: np.ndarray, descriptor: np.ndarray, T: int, W: int):
    """Matrix-based segmented reduction over one tile, compact output.

    The tile is T threads by W entries; thread j works on entries [jW, jW+W).
    Each segment starts at a head; its sum runs up to the next head or the end
    of the tile.  Thread j stores, compactly from the first slot of its work
    space, the sums of the segments whose heads lie in its range: ``tc[j]`` of
    them, starting at slot ``ts[j]`` = 0.  Returns (sums per thread, tc).
    """
    heads = np.nonzero(descriptor)[0]
    sums = {}
    for q, h in enumerate(heads):
        end = heads[q + 1] if q + 1 < len(heads) else W * T
        s = 0.0
        for k in range(h, end):
            s += product[k]
        sums[h] = s
    per_thread = []
    tc = []
    for j in range(T):
        own = [sums[h] for h in heads if j * W <= h < (j + 1) * W]
        per_thread.append(own)
        tc.append(len(own))
    return per_thread, tc


def exclusive_scan(a: List[int]) -> List[int]:
    out, acc = [], 0
    for v in a:
        out.append(acc)
        acc += v
    return out


def stage_one(row_ptr, col, val, x, T: int, W: int, S: int) -> StageOneResult:
    """The speculative execution stage (GPU side in the paper), all bunches."""
    row_ptr = [int(v) for v in row_ptr]
    m = len(row_ptr) - 1
    nnz = row_ptr[m]
    WT = W * T
    n_bunches = math.ceil(nnz / (S * WT)) if nnz > 0 else 0
    y = np.zeros(m, dtype=np.float64)
    res = StageOneResult(T, W, S, n_bunches, [], [], [], [], 0, [], [], [], [], y)
    for tb in range(n_bunches):
        boundary = tile_boundaries(nnz, T, W, S, tb)
        tile_offset = [rightmost_match(row_ptr, b) for b in boundary]
        transmitter = 0.0
        sync = None
        for i in range(S):
            b = boundary[i]
            if b >= nnz:
                break
            start, stop = tile_offset[i], tile_offset[i + 1]
            descriptor, dirty = segment_descriptor(row_ptr, start, stop, b, WT)
            # element-wise products, zero past nnz
            product = np.zeros(WT, dtype=np.float64)
            for j in range(WT):
                k = b + j
                if k < nnz:
                    product[j] = x[col[k]] * val[k]
            # carry from the previous tile of this bunch
            if not descriptor[0]:
                product[0] += transmitter
                descriptor[0] = True
            per_thread, tc = _segment_sums(product, descriptor, T, W)
            y_index = exclusive_scan(tc)
            tile_partials = []
            for j in range(T):
                for k in range(tc[j]):
                    index = start + y_index[j] + k
                    value = per_thread[j][k]
                    tile_partials.append(value)
                    if index == tile_offset[0]:
                        sync = (index, value)
                    else:
                        y[index] = value
                    if index == stop:
                        transmitter = value
            if dirty:
                res.dirty_counter += 1
                res.speculator.append((start, stop, tb * S + i))
                transmitter = 0.0
            res.tile_start.append(start)
            res.tile_stop.append(stop)
            res.descriptors.append(descriptor)
            res.dirty.append(dirty)
            res.transmitted.append(transmitter)
            res.partials.append(tile_partials)
        res.synchronizer.append(sync)
    return res


def stage_two(res: StageOneResult, row_ptr) -> np.ndarray:
    """Checking prediction: synchronization, then re-arrangement of dirty tiles.

    Returns the final y (a new array).
    """
    row_ptr = [int(v) for v in row_ptr]
    m = len(row_ptr) - 1
    nnz = row_ptr[m] if m >= 0 else 0
    WT = res.W * res.T
    y = res.y.copy()
    # synchronization: add each bunch's first-segment sum at its row
    for idx, value in res.synchronizer:
        y[idx] += value
    if res.dirty_counter == 0:
        return y
    for start, stop, tile in res.speculator:
        e = min(tile * WT + WT, nnz)
        rows = [r for r in range(start + 1, stop) if row_ptr[r] != row_ptr[r + 1]]
        ends_inside_stop = stop < m and row_ptr[stop] < e
        count = 1 + len(rows) + (1 if ends_inside_stop else 0)
        predicted = [y[start + k] for k in range(1, count)]  # gather first
        for r in range(start + 1, stop):
            y[r] = 0.0
        for k, r in enumerate(rows):
            y[r] = predicted[k]
        if ends_inside_stop:
            y[stop] += predicted[len(rows)]
    return y


def speculative_spmv(row_ptr, col, val, x, T: int, W: int, S: int):
    """Both stages.  Returns (y, stage-one record)."""
    r1 = stage_one(row_ptr, col, val, x, T, W, S)
    return stage_two(r1, row_ptr), r1


# ----------------------------------------------------------------------------
# vectorised plain definitions of the same intermediate quantities, for the
# GPU debug-dump comparison at sizes where the loop model is too slow.  The
# tests pin each of them to the loop model above on small inputs.
# ----------------------------------------------------------------------------

def tile_starts_vec(row_ptr: np.ndarray, T: int, W: int) -> np.ndarray:
    """Start row of every tile: rightmost r with row_ptr[r] <= t*W*T."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    nnz = int(rp[-1])
    n_tiles = -(-nnz // (W * T))
    b = np.arange(n_tiles + 1, dtype=np.int64) * (W * T)
    b = np.minimum(b, nnz)
    return np.searchsorted(rp, b, side="right") - 1


def dirty_tiles_vec(row_ptr: np.ndarray, T: int, W: int) -> np.ndarray:
    """Boolean per tile: some empty row r lies in [start, stop-1].

    An empty row r with row_ptr[r] = p lies in that range of tile t exactly
    when t*WT < p <= min((t+1)*WT, nnz); so its tile is (p-1) // WT for p > 0.
    """
    rp = np.asarray(row_ptr, dtype=np.int64)
    nnz = int(rp[-1])
    WT = W * T
    n_tiles = -(-nnz // WT)
    out = np.zeros(n_tiles, dtype=bool)
    p = rp[:-1][rp[:-1] == rp[1:]]
    p = p[p > 0]
    out[(p - 1) // WT] = True
    return out


def head_flags_vec(row_ptr: np.ndarray, T: int, W: int) -> np.ndarray:
    """Segment descriptor of every tile, concatenated (nnz flags, padded to
    whole tiles): a head at each non-empty row's first entry, plus the forced
    head at every tile's first slot."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    nnz = int(rp[-1])
    WT = W * T
    n_tiles = -(-nnz // WT)
    flags = np.zeros(n_tiles * WT, dtype=bool)
    ne = rp[:-1] != rp[1:]
    flags[rp[:-1][ne]] = True
    flags[::WT] = True
    return flags
