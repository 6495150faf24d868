"""The oracle's processing orders (Section 2 line scan, Section 3 Algorithm 1)
against hand-derived worked examples and properties that must hold for any
loss pattern.  The property check recounts "not yet extrapolated neighbours"
from scratch at every wave start, independently of the incremental updates
the scheduler performs."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from schedule_golden import load_examples

EXAMPLES = load_examples()


@pytest.mark.parametrize("ex", EXAMPLES, ids=[e["name"] for e in EXAMPLES])
def test_worked_examples(ex):
    nw, wave_of, seq = oracle.schedule(ex["lost"], oracle.ORDER_OPTIMIZED)
    assert nw == len(ex["waves"])
    flat = wave_of.ravel()
    for t, blocks in enumerate(ex["waves"]):
        assert sorted(np.flatnonzero(flat == t).tolist()) == blocks
    assert seq.tolist() == [b for w in ex["waves"] for b in w]


def _neighbours(i, j, hb, wb):
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if (di or dj) and 0 <= i + di < hb and 0 <= j + dj < wb:
                yield i + di, j + dj


def _recount(pending, hb, wb):
    """Not-yet-extrapolated neighbours plus missing neighbours, from scratch."""
    cnt = {}
    for (i, j) in pending:
        nb = list(_neighbours(i, j, hb, wb))
        cnt[(i, j)] = sum((y, x) in pending for (y, x) in nb) + (8 - len(nb))
    return cnt


def check_schedule_properties(lost, wave_of, nw):
    hb, wb = lost.shape
    lost_set = {(i, j) for i in range(hb) for j in range(wb) if lost[i, j]}
    # every lost block exactly once, no other block
    assert {(i, j) for i in range(hb) for j in range(wb) if wave_of[i, j] >= 0} == lost_set
    assert nw == (wave_of.max() + 1 if lost_set else 0)
    pending = set(lost_set)
    for t in range(nw):
        wave = {(i, j) for (i, j) in lost_set if wave_of[i, j] == t}
        assert wave
        cnt = _recount(pending, hb, wb)
        nmin = min(cnt.values())
        # every member had the minimum count at wave start
        assert all(cnt[b] == nmin for b in wave)
        # no two members are 8-adjacent
        for (i, j) in wave:
            assert not any(nb in wave for nb in _neighbours(i, j, hb, wb))
        # greedy raster scan: the first block with the minimum is taken, and
        # every other block with the minimum touches a member that precedes
        # it in raster order
        cands = sorted(b for b in pending if cnt[b] == nmin)
        assert cands[0] in wave
        for b in cands:
            if b not in wave:
                assert any(nb in wave and nb < b for nb in _neighbours(*b, hb, wb))
        pending -= wave
    assert not pending


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 9), st.integers(1, 9), st.integers(0, 2**31 - 1),
       st.floats(0.0, 1.0))
def test_optimized_order_properties(hb, wb, seed, p):
    lost = (np.random.default_rng(seed).random((hb, wb)) < p).astype(np.uint8)
    nw, wave_of, seq = oracle.schedule(lost, oracle.ORDER_OPTIMIZED)
    check_schedule_properties(lost, wave_of, nw)
    assert nw <= int(lost.sum())
    # the sequence lists waves in order, raster order inside a wave
    keys = [(wave_of.ravel()[b], b) for b in seq]
    assert keys == sorted(keys)


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 12), st.integers(1, 12), st.integers(0, 2**31 - 1))
def test_line_scan_is_raster_order(hb, wb, seed):
    lost = (np.random.default_rng(seed).random((hb, wb)) < 0.4).astype(np.uint8)
    nw, wave_of, seq = oracle.schedule(lost, oracle.ORDER_LINESCAN)
    assert nw == int(lost.sum())
    assert seq.tolist() == np.flatnonzero(lost.ravel()).tolist()
    assert [wave_of.ravel()[b] for b in seq] == list(range(nw))


def test_rim_penalties():
    # isolated lost blocks: interior 0, margin 3, corner 5 -> three waves
    lost = np.zeros((6, 7), np.uint8)
    lost[0, 0] = lost[0, 3] = lost[3, 3] = 1
    nw, wave_of, _ = oracle.schedule(lost)
    assert nw == 3
    assert wave_of[3, 3] == 0 and wave_of[0, 3] == 1 and wave_of[0, 0] == 2


def test_single_row_and_single_block_grids():
    nw, wave_of, _ = oracle.schedule(np.ones((1, 1), np.uint8))
    assert nw == 1 and wave_of[0, 0] == 0
    lost = np.ones((1, 5), np.uint8)
    nw, wave_of, _ = oracle.schedule(lost)
    check_schedule_properties(lost, wave_of, nw)
