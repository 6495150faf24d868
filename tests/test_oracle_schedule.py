"""The oracle's processing orders (Section 2 line scan, Section 3 Algorithm 1,
and the refined sample-count criterion Section 3 suggests) against
hand-derived worked examples and properties that must hold for any loss
pattern.  The property checks recount "not yet extrapolated neighbours" (or
their unknown samples) from scratch at every wave start, independently of the
incremental updates the schedulers perform."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from schedule_golden import GOLDEN_REFINED, load_examples

EXAMPLES = load_examples()
REFINED = load_examples(GOLDEN_REFINED)


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


# ---- refined order (sample counts) -------------------------------------------

@pytest.mark.parametrize("ex", REFINED, ids=[e["name"] for e in REFINED])
def test_refined_worked_examples(ex):
    nw, wave_of, seq = oracle.schedule_refined(ex["unknown"], ex["outside"])
    assert nw == len(ex["waves"])
    flat = wave_of.ravel()
    for t, blocks in enumerate(ex["waves"]):
        assert sorted(np.flatnonzero(flat == t).tolist()) == blocks
    assert seq.tolist() == [b for w in ex["waves"] for b in w]


def check_refined_properties(unknown, outside, wave_of, nw):
    hb, wb = unknown.shape
    lost_set = {(i, j) for i in range(hb) for j in range(wb) if unknown[i, j] > 0}
    assert {(i, j) for i in range(hb) for j in range(wb) if wave_of[i, j] >= 0} == lost_set
    assert nw == (wave_of.max() + 1 if lost_set else 0)
    pending = set(lost_set)
    for t in range(nw):
        wave = {(i, j) for (i, j) in lost_set if wave_of[i, j] == t}
        assert wave
        # unknown samples around each pending block, from scratch
        cnt = {}
        for (i, j) in pending:
            nb = list(_neighbours(i, j, hb, wb))
            cnt[(i, j)] = (sum(int(unknown[y, x]) for (y, x) in nb if (y, x) in pending)
                           + (8 - len(nb)) * outside)
        nmin = min(cnt.values())
        assert all(cnt[b] == nmin for b in wave)
        for (i, j) in wave:
            assert not any(nb in wave for nb in _neighbours(i, j, hb, wb))
        cands = sorted(b for b in pending if cnt[b] == nmin)
        assert cands[0] in wave
        for b in cands:
            if b not in wave:
                assert any(nb in wave and nb < b for nb in _neighbours(*b, hb, wb))
        pending -= wave
    assert not pending


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 9), st.integers(1, 9), st.integers(0, 2**31 - 1),
       st.floats(0.0, 1.0), st.sampled_from([4, 64, 256]))
def test_refined_order_properties(hb, wb, seed, p, outside):
    rng = np.random.default_rng(seed)
    unknown = np.where(rng.random((hb, wb)) < p, rng.integers(1, outside + 1, (hb, wb)), 0)
    nw, wave_of, seq = oracle.schedule_refined(unknown.astype(np.int32), outside)
    check_refined_properties(unknown, outside, wave_of, nw)
    keys = [(wave_of.ravel()[b], b) for b in seq]
    assert keys == sorted(keys)


@settings(max_examples=100, deadline=None)
@given(st.integers(1, 10), st.integers(1, 10), st.integers(0, 2**31 - 1),
       st.floats(0.0, 1.0))
def test_refined_order_reduces_to_algorithm1_on_whole_block_losses(hb, wb, seed, p):
    # every lost block lost entirely: N is B*B times Algorithm 1's N
    lost = (np.random.default_rng(seed).random((hb, wb)) < p).astype(np.uint8)
    a = oracle.schedule(lost, oracle.ORDER_OPTIMIZED)
    b = oracle.schedule_refined(lost.astype(np.int32) * 256, 256)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


def test_refined_conceal_equals_algorithm1_on_whole_block_losses():
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, (64, 80)).astype(np.float64)
    grid = rng.random((4, 5)) < 0.5
    lost = np.kron(grid, np.ones((16, 16), bool)).astype(np.uint8)
    p0 = oracle.Params(border_d=8, iterations=20, nthreads=4)
    p2 = oracle.Params(border_d=8, iterations=20, nthreads=4, order=oracle.ORDER_REFINED)
    a = oracle.conceal(p0, img, lost)
    b = oracle.conceal(p2, img, lost)
    assert a.waves == b.waves
    np.testing.assert_array_equal(a.wave_of, b.wave_of)
    np.testing.assert_array_equal(a.image, b.image)


def test_refined_conceal_counts_partial_losses():
    # blocks (0,0) with 1 lost sample and (1,1) with a whole 16 x 16 block
    # lost, in a 32 x 32 image: the refined order takes (1,1) first
    # (corner_counts_2x2 with 16 x 16 blocks), Algorithm 1 (0,0)
    img = np.random.default_rng(6).integers(0, 256, (32, 32)).astype(np.float64)
    lost = np.zeros((32, 32), np.uint8)
    lost[3, 5] = 1
    lost[16:, 16:] = 1
    p0 = oracle.Params(border_d=8, iterations=10, nthreads=2)
    p2 = oracle.Params(border_d=8, iterations=10, nthreads=2, order=oracle.ORDER_REFINED)
    a = oracle.conceal(p0, img, lost)
    b = oracle.conceal(p2, img, lost)
    assert a.wave_of.tolist() == [[0, -1], [-1, 1]]
    assert b.wave_of.tolist() == [[1, -1], [-1, 0]]
    # the invalid order is rejected
    with pytest.raises(ValueError):
        oracle.conceal(oracle.Params(border_d=8, iterations=10, order=3), img, lost)
