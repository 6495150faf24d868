"""The library's 26-neighbourhood processing order (fse_schedule3) against
the oracle's independent one (Algorithm 1 carried to a block grid over
frames, rows and columns), on random grids in both orders."""
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import paper_2207_00233_amd as fse


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fse.LIB_PATH):
        from paper_2207_00233_amd import build
        build.build()
    return fse.load()


@settings(max_examples=150, deadline=None)
@given(st.integers(1, 6), st.integers(1, 8), st.integers(1, 8), st.integers(0, 2**31 - 1),
       st.floats(0.0, 1.0), st.sampled_from([0, 1]))
def test_schedule3_matches_oracle(lib, tb, hb, wb, seed, p, order):
    lost = (np.random.default_rng(seed).random((tb, hb, wb)) < p).astype(np.uint8)
    a = fse.schedule3(lost, order)
    b = oracle.schedule3(lost, order)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


def test_schedule3_video_grid(lib):
    # 30 frames of a 1080p block grid with 20 % of the blocks lost
    lost = (np.random.default_rng(3).random((30, 68, 120)) < 0.2).astype(np.uint8)
    a = fse.schedule3(lost)
    b = oracle.schedule3(lost)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])


def test_schedule3_rejects(lib):
    assert lib.fse_schedule3(-1, 2, 2, None, 0, None, None) == fse.FSE_ERR_INVALID
    assert lib.fse_schedule3(2, 2, 2, None, 3, None, None) == fse.FSE_ERR_INVALID
    assert lib.fse_schedule3(0, 2, 2, None, 0, None, None) == 0
    assert lib.fse_schedule3(1, 2, 2, None, 0, None, None) == fse.FSE_ERR_INVALID
