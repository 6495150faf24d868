"""Near-tie re-scoring of FSE_FP32_RERANK: every entry inside the near window
is re-scored, however many one wavefront holds.

The input is a 44 x 44 image that is its own extrapolation area: one lost
16 x 16 block in the middle (block grid shifted by 2 samples, d = 14), with
the known samples symmetric under both reflections about the area centre
and under transposition (a texture at frequencies (2, 6) plus its transpose).  The weights of Eq. (2) have the same symmetry, so
|P[k1, k2]| = |P[-k1, k2]| = |P[k2, k1]| exactly: the largest entry comes in
a group of eight, four of which share register rows of one wavefront: after
four selections of the DC entry the window holds (+-2, +-6) and (+-6, +-2),
with (2, 6), (2, 58), (6, 2), (6, 62) in the rows of wavefront 0.  The test checks that the call reports a
wavefront with more than three candidates, and that every selection is a
maximizer of the exact residual spectrum
    P_v[k] = R0[k] - sum_{i<v} dc_i W[k - u_i]
rebuilt in double from the GPU's own trace (R0 and W from the oracle's
explicit sums; the update identity of the transform domain, pinned in the
oracle tests), to 1e-9 of the largest |R0| (the re-scoring's FP64 spectra).
"""
import numpy as np
import pytest

import oracle
import paper_2207_00233_amd as fse

pytestmark = pytest.mark.gpu

B, D, S = 16, 14, 44


def symmetric_image():
    c = (S - 1) / 2.0
    r = np.abs(np.arange(S) - c)
    a, b = np.meshgrid(r, r, indexing="ij")

    def h(p, q):  # frequencies (2, 6) and, transposed, (6, 2): rows 2 and 6 of wavefront 0
        return 45 * np.cos(2 * np.pi * 2 * p / 64) * np.cos(2 * np.pi * 6 * q / 64)

    img = np.clip(np.rint(128 + h(a, b) + h(b, a)), 0, 255).astype(np.uint8)
    assert (img == img.T).all() and (img == img[::-1]).all() and (img == img[:, ::-1]).all()
    lost = np.zeros((S, S), np.uint8)
    lost[D:D + B, D:D + B] = 1
    return img, lost


def test_many_candidates_in_one_wavefront():
    precision, rel = fse.FSE_FP32_RERANK, 1e-9
    img, lost = symmetric_image()
    K = 60
    p = fse.Params(border_d=D, iterations=K, grid_off_x=2, grid_off_y=2, precision=precision)
    print(f"[gpu] symmetric area, precision {precision}", flush=True)
    with fse.Plan(p) as plan:
        plan.set_tuning(wave_threshold_16=0, wave_threshold_8=0)  # 4 wavefronts per block
        r = plan.fse_conceal_image([img], [lost], want_float=True, trace=True)[0]
        st = plan.last_call_stats()
    print(f"[rescore] stats {st}", flush=True)
    assert st["rescored"] >= 1
    assert st["rescore_max_wave"] >= 4 and st["rescore_wide"] >= 1
    assert r.trace_block.tolist() == [1 * 3 + 1]
    op = oracle.Params(border_d=D, iterations=K, grid_off_x=2, grid_off_y=2)
    state = np.where(lost.astype(bool), 1, 0).astype(np.uint8)
    f, cls = oracle.extract_area(op, np.where(lost.astype(bool), 0.0, img.astype(np.float64)),
                                 state, 1, 1)
    R0 = oracle.block(op, f, cls, spec_iter=0).spectrum
    Wk = oracle.block(op, np.ones_like(f), cls, spec_iter=0).spectrum
    scale = np.abs(R0).max()
    u, dc = r.trace_u[0], r.trace_dc[0]
    P = R0.copy()
    for v in range(K):
        mag = np.abs(P)
        k1, k2 = divmod(int(u[v]), 64)
        assert mag[k1, k2] >= mag.max() - rel * scale, (v, int(u[v]), mag[k1, k2], mag.max())
        P = P - dc[v] * np.roll(Wk, (k1, k2), axis=(0, 1))


def test_zero_spectrum_is_not_rescored():
    """A black image: every spectrum entry is exactly 0, so all 4096 tie.  The
    float maximum never rises above the floor (2^-40 of the first maximum),
    so no iteration is re-scored and the model stays 0, as in the oracle."""
    img = np.zeros((64, 80), np.uint8)
    rng = np.random.default_rng(4)
    lost = (rng.random((64, 80)) < 0.3).astype(np.uint8)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_RERANK)
    print("[gpu] black image, re-rank", flush=True)
    with fse.Plan(p) as plan:
        r = plan.fse_conceal_image([img], [lost], want_float=True)[0]
        st = plan.last_call_stats()
    assert st["rescored"] == 0, st
    np.testing.assert_array_equal(r.out_f, 0.0)
    np.testing.assert_array_equal(r.out, img)
