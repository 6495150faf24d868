"""Pins of two whole-image behaviours of the oracle that the per-area pins do
not reach: how an area that crosses the image border is classified and
weighted, and which image a block of a wave reads.

* Border (Section 2 with Eq. (2); reading: samples outside the image carry no
  weight and no value, the block keeps its nominal geometry and only its
  samples inside the image are extrapolated).  The expected area is built
  here by hand from the image and the mask, and the expected model comes from
  a brute-force weighted least-squares search in numpy, not from the oracle.
* Snapshot (Section 3: the blocks of a wave are extrapolated in parallel;
  reading: every block of a wave reads the image and the sample states as
  they were when the wave started).  The snapshots of both waves of a small
  image with d larger than the block are rebuilt here by hand, each block is
  modelled on its hand-built area with ``oracle.block`` (pinned separately),
  and the assembled image must equal ``oracle.conceal`` bit for bit.
"""
import numpy as np

import oracle
from oracle import CLS_A, CLS_BI, CLS_BO, CLS_OUT, CLS_R

KNOWN, PENDING, RECON = 0, 1, 2


def _hand_area(img, state, y0, x0, Bh, Bw, d):
    """Values and classes of the area of the block whose top-left sample is
    (y0, x0): rows y0-d .. y0+Bh+d-1, columns likewise; positions outside the
    image are CLS_OUT with value 0."""
    H, W = img.shape
    M, N = Bh + 2 * d, Bw + 2 * d
    f = np.zeros((M, N))
    cls = np.full((M, N), CLS_OUT, np.uint8)
    for m in range(M):
        for n in range(N):
            y, x = y0 - d + m, x0 - d + n
            if not (0 <= y < H and 0 <= x < W):
                continue
            f[m, n] = img[y, x]
            if state[y, x] == KNOWN:
                cls[m, n] = CLS_A
            elif state[y, x] == RECON:
                cls[m, n] = CLS_R
            elif y0 <= y < y0 + Bh and x0 <= x < x0 + Bw:
                cls[m, n] = CLS_BI
            else:
                cls[m, n] = CLS_BO
    return f, cls


def _brute_force_model(f, cls, rho, delta, gamma, K, MF, NF):
    """Greedy weighted model by exhaustive search: every candidate
    coefficient from numpy's least-squares solver on the sqrt(w)-scaled
    problem, the candidate leaving the smallest weighted residual energy
    kept (ties within rounding to the smallest index).  Returns Re of the
    model over the area."""
    M, N = f.shape
    mm, nn = np.mgrid[0:M, 0:N]
    dist = np.sqrt((mm - (M - 1) / 2.0) ** 2 + (nn - (N - 1) / 2.0) ** 2)
    w = np.where(cls == CLS_A, rho ** dist, np.where(cls == CLS_R, delta * rho ** dist, 0.0))
    sw = np.sqrt(w).ravel()
    r = np.where(w > 0, f, 0.0).astype(np.complex128)
    g = np.zeros((M, N), np.complex128)
    for _ in range(K):
        cand = []
        for k1 in range(MF):
            for k2 in range(NF):
                phi = np.exp(2j * np.pi * (k1 * mm / MF + k2 * nn / NF))
                c = np.linalg.lstsq((sw * phi.ravel())[:, None], sw * r.ravel(), rcond=None)[0][0]
                cand.append((float(np.sum(w * np.abs(r - gamma * c * phi) ** 2)), k1 * NF + k2,
                             gamma * c, phi))
        emin = min(t[0] for t in cand)
        _, _, dc, phi = min((t for t in cand if t[0] <= emin * (1 + 1e-11) + 1e-300),
                            key=lambda t: t[1])
        r = r - dc * phi
        g = g + dc * phi
    return g.real, w


def test_corner_and_partial_edge_blocks_weigh_outside_samples_zero():
    # 6 x 7 image, 2 x 2 blocks (grid 3 x 4, the last column of blocks one
    # sample wide), d = 2: the corner block (0, 0) is lost entirely, and one
    # sample of the partial block (2, 3) at the bottom-right corner
    rng = np.random.default_rng(17)
    H, W, B, d = 6, 7, 2, 2
    img = rng.uniform(20, 230, (H, W)).round()
    lost = np.zeros((H, W), np.uint8)
    lost[0:2, 0:2] = 1
    lost[5, 6] = 1
    p = oracle.Params(block_w=B, block_h=B, border_d=d, fft_w=8, fft_h=8, iterations=6,
                      rho=0.7, delta=0.3, gamma=0.5)
    res = oracle.conceal(p, img, lost)
    assert res.waves == 1  # the two lost blocks are not adjacent: one wave
    state = np.where(lost > 0, PENDING, KNOWN).astype(np.uint8)
    work = np.where(lost > 0, 0.0, img)
    for (bi, bj) in ((0, 0), (2, 3)):
        f, cls = _hand_area(work, state, bi * B, bj * B, B, B, d)
        # the oracle's own area extraction agrees with the hand-built classes
        fo, co = oracle.extract_area(p, work, state, bi, bj)
        np.testing.assert_array_equal(co, cls)
        assert (cls == CLS_OUT).sum() == (20 if (bi, bj) == (0, 0) else 24)
        g, w = _brute_force_model(f, cls, p.rho, p.delta, p.gamma, p.iterations, 8, 8)
        assert w[cls == CLS_OUT].sum() == 0.0
        for m, n in zip(*np.nonzero(cls == CLS_BI)):
            y, x = bi * B - d + m, bj * B - d + n
            assert abs(res.image[y, x] - g[m, n]) <= 1e-9, (bi, bj, m, n)
    # the samples outside the blocks' image part are never written
    np.testing.assert_array_equal(res.image[lost == 0], img[lost == 0])


def test_blocks_of_a_wave_read_the_snapshot_of_its_start():
    # 8 x 12 image, 2 x 2 blocks (grid 4 x 6), d = 3 > block size: lost
    # blocks (1, 1), (1, 3), (2, 1), (2, 3).  All four start with N = 1, so
    # wave 0 = {(1, 1), (1, 3)} and wave 1 = {(2, 1), (2, 3)}; the area of
    # either block of a wave reaches into the other block of the same wave.
    rng = np.random.default_rng(23)
    H, W, B, d = 8, 12, 2, 3
    img = rng.uniform(20, 230, (H, W)).round()
    lost = np.zeros((H, W), np.uint8)
    blocks = [(1, 1), (1, 3), (2, 1), (2, 3)]
    for bi, bj in blocks:
        lost[bi * B:(bi + 1) * B, bj * B:(bj + 1) * B] = 1
    p = oracle.Params(block_w=B, block_h=B, border_d=d, fft_w=8, fft_h=8, iterations=5,
                      rho=0.75, delta=0.3, gamma=0.5, nthreads=1)
    res = oracle.conceal(p, img, lost)
    assert res.waves == 2
    assert [res.wave_of[b] for b in blocks] == [0, 0, 1, 1]

    work = np.where(lost > 0, 0.0, img)
    state = np.where(lost > 0, PENDING, KNOWN).astype(np.uint8)
    for wave in ([(1, 1), (1, 3)], [(2, 1), (2, 3)]):
        snap, snap_state = work.copy(), state.copy()  # the wave's snapshot
        results = []
        for bi, bj in wave:
            f, cls = _hand_area(snap, snap_state, bi * B, bj * B, B, B, d)
            # the other block of the wave is still pending in this snapshot
            assert (cls == CLS_BO).sum() > 0
            if wave[0][0] == 2:  # the second wave reads the first one's samples
                assert (cls == CLS_R).sum() > 0
            results.append((bi, bj, cls, oracle.block(p, f, cls).g))
        for bi, bj, cls, g in results:
            for m, n in zip(*np.nonzero(cls == CLS_BI)):
                y, x = bi * B - d + m, bj * B - d + n
                work[y, x] = g[m, n]
                state[y, x] = RECON
    np.testing.assert_array_equal(res.image, work)
