"""Pins of the three-dimensional FP64 oracle (``oracle/fse_oracle3d.c``, the
3-D form of FSE that the paper's conclusion names for video volumes).

Each test checks the 3-D oracle against something other than itself:
  * one frame: a volume one frame deep with a one-frame basis grid runs the
    two-dimensional oracle's arithmetic, so every result equals the 2-D
    oracle's bit for bit (block, trace and whole image), and its processing
    order equals Algorithm 1 (whose hand-derived examples are pinned in
    test_oracle_schedule.py);
  * brute force on tiny volumes: numpy's least-squares projection on every
    3-D basis function and the explicitly evaluated weighted energy choose
    the same indices and increments;
  * the initial spectrum against numpy's 3-D FFT, 3-D Parseval at several
    iterations (residual rebuilt from the trace), the energy-decrease
    identity of the greedy step, and a single 3-D exponential recovered in
    closed form;
  * the 26-neighbourhood order: hand-derived examples and properties
    recounted here from the definition.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import CLS_A, CLS_BI, CLS_BO, CLS_R


def _area3(rng, Mt, M, N, p_lost=0.3, p_rec=0.2):
    f = rng.uniform(0, 255, size=(Mt, M, N))
    u = rng.random((Mt, M, N))
    cls = np.full((Mt, M, N), CLS_A, np.uint8)
    cls[u < p_lost] = CLS_BO
    cls[(u >= p_lost) & (u < p_lost + p_rec)] = CLS_R
    cls[Mt // 2, M // 3:M // 3 + max(1, M // 3), N // 3:N // 3 + max(1, N // 3)] = CLS_BI
    return f, cls


def _weights(cls, rho, delta):
    Mt, M, N = cls.shape
    tt, mm, nn = np.mgrid[0:Mt, 0:M, 0:N]
    dist = np.sqrt((tt - (Mt - 1) / 2.0) ** 2 + (mm - (M - 1) / 2.0) ** 2 +
                   (nn - (N - 1) / 2.0) ** 2)
    return np.where(cls == CLS_A, rho ** dist, np.where(cls == CLS_R, delta * rho ** dist, 0.0))


def _basis(F, shape):
    Ft, Fh, Fw = F
    tt, mm, nn = np.mgrid[0:shape[0], 0:shape[1], 0:shape[2]]
    def phi(k):
        k1, k2, k3 = k // (Fh * Fw), (k // Fw) % Fh, k % Fw
        return np.exp(2j * np.pi * (k1 * tt / Ft + k2 * mm / Fh + k3 * nn / Fw))
    return phi


# ------------------------------------------------------------- one frame

def test_one_frame_block_equals_the_2d_oracle_bitwise():
    rng = np.random.default_rng(0)
    M, N = 20, 24
    f, cls = _area3(rng, 1, M, N)
    p3 = oracle.Params3(block_t=1, border_t=0, fft_t=1, fft_h=32, fft_w=32, iterations=40,
                        rho=0.8, delta=0.2, gamma=0.5)
    p2 = oracle.Params(fft_h=32, fft_w=32, iterations=40, rho=0.8, delta=0.2, gamma=0.5)
    r3 = oracle.block3(p3, f, cls, spec_iter=17)
    r2 = oracle.block(p2, f[0], cls[0], spec_iter=17)
    np.testing.assert_array_equal(r3.u, r2.u)
    np.testing.assert_array_equal(r3.dc, r2.dc)
    np.testing.assert_array_equal(r3.g[0], r2.g)
    np.testing.assert_array_equal(r3.energy, r2.energy)
    np.testing.assert_array_equal(r3.spectrum[0], r2.spectrum)
    assert r3.w0 == r2.w0


def test_one_frame_volume_equals_the_2d_oracle_bitwise():
    rng = np.random.default_rng(1)
    img = rng.integers(40, 220, size=(48, 64)).astype(np.float64)
    lost = np.zeros((48, 64), np.uint8)
    lost[16:32, 0:48] = 1
    lost[0:16, 48:64] = 1
    p3 = oracle.Params3(block_t=1, block_h=16, block_w=16, border_t=0, border_d=8, fft_t=1,
                        fft_h=32, fft_w=32, iterations=30)
    p2 = oracle.Params(block_h=16, block_w=16, border_d=8, fft_h=32, fft_w=32, iterations=30)
    r3 = oracle.conceal3(p3, img[None], lost[None])
    r2 = oracle.conceal(p2, img, lost)
    assert r3.waves == r2.waves
    np.testing.assert_array_equal(r3.wave_of[0], r2.wave_of)
    np.testing.assert_array_equal(r3.volume[0], r2.image)


def test_one_frame_schedule_equals_algorithm_1():
    rng = np.random.default_rng(2)
    for _ in range(60):
        hb, wb = (int(v) for v in rng.integers(1, 9, 2))
        lost = (rng.random((hb, wb)) < rng.uniform(0.1, 0.9)).astype(np.uint8)
        for order in (oracle.ORDER_OPTIMIZED, oracle.ORDER_LINESCAN):
            n3, w3, s3 = oracle.schedule3(lost[None], order)
            n2, w2, s2 = oracle.schedule(lost, order)
            assert n3 == n2
            np.testing.assert_array_equal(w3[0], w2)
            np.testing.assert_array_equal(s3, s2)


# ----------------------------------------------------------- brute force

def _brute_force3(f, cls, p, F):
    w = _weights(cls, p.rho, p.delta)
    sw = np.sqrt(w).ravel()
    r = np.where((cls == CLS_A) | (cls == CLS_R), f, 0.0).astype(np.complex128)
    phi = _basis(F, f.shape)
    nF = F[0] * F[1] * F[2]
    basis = [phi(k) for k in range(nF)]
    us, dcs = [], []
    for _ in range(p.iterations):
        cand = []
        for k in range(nF):
            a = (sw * basis[k].ravel())[:, None]
            c = np.linalg.lstsq(a, sw * r.ravel(), rcond=None)[0][0]
            e = float(np.sum(w * np.abs(r - p.gamma * c * basis[k]) ** 2))
            cand.append((e, k, c))
        emin = min(c[0] for c in cand)
        tied = [c for c in cand if c[0] <= emin * (1 + 1e-11) + 1e-300]
        e, k, c = min(tied, key=lambda t: t[1])
        us.append(k)
        dcs.append(p.gamma * c)
        r = r - p.gamma * c * basis[k]
    return np.array(us), np.array(dcs), w


@pytest.mark.parametrize("seed,shape,F", [(0, (2, 3, 3), (4, 4, 4)), (1, (3, 2, 4), (4, 4, 8)),
                                          (2, (2, 4, 3), (2, 8, 4))])
def test_brute_force_tiny_volumes(seed, shape, F):
    rng = np.random.default_rng(seed)
    f, cls = _area3(rng, *shape)
    p = oracle.Params3(fft_t=F[0], fft_h=F[1], fft_w=F[2], iterations=6, rho=0.7, delta=0.3,
                       gamma=0.5)
    res = oracle.block3(p, f, cls)
    us, dcs, w = _brute_force3(f, cls, p, F)
    assert res.w0 == pytest.approx(w.sum(), rel=1e-14)
    np.testing.assert_array_equal(res.u, us)
    np.testing.assert_allclose(res.dc, dcs, rtol=1e-9, atol=1e-9)


# ------------------------------------------- FFT, Parseval, energy, closed form

def test_initial_spectrum_matches_numpy_fftn():
    rng = np.random.default_rng(3)
    f, cls = _area3(rng, 5, 20, 18, p_lost=0.1)
    p = oracle.Params3(iterations=1)
    res = oracle.block3(p, f, cls, spec_iter=0)
    w = _weights(cls, p.rho, p.delta)
    x = np.zeros((p.fft_t, p.fft_h, p.fft_w))
    x[:5, :20, :18] = w * np.where(w > 0, f, 0.0)
    np.testing.assert_allclose(res.spectrum, np.fft.fftn(x), rtol=1e-10, atol=1e-8)


def test_known_frames_at_odd_offsets_only_tie_k1_and_k1_plus_4():
    # Degenerate case of the 3-D method: known samples only at area frames
    # t = 1 and t = 3 (one lost frame between two known ones, the others
    # outside the volume).  On the 8-frame grid e^{-j 2 pi 4 t / 8} = -1 for
    # odd t, so R[k1 + 4] = -R[k1]: every selection is an exact tie between
    # two frequencies of opposite sign on the lost frame t = 2.
    rng = np.random.default_rng(11)
    f = rng.uniform(0.0, 255.0, (5, 32, 32))
    cls = np.full((5, 32, 32), oracle.CLS_OUT, np.uint8)
    cls[1] = cls[3] = oracle.CLS_A
    cls[2] = oracle.CLS_BO
    cls[2, 8:24, 8:24] = oracle.CLS_BI
    p = oracle.Params3(iterations=1)
    sp = oracle.block3(p, f, cls, spec_iter=0).spectrum
    np.testing.assert_allclose(sp[4:], -sp[:4], rtol=0, atol=1e-9 * np.abs(sp).max())


@pytest.mark.parametrize("it", [0, 3, 9])
def test_parseval_3d(it):
    rng = np.random.default_rng(4)
    shape = (4, 10, 12)
    f, cls = _area3(rng, *shape)
    p = oracle.Params3(fft_t=8, fft_h=16, fft_w=16, iterations=12)
    res = oracle.block3(p, f, cls, spec_iter=it)
    w = _weights(cls, p.rho, p.delta)
    phi = _basis((8, 16, 16), shape)
    r = np.where(w > 0, f, 0.0).astype(np.complex128)
    for i in range(it):
        r = r - res.dc[i] * phi(int(res.u[i]))
    lhs = np.sum(np.abs(res.spectrum) ** 2)
    rhs = 8 * 16 * 16 * np.sum(w ** 2 * np.abs(r) ** 2)
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_energy_decrease_identity_3d():
    rng = np.random.default_rng(5)
    f, cls = _area3(rng, 3, 12, 12)
    p = oracle.Params3(fft_t=4, fft_h=16, fft_w=16, iterations=10, gamma=0.5)
    res = oracle.block3(p, f, cls)
    for v in range(1, p.iterations + 1):
        spec = oracle.block3(p, f, cls, spec_iter=v - 1).spectrum
        k = int(res.u[v - 1])
        P = spec.ravel()[k]
        drop = res.energy[v - 1] - res.energy[v]
        g = p.gamma
        assert drop == pytest.approx((2 * g - g * g) * abs(P) ** 2 / res.w0, rel=1e-9)
        assert res.energy[v] <= res.energy[v - 1] * (1 + 1e-12)


def test_single_3d_exponential_closed_form():
    shape, F = (4, 8, 8), (4, 16, 16)
    k0 = (1 * 16 + 5) * 16 + 3
    phi = _basis(F, shape)
    c = 37.0 - 12.0j
    f = c * phi(k0)
    cls = np.full(shape, CLS_A, np.uint8)
    p = oracle.Params3(fft_t=4, fft_h=16, fft_w=16, iterations=12, gamma=0.5)
    res = oracle.block3(p, f, cls)
    assert (res.u == k0).all()
    C = np.cumsum(res.dc)
    nu = np.arange(1, p.iterations + 1)
    np.testing.assert_allclose(C, c * (1 - (1 - p.gamma) ** nu), rtol=1e-12)


# ------------------------------------------------- 26-neighbourhood order

def test_schedule_2x2x2_all_lost_one_block_per_wave():
    nw, wave_of, seq = oracle.schedule3(np.ones((2, 2, 2), np.uint8))
    # all eight blocks are mutually 26-adjacent: one per wave, raster order
    assert nw == 8
    np.testing.assert_array_equal(seq, np.arange(8))
    np.testing.assert_array_equal(wave_of.ravel(), np.arange(8))


def test_schedule_run_of_three_frames_closes_from_both_sides():
    # three lost blocks one behind the other in time: N = 26 each (the ends
    # miss 25 neighbours and have one lost one, the middle misses 24 and has
    # two), raster order takes the first end, skips the middle, takes the
    # other end; the middle follows
    nw, wave_of, _ = oracle.schedule3(np.ones((3, 1, 1), np.uint8))
    assert nw == 2
    assert wave_of.ravel().tolist() == [0, 1, 0]


def _recount(pending, b, shape):
    tb, hb, wb = shape
    t, i, j = b
    c = 0
    for a, di, dj in itertools.product((-1, 0, 1), repeat=3):
        if not (a or di or dj):
            continue
        tt, ii, jj = t + a, i + di, j + dj
        if not (0 <= tt < tb and 0 <= ii < hb and 0 <= jj < wb) or pending[tt, ii, jj]:
            c += 1
    return c


def test_schedule_properties_recounted_from_the_definition():
    rng = np.random.default_rng(6)
    for _ in range(40):
        shape = tuple(int(v) for v in rng.integers(1, 6, 3))
        lost = (rng.random(shape) < rng.uniform(0.2, 0.9)).astype(np.uint8)
        nw, wave_of, seq = oracle.schedule3(lost)
        flat = [tuple(int(v) for v in np.unravel_index(b, shape)) for b in seq]
        assert sorted(flat) == sorted(map(tuple, np.argwhere(lost)))  # each lost block once
        pending = lost.astype(bool).copy()
        for w in range(nw):
            members = [b for b in flat if wave_of[b] == w]
            counts = {b: _recount(pending, b, shape) for b in map(tuple, np.argwhere(pending))}
            nmin = min(counts.values())
            assert all(counts[b] == nmin for b in members)
            for b1, b2 in itertools.combinations(members, 2):
                assert max(abs(x - y) for x, y in zip(b1, b2)) > 1  # not 26-adjacent
            # the first pending block in raster order with the minimal count joins
            first = min(b for b in counts if counts[b] == nmin)
            assert first in members
            # maximal: every other candidate is adjacent to a member
            for b in counts:
                if counts[b] == nmin and b not in members:
                    assert any(max(abs(x - y) for x, y in zip(b, m)) <= 1 for m in members)
            for b in members:
                pending[b] = False
        assert not pending.any()


def test_isolated_losses_give_the_same_volume_in_both_orders():
    # 3-D analogue of the paper's isolated-loss rows (0.00 dB between the
    # orders): lost blocks with no lost 26-neighbour and areas that reach no
    # further than the neighbouring blocks (d_t <= B_t, d <= B) read only
    # known samples, so the processing order cannot matter: bit for bit equal
    rng = np.random.default_rng(21)
    T, H, W = 6, 48, 64
    vol = rng.integers(0, 256, (T, H, W)).astype(np.uint8)
    lost = np.zeros_like(vol)
    for t in range(0, T, 2):
        for i in range(0, H // 8, 2):
            for j in range(0, W // 8, 2):
                if rng.random() < 0.6:
                    lost[t, 8 * i:8 * i + 8, 8 * j:8 * j + 8] = 1
    kw = dict(block_t=1, block_h=8, block_w=8, border_t=1, border_d=8, iterations=20)
    a = oracle.conceal3(oracle.Params3(order=oracle.ORDER_OPTIMIZED, **kw), vol, lost)
    b = oracle.conceal3(oracle.Params3(order=oracle.ORDER_LINESCAN, **kw), vol, lost)
    assert a.waves < b.waves == int(lost[:, ::8, ::8].sum())
    np.testing.assert_array_equal(a.volume, b.volume)
