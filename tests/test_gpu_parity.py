"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (stated for this workload, on the 8-bit sample scale):
  * FSE_FP64: 1e-7 max-abs (teacher-forced and free-running); both sides
    compute the same sums in double, only the summation order differs.
  * FSE_FP32_RERANK (FP64 transforms, float iteration, exact re-scoring of
    near ties): 0.5 max-abs for every block when the block gets exactly the
    input the oracle gets (teacher-forced), and 0.02 dB PSNR gap over the
    lost samples of whole images run free.  Free-running max-abs is
    reported, not bounded: the greedy selection is discontinuous at
    near-ties, so any upstream difference (even one the oracle itself would
    make under a 1e-6 input change) can switch a later block to another,
    equally good model.
  * FSE_FP32 and FSE_FP32_F16X3 (float transforms) do NOT meet the 0.5
    bar on every block: their spectra carry rounding of about 1e-7 of the
    largest spectrum entry, which decides near ties differently from FP64 in
    a few blocks in a hundred (measured worst 2.9 on the 8-bit scale).  Their
    tests are characterizations, marked as such: the PSNR gap, the median
    block error and the share of blocks within 0.5.
Selected indices are compared modulo the mirror k -> -k, because a real
residual gives exact ties |R[k]| = |R[-k]| whose choice does not change the
real part of the model.
"""
import dataclasses
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import paper_2207_00233_amd as fse
from paper_2207_00233_amd import synth
from parity import index_agreement, mirror, psnr, teacher_forced_block

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-7
FP32_TOL = 0.5
PSNR_GAP = 0.02


def below_bar_characterization(errs, label):
    """FSE_FP32 / FSE_FP32_F16X3 (below the 0.5 bar, see the module
    docstring): typical blocks agree, a few near ties go the other way."""
    print(f"[below-bar] {label}: median {np.median(errs):.3e} max {errs.max():.3e}, "
          f"{np.mean(errs <= FP32_TOL):.3f} within {FP32_TOL} over {len(errs)} blocks", flush=True)
    assert np.median(errs) <= 0.05
    assert np.mean(errs <= FP32_TOL) >= 0.9


def oracle_params(p: fse.Params, nthreads=0) -> oracle.Params:
    return oracle.Params(block_w=p.block_w, block_h=p.block_h, border_d=p.border_d,
                         fft_w=p.fft_w, fft_h=p.fft_h, rho=p.rho, delta=p.delta,
                         gamma=p.gamma, iterations=p.iterations, order=p.order,
                         empty_fill=p.empty_fill, nthreads=nthreads,
                         grid_off_x=p.grid_off_x, grid_off_y=p.grid_off_y)


def run_gpu(p, images, losts, trace=False):
    print(f"[gpu] conceal {len(images)} frame(s) {[im.shape for im in images]} "
          f"prec={p.precision} K={p.iterations} d={p.border_d} B={p.block_h}x{p.block_w}",
          flush=True)
    with fse.Plan(p) as plan:
        return plan.fse_conceal_image(images, losts, want_float=True, trace=trace)


def quantize(v, lost, image):
    q = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return np.where(lost.astype(bool), q, image)


def check_free_running(p, img, lost, tol, psnr_gap=None):
    r = run_gpu(p, [img], [lost])[0]
    o = oracle.conceal(oracle_params(p, nthreads=8), img, lost)
    m = lost.astype(bool)
    assert r.waves == o.waves
    err = np.abs(r.out_f[m] - o.image[m]).max() if m.any() else 0.0
    print(f"[parity] free-running max-abs {err:.3e}", flush=True)
    if tol is not None:
        assert err <= tol, err
    # known samples are copied bit for bit
    np.testing.assert_array_equal(r.out[~m], img[~m])
    np.testing.assert_array_equal(r.out, quantize(r.out_f, lost, img))
    if psnr_gap is not None and m.any():
        gap = abs(psnr(r.out, img, lost) - psnr(quantize(o.image, lost, img), img, lost))
        assert gap <= psnr_gap, gap
    return r, o


# ------------------------------------------------------------ config 1

def config1_params(precision):
    return fse.Params(border_d=8, iterations=100, grid_off_x=8, grid_off_y=8,
                      precision=precision)


def test_config1_fp64_matches_oracle():
    fr = synth.config1()
    p = config1_params(fse.FSE_FP64)
    r = run_gpu(p, [fr.image], [fr.lost], trace=True)[0]
    o = oracle.conceal(oracle_params(p), fr.image, fr.lost, trace=True)
    m = fr.lost.astype(bool)
    assert np.abs(r.out_f[m] - o.image[m]).max() <= FP64_TOL
    assert r.trace_block.tolist() == [2 * 5 + 2]
    agree, first_bad = index_agreement(o.u[2, 2], r.trace_u[0])
    assert agree == 1.0, (agree, first_bad)


def test_config1_fp32_within_tolerance():
    fr = synth.config1()
    check_free_running(config1_params(fse.FSE_FP32), fr.image, fr.lost, FP32_TOL, PSNR_GAP)


# ------------------------------------------------------------ whole images

@pytest.mark.parametrize("order", [fse.FSE_ORDER_OPTIMIZED, fse.FSE_ORDER_LINESCAN])
def test_fp64_free_running_polygon_image(order):
    rng = np.random.default_rng(21)
    img = synth.polygon_image(rng, 100, 120, radius=(10, 60))
    lost = synth.bernoulli_block_loss(rng, 100, 120, 16, 0.35)
    p = fse.Params(border_d=14, iterations=60, precision=fse.FSE_FP64, order=order)
    check_free_running(p, img, lost, FP64_TOL)


@pytest.mark.parametrize("order", [fse.FSE_ORDER_OPTIMIZED, fse.FSE_ORDER_LINESCAN])
def test_fp32_free_running_polygon_image(order):
    rng = np.random.default_rng(22)
    img = synth.polygon_image(rng, 100, 120, radius=(10, 60))
    lost = synth.bernoulli_block_loss(rng, 100, 120, 16, 0.35)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32, order=order)
    check_free_running(p, img, lost, None, PSNR_GAP)


@pytest.mark.parametrize("seed", [5, 11])
def test_fp32_teacher_forced_blocks(seed):
    fr = synth.config2(seed=seed, size=128)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32)
    r = run_gpu(p, [fr.image], [fr.lost])[0]
    op = oracle_params(p)
    _, wave_of, seq = oracle.schedule(
        fr.lost.reshape(8, 16, 8, 16).any(axis=(1, 3)).astype(np.uint8))
    worst = 0.0
    for b in seq:
        o_v, g_v, _ = teacher_forced_block(fr.image, fr.lost, r.out_f.astype(np.float64),
                                           wave_of, op, b // 8, b % 8)
        worst = max(worst, np.abs(o_v - g_v).max())
    print(f"[parity] FP32 teacher-forced max-abs over {len(seq)} blocks: {worst:.3e}", flush=True)
    assert worst <= FP32_TOL, worst


def test_fp64_trace_matches_oracle_trace():
    fr = synth.config2(seed=6, size=96)
    p = fse.Params(border_d=14, iterations=40, precision=fse.FSE_FP64)
    r = run_gpu(p, [fr.image], [fr.lost], trace=True)[0]
    o = oracle.conceal(oracle_params(p, nthreads=8), fr.image, fr.lost, trace=True)
    wb = 6
    for slot, b in enumerate(r.trace_block):
        assert r.trace_wave[slot] == o.wave_of[b // wb, b % wb]
        agree, first_bad = index_agreement(o.u[b // wb, b % wb], r.trace_u[slot])
        assert agree == 1.0, (b, agree, first_bad)


# ------------------------------------------------------------ f16x3 transforms
# FSE_FP32_F16X3 computes both DFT stages on matrix cores with every operand
# split into two f16 parts (about 22 significant bits, three products each,
# float accumulation).  The bar: the first coefficient increment
# gamma X[u] / W0 of every block within 1e-5 relative of the oracle's on the
# same area (three split products lose ~2^-21 per term, float accumulation
# ~1e-7 more), and the PSNR gap on whole images; per block the mode is below
# the 0.5 bar (characterized, see the module docstring).

F16X3_DC_TOL = 1e-5


def test_f16x3_first_increment_matches_oracle():
    fr = synth.config2(seed=6, size=96)
    p = fse.Params(border_d=14, iterations=1, precision=fse.FSE_FP32_F16X3)
    r = run_gpu(p, [fr.image], [fr.lost], trace=True)[0]
    op = oracle_params(p)
    grid = fr.lost.reshape(6, 16, 6, 16).any(axis=(1, 3)).astype(np.uint8)
    _, wave_of, _ = oracle.schedule(grid)
    worst = 0.0
    for slot, b in enumerate(r.trace_block):
        _, _, res = teacher_forced_block(fr.image, fr.lost, r.out_f.astype(np.float64),
                                         wave_of, op, b // 6, b % 6)
        u_o, dc_o = int(res.u[0]), complex(res.dc[0])
        u_g, dc_g = int(r.trace_u[slot][0]), complex(r.trace_dc[slot][0])
        if u_g != u_o:  # the exact mirror tie of a real area
            assert u_g == int(mirror(u_o)), (b, u_g, u_o)
            dc_o = dc_o.conjugate()
        worst = max(worst, abs(dc_g - dc_o) / abs(dc_o))
    print(f"[parity] f16x3 first increment: worst relative error {worst:.3e} over "
          f"{len(r.trace_block)} blocks", flush=True)
    assert worst <= F16X3_DC_TOL, worst


@pytest.mark.parametrize("seed", [5, 11])
def test_f16x3_teacher_forced_blocks(seed):
    fr = synth.config2(seed=seed, size=128)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_F16X3)
    r = run_gpu(p, [fr.image], [fr.lost])[0]
    op = oracle_params(p)
    _, wave_of, seq = oracle.schedule(
        fr.lost.reshape(8, 16, 8, 16).any(axis=(1, 3)).astype(np.uint8))
    errs = np.array([np.abs(np.subtract(*teacher_forced_block(
        fr.image, fr.lost, r.out_f.astype(np.float64), wave_of, op, b // 8, b % 8)[:2])).max()
        for b in seq])
    print(f"[parity] f16x3 teacher-forced median {np.median(errs):.3e} max {errs.max():.3e}, "
          f"{np.mean(errs <= FP32_TOL):.3f} within {FP32_TOL} over {len(seq)} blocks", flush=True)
    below_bar_characterization(errs, "FSE_FP32_F16X3 teacher-forced")


def test_f16x3_free_running_and_batch_identity():
    rng = np.random.default_rng(22)
    img = synth.polygon_image(rng, 100, 120, radius=(10, 60))
    lost = synth.bernoulli_block_loss(rng, 100, 120, 16, 0.35)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_F16X3)
    r, _ = check_free_running(p, img, lost, None, PSNR_GAP)
    other = synth.polygon_image(rng, 64, 80, radius=(10, 30))
    olost = synth.slice_loss(rng, 64, 80, 16, (0.2, 0.4))
    rb = run_gpu(p, [other, img], [olost, lost])[1]
    np.testing.assert_array_equal(rb.out_f, r.out_f)


def test_f16x3_reconstructed_samples_above_256():
    """A bright square-wave texture whose extrapolation overshoots 256: later
    blocks read reconstructed samples above 256, which the f16 transforms
    scale down by a power of two (and back) to keep every operand in range."""
    rng = np.random.default_rng(3)
    yy, xx = np.mgrid[0:96, 0:96]
    img = np.clip(200 + 60 * np.sign(np.sin(2 * np.pi * xx / 7.0) * np.sin(2 * np.pi * yy / 9.0)),
                  0, 255).astype(np.uint8)
    lost = synth.slice_loss(rng, 96, 96, 16, (0.3, 0.5))
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_F16X3)
    r, _ = check_free_running(p, img, lost, None, PSNR_GAP)
    assert r.out_f[lost.astype(bool)].max() > 256.0  # the scaled path ran
    op = oracle_params(p)
    _, wave_of, seq = oracle.schedule(lost.reshape(6, 16, 6, 16).any(axis=(1, 3)).astype(np.uint8))
    errs = np.array([np.abs(np.subtract(*teacher_forced_block(
        img, lost, r.out_f.astype(np.float64), wave_of, op, b // 6, b % 6)[:2])).max()
        for b in seq])
    print(f"[parity] f16x3 bright texture: teacher-forced median {np.median(errs):.3e} "
          f"max {errs.max():.3e} over {len(seq)} blocks", flush=True)
    below_bar_characterization(errs, "FSE_FP32_F16X3 bright texture")


# ------------------------------------------------------------ edge cases

def test_no_losses_is_identity():
    img = np.random.default_rng(0).integers(0, 256, (70, 90)).astype(np.uint8)
    for prec in (fse.FSE_FP64, fse.FSE_FP32):
        r = run_gpu(fse.Params(border_d=14, iterations=20, precision=prec),
                    [img], [np.zeros_like(img)])[0]
        assert r.waves == 0 and r.lost_blocks == 0
        np.testing.assert_array_equal(r.out, img)


def test_everything_lost_uses_empty_fill_then_reconstructed_support():
    img = np.full((48, 64), 77, np.uint8)
    lost = np.ones_like(img)
    p = fse.Params(border_d=8, iterations=10, precision=fse.FSE_FP64, empty_fill=128.0)
    check_free_running(p, img, lost, FP64_TOL)


def test_partial_blocks_grid_shift_and_small_images():
    rng = np.random.default_rng(3)
    for (H, W, goy, gox) in [(37, 53, 0, 0), (37, 53, 5, 11), (9, 7, 0, 0), (20, 33, 15, 1)]:
        img = synth.polygon_image(rng, H, W, radius=(5, 20))
        lost = (rng.random((H, W)) < 0.3).astype(np.uint8)
        p = fse.Params(border_d=12, iterations=25, precision=fse.FSE_FP64,
                       grid_off_x=gox, grid_off_y=goy)
        check_free_running(p, img, lost, FP64_TOL)


def test_border_wider_than_block_uses_wave_snapshots():
    # d > block size: areas of blocks of one wave overlap
    rng = np.random.default_rng(4)
    img = synth.polygon_image(rng, 48, 40, radius=(5, 25))
    lost = synth.bernoulli_block_loss(rng, 48, 40, 4, 0.5)
    for prec, tol, gap in ((fse.FSE_FP64, FP64_TOL, None), (fse.FSE_FP32, None, PSNR_GAP)):
        p = fse.Params(block_w=4, block_h=4, border_d=16, iterations=30, precision=prec)
        check_free_running(p, img, lost, tol, gap)


def test_single_iteration_and_rho_one():
    fr = synth.config2(seed=7, size=64)
    for p in (fse.Params(border_d=14, iterations=1, precision=fse.FSE_FP64),
              fse.Params(border_d=10, iterations=15, rho=1.0, delta=0.0,
                         precision=fse.FSE_FP64)):
        check_free_running(p, fr.image, fr.lost, FP64_TOL)


def test_batch_equals_single_frames(monkeypatch):
    # bit for bit with the workgroup shape pinned (every launch on 4
    # wavefronts): across shapes results agree only to the stated tolerance,
    # and a batch may give its deepest frames a shape of their own
    monkeypatch.setenv("FSE_WAVE_THRESHOLDS", "0,0")
    monkeypatch.setenv("FSE_CRIT_WAVES", "4")
    rng = np.random.default_rng(8)
    frames = []
    for (H, W) in [(64, 80), (45, 33), (96, 64)]:
        img = synth.polygon_image(rng, H, W, radius=(8, 30))
        frames.append((img, synth.slice_loss(rng, H, W, 16, (0.2, 0.4))))
    for prec in (fse.FSE_FP32, fse.FSE_FP64):
        p = fse.Params(border_d=14, iterations=50, precision=prec)
        batch = run_gpu(p, [f[0] for f in frames], [f[1] for f in frames])
        for (img, lost), rb in zip(frames, batch):
            ra = run_gpu(p, [img], [lost])[0]
            np.testing.assert_array_equal(ra.out, rb.out)
            np.testing.assert_array_equal(ra.out_f, rb.out_f)


def test_repeated_runs_are_bitwise_identical():
    fr = synth.config2(seed=9, size=96)
    p = fse.Params(border_d=14, iterations=80, precision=fse.FSE_FP32)
    a = run_gpu(p, [fr.image], [fr.lost])[0]
    b = run_gpu(p, [fr.image], [fr.lost])[0]
    np.testing.assert_array_equal(a.out_f, b.out_f)


# ------------------------------------------------------------ maximum sizes
# The largest area the 64 x 64 basis holds (32 x 32 blocks with d = 16: M =
# N = 64) and the largest iteration count (FSE_MAX_ITERATIONS): the LDS
# layouts at their largest (FP64 on 16 wavefronts: 158.8 KB of 160 KB).

def _max_area_frame(seed, H=96, W=128):
    rng = np.random.default_rng(seed)
    img = synth.polygon_image(rng, H, W, radius=(10, 50))
    lost = np.zeros((H, W), np.uint8)
    lost[5:12, :] = 1          # a strip through the first block row
    lost[32:64, 32:64] = 1     # a whole 32 x 32 block
    lost[40:60, 72:90] = 1     # most of another
    return img, lost


def test_maximum_area_and_iterations_fp64():
    img, lost = _max_area_frame(31)
    p = fse.Params(block_w=32, block_h=32, border_d=16, iterations=fse.FSE_MAX_ITERATIONS,
                   precision=fse.FSE_FP64)
    check_free_running(p, img, lost, FP64_TOL)


def test_maximum_area_and_iterations_rerank():
    img, lost = _max_area_frame(32)
    p = fse.Params(block_w=32, block_h=32, border_d=16, iterations=fse.FSE_MAX_ITERATIONS,
                   precision=fse.FSE_FP32_RERANK)
    r = run_gpu(p, [img], [lost])[0]
    op = oracle_params(p)
    grid = np.zeros((3, 4), np.uint8)
    for b in range(12):
        grid[b // 4, b % 4] = lost[32 * (b // 4):32 * (b // 4) + 32, 32 * (b % 4):32 * (b % 4) + 32].any()
    _, wave_of, seq = oracle.schedule(grid)
    out_f = r.out_f.astype(np.float64)
    with ThreadPoolExecutor(8) as pool:  # the oracle's C calls release the GIL
        errs = list(pool.map(lambda b: float(np.abs(np.subtract(*teacher_forced_block(
            img, lost, out_f, wave_of, op, b // 4, b % 4)[:2])).max()), seq))
    print(f"[parity] re-rank M = N = 64, K = {p.iterations}: teacher-forced max-abs "
          f"{max(errs):.3e} over {len(seq)} blocks", flush=True)
    assert max(errs) <= FP32_TOL


def test_maximum_area_f16x3_first_increment():
    img, lost = _max_area_frame(33)
    p = fse.Params(block_w=32, block_h=32, border_d=16, iterations=1,
                   precision=fse.FSE_FP32_F16X3)
    r = run_gpu(p, [img], [lost], trace=True)[0]
    op = oracle_params(p)
    grid = np.zeros((3, 4), np.uint8)
    for b in range(12):
        grid[b // 4, b % 4] = lost[32 * (b // 4):32 * (b // 4) + 32, 32 * (b % 4):32 * (b % 4) + 32].any()
    _, wave_of, _ = oracle.schedule(grid)
    worst = 0.0
    for slot, b in enumerate(r.trace_block):
        _, _, res = teacher_forced_block(img, lost, r.out_f.astype(np.float64), wave_of, op,
                                         b // 4, b % 4)
        u_o, dc_o = int(res.u[0]), complex(res.dc[0])
        u_g, dc_g = int(r.trace_u[slot][0]), complex(r.trace_dc[slot][0])
        if u_g != u_o:
            assert u_g == int(mirror(u_o)), (b, u_g, u_o)
            dc_o = dc_o.conjugate()
        worst = max(worst, abs(dc_g - dc_o) / abs(dc_o))
    print(f"[parity] f16x3 M = N = 64 first increment: worst relative error {worst:.3e}",
          flush=True)
    assert worst <= F16X3_DC_TOL


# ------------------------------------------------------------ full size

def test_config3_full_batch_sampled_blocks():
    """The 64-frame mixed-resolution batch at K=200 in plain FP32, in one call.
    Properties at full size, and 24 seeded blocks against the oracle fed with
    the exact area each block saw (FSE_FP32 is below the 0.5 bar: the share
    within 0.5 and the median are characterized; the re-rank mode's test
    below holds every block to 0.5)."""
    frames = synth.config3(seed=0)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32)
    res = run_gpu(p, [f.image for f in frames], [f.lost for f in frames])
    op = oracle_params(p)
    rng = np.random.default_rng(0)
    errs = []
    for fi in rng.choice(len(frames), 12, replace=False):
        fr, r = frames[fi], res[fi]
        m = fr.lost.astype(bool)
        np.testing.assert_array_equal(r.out[~m], fr.image[~m])
        assert np.isfinite(r.out_f).all()
        H, W = fr.image.shape
        hb, wb = -(-H // 16), -(-W // 16)
        pad = np.zeros((hb * 16, wb * 16), bool)
        pad[:H, :W] = m
        grid = pad.reshape(hb, 16, wb, 16).any(axis=(1, 3)).astype(np.uint8)
        _, wave_of, seq = oracle.schedule(grid)
        assert r.waves == wave_of.max() + 1
        for b in rng.choice(seq, 2, replace=False):
            o_v, g_v, _ = teacher_forced_block(fr.image, fr.lost, r.out_f.astype(np.float64),
                                               wave_of, op, b // wb, b % wb)
            errs.append(np.abs(o_v - g_v).max())
    errs = np.array(errs)
    print(f"[parity] FP32 full-size teacher-forced: median {np.median(errs):.3e} "
          f"max {errs.max():.3e} within 0.5: {np.mean(errs <= FP32_TOL):.3f}", flush=True)
    below_bar_characterization(errs, "FSE_FP32 full-size batch")


# ------------------------------------------------------------ FP32 + FP64 re-rank

@pytest.mark.parametrize("seed", [5, 11])
def test_rerank_teacher_forced_blocks(seed):
    fr = synth.config2(seed=seed, size=128)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_RERANK)
    r = run_gpu(p, [fr.image], [fr.lost])[0]
    op = oracle_params(p)
    _, wave_of, seq = oracle.schedule(
        fr.lost.reshape(8, 16, 8, 16).any(axis=(1, 3)).astype(np.uint8))
    worst = 0.0
    for b in seq:
        o_v, g_v, _ = teacher_forced_block(fr.image, fr.lost, r.out_f.astype(np.float64),
                                           wave_of, op, b // 8, b % 8)
        worst = max(worst, np.abs(o_v - g_v).max())
    print(f"[parity] FP32+rerank teacher-forced max-abs over {len(seq)} blocks: {worst:.3e}",
          flush=True)
    assert worst <= FP32_TOL, worst


def test_rerank_free_running_and_batch_identity():
    rng = np.random.default_rng(22)
    img = synth.polygon_image(rng, 100, 120, radius=(10, 60))
    lost = synth.bernoulli_block_loss(rng, 100, 120, 16, 0.35)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_RERANK)
    r, _ = check_free_running(p, img, lost, None, PSNR_GAP)
    other = synth.polygon_image(rng, 64, 80, radius=(10, 30))
    olost = synth.slice_loss(rng, 64, 80, 16, (0.2, 0.4))
    rb = run_gpu(p, [other, img], [olost, lost])[1]
    np.testing.assert_array_equal(rb.out_f, r.out_f)


def test_rerank_index_agreement_with_oracle():
    fr = synth.config2(seed=6, size=96)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_RERANK)
    r = run_gpu(p, [fr.image], [fr.lost], trace=True)[0]
    op = oracle_params(p)
    grid = fr.lost.reshape(6, 16, 6, 16).any(axis=(1, 3)).astype(np.uint8)
    _, wave_of, seq = oracle.schedule(grid)
    agrees = []
    for slot, b in enumerate(r.trace_block):
        _, _, res = teacher_forced_block(fr.image, fr.lost, r.out_f.astype(np.float64),
                                         wave_of, op, b // 6, b % 6)
        agree, _ = index_agreement(res.u, r.trace_u[slot])
        agrees.append(agree)
    print(f"[parity] FP32+rerank index agreement: mean {np.mean(agrees):.4f} "
          f"min {np.min(agrees):.4f}", flush=True)
    assert np.mean(agrees) >= 0.95


def test_config3_full_batch_rerank_sampled_blocks():
    """The 64-frame batch at K=200 with FP32 iterations and FP64 re-ranking:
    24 seeded blocks, each fed to the oracle with the exact area it saw, all
    within 0.5 on the 8-bit scale."""
    frames = synth.config3(seed=0)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_RERANK)
    res = run_gpu(p, [f.image for f in frames], [f.lost for f in frames])
    op = oracle_params(p)
    rng = np.random.default_rng(0)
    errs = []
    for fi in rng.choice(len(frames), 12, replace=False):
        fr, r = frames[fi], res[fi]
        m = fr.lost.astype(bool)
        np.testing.assert_array_equal(r.out[~m], fr.image[~m])
        H, W = fr.image.shape
        hb, wb = -(-H // 16), -(-W // 16)
        pad = np.zeros((hb * 16, wb * 16), bool)
        pad[:H, :W] = m
        grid = pad.reshape(hb, 16, wb, 16).any(axis=(1, 3)).astype(np.uint8)
        _, wave_of, seq = oracle.schedule(grid)
        for b in rng.choice(seq, 2, replace=False):
            o_v, g_v, _ = teacher_forced_block(fr.image, fr.lost, r.out_f.astype(np.float64),
                                               wave_of, op, b // wb, b % wb)
            errs.append(np.abs(o_v - g_v).max())
    errs = np.array(errs)
    print(f"[parity] FP32+rerank full-size teacher-forced: median {np.median(errs):.3e} "
          f"max {errs.max():.3e}", flush=True)
    assert errs.max() <= FP32_TOL


def _grid_of(lost, Bh=16, Bw=16):
    H, W = lost.shape
    hb, wb = -(-H // Bh), -(-W // Bw)
    pad = np.zeros((hb * Bh, wb * Bw), bool)
    pad[:H, :W] = lost.astype(bool)
    return pad.reshape(hb, Bh, wb, Bw).any(axis=(1, 3)).astype(np.uint8)


@pytest.mark.parametrize("precision,K,tol", [(fse.FSE_FP32_RERANK, 200, FP32_TOL),
                                             (fse.FSE_FP64, 40, FP64_TOL)])
def test_2160p_frame_sampled_blocks(precision, K, tol):
    """The largest frame of the serving mix (3840 x 2160, slice losses): known
    samples bit for bit, 12 seeded blocks fed to the oracle with the exact
    area each saw."""
    rng = np.random.default_rng(31)
    img = synth.drifting_frame(np.random.default_rng(5), 2160, 3840, 0.0, rng)
    lost = synth.slice_loss(rng, 2160, 3840, 16, (0.04, 0.08))
    p = fse.Params(border_d=14, iterations=K, precision=precision)
    r = run_gpu(p, [img], [lost])[0]
    m = lost.astype(bool)
    np.testing.assert_array_equal(r.out[~m], img[~m])
    grid = _grid_of(lost)
    wb = grid.shape[1]
    _, wave_of, seq = oracle.schedule(grid)
    op = oracle_params(p)
    errs = []
    for b in rng.choice(seq, 12, replace=False):
        o_v, g_v, _ = teacher_forced_block(img, lost, r.out_f.astype(np.float64), wave_of, op,
                                           b // wb, b % wb)
        errs.append(np.abs(o_v - g_v).max())
    print(f"[parity] 2160p prec {precision}: {len(seq)} lost blocks, {r.waves} waves, sampled "
          f"max-abs {max(errs):.3e}", flush=True)
    assert r.waves == int(wave_of.max()) + 1
    assert max(errs) <= tol


@pytest.mark.parametrize("Bh,Bw,d", [(8, 16, 6), (16, 8, 10), (12, 4, 10)])
def test_rectangular_blocks_fp64(Bh, Bw, d):
    """Blocks of unequal height and width (areas of (Bh + 2d) x (Bw + 2d)),
    with d below and above the smaller block side."""
    rng = np.random.default_rng(Bh * 100 + Bw)
    img = synth.polygon_image(rng, 72, 88, radius=(8, 40))
    lost = np.zeros_like(img)
    grid = rng.random((-(-72 // Bh), -(-88 // Bw))) < 0.3
    for i, j in zip(*np.nonzero(grid)):
        lost[i * Bh:(i + 1) * Bh, j * Bw:(j + 1) * Bw] = 1
    p = fse.Params(block_h=Bh, block_w=Bw, border_d=d, iterations=30, precision=fse.FSE_FP64)
    check_free_running(p, img, lost, FP64_TOL)


# ------------------------------------------------------------ launch shapes

SHAPES = {"4 wavefronts": "0,0", "8 wavefronts": "0,1000000", "16 wavefronts": "1000000,0"}


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("precision", [fse.FSE_FP64, fse.FSE_FP32_RERANK, fse.FSE_FP32])
def test_every_launch_shape_matches_oracle(monkeypatch, shape, precision):
    """Each workgroup shape (4, 8 or 16 wavefronts per block, forced for every
    launch) against the oracle: FP64 free-running to 1e-7; FSE_FP32_RERANK
    teacher-forced, every block within 0.5; FSE_FP32 characterized (below
    the bar)."""
    monkeypatch.setenv("FSE_WAVE_THRESHOLDS", SHAPES[shape])
    if precision == fse.FSE_FP64:
        rng = np.random.default_rng(21)
        img = synth.polygon_image(rng, 100, 120, radius=(10, 60))
        lost = synth.bernoulli_block_loss(rng, 100, 120, 16, 0.35)
        p = fse.Params(border_d=14, iterations=60, precision=precision)
        check_free_running(p, img, lost, FP64_TOL)
        return
    fr = synth.config2(seed=5, size=128)
    p = fse.Params(border_d=14, iterations=200, precision=precision)
    r = run_gpu(p, [fr.image], [fr.lost])[0]
    op = oracle_params(p)
    _, wave_of, seq = oracle.schedule(
        fr.lost.reshape(8, 16, 8, 16).any(axis=(1, 3)).astype(np.uint8))
    errs = np.array([np.abs(np.subtract(*teacher_forced_block(
        fr.image, fr.lost, r.out_f.astype(np.float64), wave_of, op, b // 8, b % 8)[:2])).max()
        for b in seq])
    print(f"[parity] {shape} precision {precision}: teacher-forced median "
          f"{np.median(errs):.3e} max {errs.max():.3e} over {len(seq)} blocks", flush=True)
    if precision == fse.FSE_FP32_RERANK:
        assert errs.max() <= FP32_TOL, errs.max()
    else:
        below_bar_characterization(errs, f"{shape} FSE_FP32")


# ------------------------------------------------------------ host buffers

def _conceal_raw(plan, frames):
    """fse_conceal_image through the C ABI with the given fse_frame fields:
    (image, stride, lost, lost_stride, out, out_stride, width, height)."""
    arr = (fse._Frame * len(frames))()
    for c, (img, st, lost, lst, out, ost, W, H) in zip(arr, frames):
        c.image, c.width, c.height, c.stride = img, W, H, st
        c.lost, c.lost_stride, c.out, c.out_stride = lost, lst, out, ost
        c.out_f32 = c.out_f64 = None
        c.trace = None
        c.stats = None
    rc = plan._lib.fse_conceal_image(plan.handle, arr, len(frames))
    assert rc == 0, plan._lib.fse_strerror(rc)


@pytest.mark.parametrize("precision", [fse.FSE_FP32_RERANK, fse.FSE_FP64])
def test_host_strides_and_aliased_output(precision):
    """Host frames with row strides larger than the width (image, mask and
    output each padded differently) and with the output aliasing the input
    give the results of contiguous buffers, bit for bit; padding bytes are
    left untouched."""
    rng = np.random.default_rng(51)
    shapes = [(70, 90), (33, 47), (128, 96)]
    imgs = [synth.polygon_image(rng, H, W, radius=(8, 30)) for H, W in shapes]
    losts = [synth.slice_loss(rng, H, W, 16, (0.2, 0.4)) for H, W in shapes]
    p = fse.Params(border_d=14, iterations=40, precision=precision)
    with fse.Plan(p) as plan:
        ref = plan.fse_conceal_image(imgs, losts)
        # padded strides
        pads = []
        raw = []
        for im, lo in zip(imgs, losts):
            H, W = im.shape
            pi = np.full((H, W + 13), 7, np.uint8); pi[:, :W] = im
            pl = np.full((H, W + 5), 3, np.uint8); pl[:, :W] = lo
            po = np.full((H, W + 29), 201, np.uint8)
            pads.append((pi, pl, po))
            raw.append((pi.ctypes.data, pi.strides[0], pl.ctypes.data, pl.strides[0],
                        po.ctypes.data, po.strides[0], W, H))
        _conceal_raw(plan, raw)
        for (pi, pl, po), r, im in zip(pads, ref, imgs):
            W = im.shape[1]
            np.testing.assert_array_equal(po[:, :W], r.out)
            assert (po[:, W:] == 201).all()
            assert (pi[:, W:] == 7).all() and (pl[:, W:] == 3).all()
        # output aliasing the input image
        alias = [np.ascontiguousarray(im).copy() for im in imgs]
        lcont = [np.ascontiguousarray(lo) for lo in losts]
        raw = [(a.ctypes.data, a.strides[0], lo.ctypes.data, lo.strides[0],
                a.ctypes.data, a.strides[0], a.shape[1], a.shape[0])
               for a, lo in zip(alias, lcont)]
        _conceal_raw(plan, raw)
        for a, r in zip(alias, ref):
            np.testing.assert_array_equal(a, r.out)


# ------------------------------------------------------------ frame groups

@pytest.mark.parametrize("precision", [fse.FSE_FP64, fse.FSE_FP32_RERANK, fse.FSE_FP32,
                                       fse.FSE_FP32_F16X3])
def test_frame_groups_equal_one_group(monkeypatch, precision):
    """A batch split into frame groups on separate streams gives bit for bit
    the results of one group, also with the deepest frames in a group of their
    own (each frame keeps its wave order; the workgroup shape is pinned so
    that all runs use the same kernels)."""
    monkeypatch.setenv("FSE_WAVE_THRESHOLDS", "0,0")
    rng = np.random.default_rng(41)
    frames = []
    for (H, W) in [(96, 128), (64, 80), (130, 70), (48, 48), (112, 96), (80, 160)]:
        img = synth.polygon_image(rng, H, W, radius=(8, 40))
        frames.append((img, synth.slice_loss(rng, H, W, 16, (0.2, 0.5))))
    imgs, losts = [f[0] for f in frames], [f[1] for f in frames]
    p = fse.Params(border_d=14, iterations=60, precision=precision)
    res = {}
    # "4c": the deepest frames in a group of their own with raised wave
    # priority (the schedules here have 2 to 16 waves; 3 frames reach 8)
    for key, groups, crit in (("1", "1", "0"), ("4", "4", "0"), ("4c", "4", "0.5")):
        monkeypatch.setenv("FSE_FRAME_GROUPS", groups)
        monkeypatch.setenv("FSE_CRIT_DEPTH", crit)
        with fse.Plan(p) as plan:
            res[key] = plan.fse_conceal_image(imgs, losts, want_float=True, trace=True)
            assert plan.last_call_stats()["groups"] == int(groups)
    for key in ("4", "4c"):
        for a, b in zip(res["1"], res[key]):
            np.testing.assert_array_equal(a.out_f, b.out_f)
            np.testing.assert_array_equal(a.out, b.out)
            np.testing.assert_array_equal(a.trace_u, b.trace_u)


# ------------------------------------------------------------ single launch

@pytest.mark.skip(reason="the single-launch batch path (one dependency-driven launch with "
                         "per-(frame, wave) completion counters) was taken out of the library: "
                         "its first GPU run of this test did not finish within 180 s, without a "
                         "fault, and no cause was shown by reading the code")
@pytest.mark.parametrize("precision", [fse.FSE_FP64, fse.FSE_FP32_RERANK, fse.FSE_FP32])
def test_single_launch_equals_launch_per_step(monkeypatch, precision):
    """A batch run as one dependency-driven launch gives bit for bit the
    results of one launch per step (the same kernels in the same wave order);
    covers several frames, both orders and the trace."""
    rng = np.random.default_rng(31)
    frames = []
    for (H, W) in [(96, 128), (64, 80), (130, 70), (48, 48)]:
        img = synth.polygon_image(rng, H, W, radius=(8, 40))
        frames.append((img, synth.slice_loss(rng, H, W, 16, (0.2, 0.5))))
    imgs, losts = [f[0] for f in frames], [f[1] for f in frames]
    for order in (fse.FSE_ORDER_OPTIMIZED, fse.FSE_ORDER_LINESCAN):
        p = fse.Params(border_d=14, iterations=60, precision=precision, order=order)
        monkeypatch.setenv("FSE_SINGLE_LAUNCH", "1")
        with fse.Plan(p) as plan:
            one = plan.fse_conceal_image(imgs, losts, want_float=True, trace=True)
            assert plan.last_call_stats()["launches"] == 1
        monkeypatch.setenv("FSE_SINGLE_LAUNCH", "0")
        with fse.Plan(p) as plan:
            per_step = plan.fse_conceal_image(imgs, losts, want_float=True, trace=True)
            assert plan.last_call_stats()["launches"] > 1
        for a, b in zip(one, per_step):
            np.testing.assert_array_equal(a.out_f, b.out_f)
            np.testing.assert_array_equal(a.out, b.out)
            np.testing.assert_array_equal(a.trace_u, b.trace_u)
