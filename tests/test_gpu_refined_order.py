"""The refined processing order (FSE_ORDER_REFINED: Algorithm 1 with the
neighbours' unknown samples counted, the alternative criterion Section 3
suggests) on the GPU, against the FP64 oracle running the same order.

Losses mix whole blocks, slices and small partial-block holes, so the refined
order differs from Algorithm 1 on these frames (checked on the oracle).
Bars as in the other parity tests: FP64 1e-7 max-abs free-running with the
oracle's waves; the re-rank mode 0.5 max-abs per block teacher-forced.  The
per-block lost-sample counts come from the host staging loop for host frames,
from the init kernel for device frames and from the submit path for served
frames; all three must give the same schedule and bit-identical outputs.
"""
import numpy as np
import pytest

import oracle
import paper_2207_00233_amd as fse
from paper_2207_00233_amd import synth
from parity import teacher_forced_block

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-7
FP32_TOL = 0.5


def _oracle_params(p, nthreads=8):
    return oracle.Params(block_w=p.block_w, block_h=p.block_h, border_d=p.border_d,
                         fft_w=p.fft_w, fft_h=p.fft_h, rho=p.rho, delta=p.delta,
                         gamma=p.gamma, iterations=p.iterations, order=p.order,
                         empty_fill=p.empty_fill, nthreads=nthreads,
                         grid_off_x=p.grid_off_x, grid_off_y=p.grid_off_y)


def _frame(seed, H=112, W=144):
    """Polygon image with a slice, whole lost blocks and small holes."""
    rng = np.random.default_rng(seed)
    img = synth.polygon_image(rng, H, W, radius=(10, 60))
    lost = synth.slice_loss(rng, H, W, 16, (0.1, 0.15))
    lost |= synth.bernoulli_block_loss(rng, H, W, 16, 0.15)
    for _ in range(12):  # holes of 1..10 x 1..10 samples anywhere
        h, w = rng.integers(1, 11, 2)
        y, x = rng.integers(0, H - h), rng.integers(0, W - w)
        lost[y:y + h, x:x + w] = 1
    return img, lost


def _block_counts(lost, B=16):
    H, W = lost.shape
    hb, wb = -(-H // B), -(-W // B)
    pad = np.zeros((hb * B, wb * B), np.int32)
    pad[:H, :W] = lost != 0
    return pad.reshape(hb, B, wb, B).sum(axis=(1, 3)).astype(np.int32)


def test_frames_order_differently_than_algorithm1():
    for seed in (1, 2):
        _, lost = _frame(seed)
        cnt = _block_counts(lost)
        a = oracle.schedule((cnt > 0).astype(np.uint8))
        b = oracle.schedule_refined(cnt, 256)
        assert not np.array_equal(a[1], b[1]), seed


@pytest.mark.parametrize("seed", [1, 2])
def test_refined_fp64_matches_oracle(seed):
    img, lost = _frame(seed)
    p = fse.Params(border_d=14, iterations=60, precision=fse.FSE_FP64, order=fse.FSE_ORDER_REFINED)
    print(f"[gpu] refined order FP64 seed {seed} {img.shape}", flush=True)
    with fse.Plan(p) as plan:
        r = plan.fse_conceal_image([img], [lost], want_float=True, trace=True)[0]
    o = oracle.conceal(_oracle_params(p), img, lost)
    assert r.waves == o.waves
    wb = o.wave_of.shape[1]
    for slot, b in enumerate(r.trace_block):
        assert r.trace_wave[slot] == o.wave_of[b // wb, b % wb]
    assert len(r.trace_block) == int((o.wave_of >= 0).sum())
    m = lost.astype(bool)
    err = float(np.abs(r.out_f[m] - o.image[m]).max())
    print(f"[parity] refined FP64 max-abs {err:.3e} over {r.waves} waves", flush=True)
    assert err <= FP64_TOL
    np.testing.assert_array_equal(r.out[~m], img[~m])


def test_refined_rerank_teacher_forced_blocks():
    img, lost = _frame(3)
    p = fse.Params(border_d=14, iterations=200, precision=fse.FSE_FP32_RERANK,
                   order=fse.FSE_ORDER_REFINED)
    print(f"[gpu] refined order re-rank {img.shape}", flush=True)
    with fse.Plan(p) as plan:
        r = plan.fse_conceal_image([img], [lost], want_float=True, trace=True)[0]
    op = _oracle_params(p)
    _, wave_of, seq = oracle.schedule_refined(_block_counts(lost), 256)
    assert r.waves == int(wave_of.max()) + 1
    wb = wave_of.shape[1]
    worst = 0.0
    for b in seq:
        o_v, g_v, _ = teacher_forced_block(img, lost, r.out_f.astype(np.float64), wave_of, op,
                                           b // wb, b % wb)
        worst = max(worst, float(np.abs(o_v - g_v).max()))
    print(f"[parity] refined re-rank teacher-forced max-abs {worst:.3e} over {len(seq)} blocks",
          flush=True)
    assert worst <= FP32_TOL


@pytest.mark.parametrize("order", [fse.FSE_ORDER_OPTIMIZED, fse.FSE_ORDER_REFINED])
def test_device_frames_equal_host_frames(order):
    """Device-resident frames (FSE_FLAG_DEVICE_PTRS): the init kernel marks
    the lost blocks (or counts their lost samples for the refined order); the
    result equals the host-frame call bit for bit."""
    import torch
    frames = [_frame(4), _frame(5, 96, 160), _frame(6, 64, 48)]
    p = fse.Params(border_d=14, iterations=60, precision=fse.FSE_FP32, order=order)
    with fse.Plan(p) as plan:
        ref = plan.fse_conceal_image([f[0] for f in frames], [f[1] for f in frames],
                                     want_float=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    imgs = [torch.from_numpy(f[0]).to(dev) for f in frames]
    losts = [torch.from_numpy(f[1]).to(dev) for f in frames]
    outs = [torch.empty_like(t) for t in imgs]
    outf = [torch.empty(t.shape, dtype=torch.float32, device=dev) for t in imgs]
    torch.cuda.synchronize()
    descs = [{"image": i.data_ptr(), "lost": l.data_ptr(), "out": o.data_ptr(),
              "out_f32": of.data_ptr(), "width": i.shape[1], "height": i.shape[0]}
             for i, l, o, of in zip(imgs, losts, outs, outf)]
    pd = fse.Params(border_d=14, iterations=60, precision=fse.FSE_FP32, order=order,
                    flags=fse.FSE_FLAG_DEVICE_PTRS)
    print(f"[gpu] device frames, order {order}", flush=True)
    with fse.Plan(pd, hip_stream=torch.cuda.current_stream().cuda_stream) as plan:
        plan.conceal_device(descs)
        torch.cuda.synchronize()
    for r, o, of in zip(ref, outs, outf):
        np.testing.assert_array_equal(o.cpu().numpy(), r.out)
        np.testing.assert_array_equal(of.cpu().numpy(), r.out_f)


def test_served_refined_frames_equal_batched():
    frames = [_frame(7), _frame(8, 80, 96)]
    p = fse.Params(border_d=14, iterations=60, precision=fse.FSE_FP32,
                   order=fse.FSE_ORDER_REFINED)
    with fse.Plan(p) as plan:
        ref = [plan.fse_conceal_image([im], [ls], want_float=True)[0] for im, ls in frames]
    print("[serve] refined order, 2 frames", flush=True)
    with fse.Plan(p) as plan:
        tickets = [plan.fse_submit(im, ls, want_float=True) for im, ls in frames]
        res = [plan.fse_poll(t, timeout_us=-1) for t in tickets]
    for (im, ls), r, a in zip(frames, res, ref):
        np.testing.assert_array_equal(r.out, a.out)
        np.testing.assert_array_equal(r.out_f, a.out_f)
        assert r.waves == a.waves == oracle.schedule_refined(_block_counts(ls), 256)[0]


@pytest.mark.parametrize("shape,off", [((70, 90), (5, 11)), ((45, 130), (15, 0))])
def test_refined_grid_offsets_and_ragged_edges(shape, off):
    """Blocks partly outside the image (grid shifted, sizes not multiples of
    16): the counts cover the in-image samples only, outside cells count a
    whole block; host frames, device frames and the oracle agree (FP64)."""
    import torch
    H, W = shape
    rng = np.random.default_rng(9)
    img = synth.polygon_image(rng, H, W, radius=(8, 40))
    lost = np.maximum(synth.hole_loss(rng, H, W, 20),
                      synth.bernoulli_block_loss(rng, H, W, 16, 0.2))
    p = fse.Params(border_d=12, iterations=40, precision=fse.FSE_FP64,
                   order=fse.FSE_ORDER_REFINED, grid_off_x=off[0], grid_off_y=off[1])
    print(f"[gpu] refined order {shape} offsets {off}", flush=True)
    with fse.Plan(p) as plan:
        r = plan.fse_conceal_image([img], [lost], want_float=True)[0]
    o = oracle.conceal(_oracle_params(p), img, lost)
    m = lost.astype(bool)
    assert r.waves == o.waves
    assert float(np.abs(r.out_f[m] - o.image[m]).max()) <= FP64_TOL
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ti, tl = torch.from_numpy(img).to(dev), torch.from_numpy(lost).to(dev)
    to = torch.empty_like(ti)
    tf = torch.empty((H, W), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    pd = fse.Params(border_d=12, iterations=40, precision=fse.FSE_FP64,
                    order=fse.FSE_ORDER_REFINED, grid_off_x=off[0], grid_off_y=off[1],
                    flags=fse.FSE_FLAG_DEVICE_PTRS)
    with fse.Plan(pd, hip_stream=torch.cuda.current_stream().cuda_stream) as plan:
        plan.conceal_device([{"image": ti.data_ptr(), "lost": tl.data_ptr(), "out": to.data_ptr(),
                              "out_f64": tf.data_ptr(), "width": W, "height": H}])
        torch.cuda.synchronize()
    np.testing.assert_array_equal(to.cpu().numpy(), r.out)
    np.testing.assert_array_equal(tf.cpu().numpy(), r.out_f)


@pytest.mark.parametrize("precision,tol", [(fse.FSE_FP64, FP64_TOL * 255),
                                           (fse.FSE_FP32_RERANK, FP32_TOL)])
def test_refined_full_size_holes_sampled_blocks(precision, tol):
    """The refined-order experiment's own input at its full size: a 512 x 512
    polygon image with 300 unaligned holes of 1..12 x 1..12 samples plus
    isolated 16 x 16 losses (p = 0.12), d = 16, K = 200.  The GPU runs the
    whole frame; blocks sampled from the first, middle and last waves are
    teacher-forced against the oracle (the area each one read is rebuilt
    from the GPU's final image and the oracle's schedule)."""
    rng = np.random.default_rng(0)
    img = synth.polygon_image(rng, 512, 512)
    lost = np.maximum(synth.hole_loss(rng, 512, 512, 300),
                      synth.isolated_block_loss(rng, 512, 512, 16, 0.12))
    p = fse.Params(border_d=16, iterations=200, precision=precision, order=fse.FSE_ORDER_REFINED)
    print(f"[gpu] refined order 512x512 holes prec={precision}", flush=True)
    with fse.Plan(p) as plan:
        r = plan.fse_conceal_image([img], [lost], want_float=True)[0]
    op = _oracle_params(p)
    _, wave_of, seq = oracle.schedule_refined(_block_counts(lost), 256)
    assert r.waves == int(wave_of.max()) + 1
    wb = wave_of.shape[1]
    picks = list(seq[:4]) + list(np.random.default_rng(1).choice(seq, 6, replace=False)) + list(seq[-4:])
    worst = 0.0
    for b in picks:
        o_v, g_v, _ = teacher_forced_block(img, lost, r.out_f.astype(np.float64), wave_of, op,
                                           b // wb, b % wb)
        worst = max(worst, float(np.abs(o_v - g_v).max()))
    print(f"[parity] refined 512x512 prec={precision}: worst {worst:.3e} over {len(picks)} blocks",
          flush=True)
    assert worst <= tol
