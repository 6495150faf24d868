"""fse_conceal_image_noalloc (no allocation: every device buffer of the call is
a slice of the library's fixed scratch) against fse_conceal_image, through
the C ABI, on device frames.

Both plans run one frame group (tuning frame_groups = 1), so both issue the
same launches and the results agree bit for bit.  Two calls in a row, the
second with a smaller input, check that nothing of the first call's scratch
contents leaks into the second; a frame larger than the scratch is rejected
with FSE_ERR_NOMEM before anything runs.
"""
import numpy as np
import pytest

import paper_2207_00233_amd as fse
from paper_2207_00233_amd import synth

pytestmark = pytest.mark.gpu


def _frames(seed, shapes):
    rng = np.random.default_rng(seed)
    return [(synth.polygon_image(rng, H, W, radius=(8, 40)),
             synth.slice_loss(rng, H, W, 16, (0.1, 0.3))) for H, W in shapes]


def _run(torch, plan, frames, noalloc):
    dev = torch.device("cuda:0")
    imgs = [torch.from_numpy(im).to(dev) for im, _ in frames]
    losts = [torch.from_numpy(lo).to(dev) for _, lo in frames]
    outs = [torch.full_like(t, 7) for t in imgs]
    outf = [torch.full(t.shape, -1.0, dtype=torch.float32, device=dev) for t in imgs]
    torch.cuda.synchronize()
    descs = [{"image": i.data_ptr(), "lost": l.data_ptr(), "out": o.data_ptr(),
              "out_f32": f.data_ptr(), "width": i.shape[1], "height": i.shape[0]}
             for i, l, o, f in zip(imgs, losts, outs, outf)]
    (plan.conceal_device_noalloc if noalloc else plan.conceal_device)(descs)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], [f.cpu().numpy() for f in outf]


@pytest.mark.parametrize("precision", [fse.FSE_FP32_RERANK, fse.FSE_FP64, fse.FSE_FP32])
def test_noalloc_equals_conceal_image(precision):
    import torch
    p = fse.Params(border_d=14, iterations=60, precision=precision,
                   flags=fse.FSE_FLAG_DEVICE_PTRS)
    stream = torch.cuda.current_stream().cuda_stream
    big = _frames(1, [(144, 176), (96, 128), (200, 120)])
    small = _frames(2, [(64, 80)])
    with fse.Plan(p, hip_stream=stream) as ref, fse.Plan(p, hip_stream=stream) as na:
        ref.set_tuning(frame_groups=1)
        na.set_tuning(frame_groups=1)
        for frames in (big, small):
            print(f"[gpu] noalloc precision {precision}: {len(frames)} frame(s)", flush=True)
            r_out, r_f = _run(torch, ref, frames, False)
            n_out, n_f = _run(torch, na, frames, True)
            st = na.last_call_stats()
            assert st["blocks"] > 0 and st["groups"] == 1
            for (im, lo), a, b, fa, fb in zip(frames, r_out, n_out, r_f, n_f):
                np.testing.assert_array_equal(a, b)
                np.testing.assert_array_equal(fa, fb)
                m = lo.astype(bool)
                np.testing.assert_array_equal(b[~m], im[~m])


def test_noalloc_rejects_a_frame_larger_than_the_scratch():
    import torch
    p = fse.Params(border_d=14, iterations=10, precision=fse.FSE_FP64,
                   flags=fse.FSE_FLAG_DEVICE_PTRS)
    H = W = 4096  # 8 bytes of working image + 1 of state per pixel: 151 MB
    assert H * W * 9 > fse.FSE_NOALLOC_SCRATCH_BYTES
    dev = torch.device("cuda:0")
    img = torch.zeros((H, W), dtype=torch.uint8, device=dev)
    lost = torch.zeros_like(img)
    lost[:16, :16] = 1
    out = torch.empty_like(img)
    with fse.Plan(p, hip_stream=torch.cuda.current_stream().cuda_stream) as plan:
        with pytest.raises(fse.FseError) as e:
            plan.conceal_device_noalloc([{"image": img.data_ptr(), "lost": lost.data_ptr(),
                                          "out": out.data_ptr(), "width": W, "height": H}])
        assert e.value.code == fse.FSE_ERR_NOMEM
