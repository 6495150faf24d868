"""Benchmark: lost blocks extrapolated per second at K = 200.

Workload: the 64-frame mixed-resolution batch (16 frames each of 352x288,
704x576, 1280x720 and 1920x1080, polygon textures, 5-30 % slice losses,
16x16 blocks, d = 14, 64x64 DFT basis, K = 200), FP32 iterations, all frames
of a wave in one launch, inputs and outputs resident in device memory.  One
step = one fse_conceal_image call over the whole batch.  Also reported: the
same batch in the plain FP64 form (one frame per call), the roofline of the
fused block kernel, and the FP64 CPU oracle on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

K_ITER = 200
BORDER = 14
BLOCK = 16
# Algorithmic work per lost block (flops): per iteration and spectrum entry the
# update R -= dc * W[k-u] (4 FMA = 8 flop) and |R|^2 (3 flop), 4096 entries;
# two real 64x64 transforms at FFT cost (2 * 2.5 * 4096 * log2(4096) flop);
# the synthesis on 16x16 lost samples (4 flop per sample and iteration).
ITER_FLOPS = 11 * 4096 * K_ITER
TRANSFORM_FLOPS = 2 * 2.5 * 4096 * 12
SYNTH_FLOPS = 256 * K_ITER * 4
FLOPS_PER_BLOCK = ITER_FLOPS + TRANSFORM_FLOPS + SYNTH_FLOPS
PEAK_FP32_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (non-packed FMA)
PEAK_FP32_PUBLISHED = 157.3  # MI355X's published FP32 vector peak (packed FP32)
# The method's own HBM bytes per lost block: the 44 x 44 area read (float
# sample + state byte) and the 16 x 16 block written back (float + state).
ALG_HBM_BYTES_PER_BLOCK = (BLOCK + 2 * BORDER) ** 2 * 5 + BLOCK * BLOCK * 5
# LDS bytes of the shifted read of W per lost block: K iterations x 4096
# entries x 8 bytes (float complex)
LDS_BYTES_PER_BLOCK = K_ITER * 4096 * 8
# whether a precision mode meets the parity bar (0.5 max-abs on every block,
# teacher-forced; tests/test_gpu_precision_sweep.py)
MEETS_BAR = {"fp64": True, "fp32_rerank": True, "fp32": False, "fp32_f16x3": False}
SIMDS = 256 * 4            # compute units x SIMDs
CLOCK_HZ = 2.4e9


# sources whose change invalidates a committed traffic measurement: the
# kernels and the host code that chooses their launches
TRAFFIC_SOURCES = ("paper_2207_00233_amd/csrc/fse_kernels.hip", "paper_2207_00233_amd/csrc/fse_device.h",
                   "paper_2207_00233_amd/csrc/fse_dft.h",
                   "paper_2207_00233_amd/csrc/fse_runtime.cpp", "paper_2207_00233_amd/csrc/fse_internal.h")


def measured_record(precision):
    """The committed rocprofv3 counter record of the block kernel over one
    step (HBM bytes from FETCH_SIZE/WRITE_SIZE, VALU wavefront-instructions
    from SQ_INSTS_VALU), if it was taken on this kernel source, launch
    configuration (host runtime) and precision; None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "fse_block_kernel_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for fn in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, fn), "rb").read())
    if rec.get("precision") != precision or rec.get("kernel_source_sha256") != h.hexdigest():
        return None
    return rec


def measured_traffic(precision):
    """HBM bytes of the block kernel per launch (see measured_record), or None."""
    rec = measured_record(precision)
    return rec["traffic_bytes_per_launch"] if rec else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(frames, budget_s=15.0):
    """The FP64 oracle on whole frames of the batch (smallest first), all host
    cores, until about ``budget_s`` seconds of work are done."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    p = oracle.Params(border_d=BORDER, iterations=K_ITER, nthreads=cores)
    order = sorted(range(len(frames)), key=lambda i: frames[i].image.size)
    blocks = 0
    used = []
    t0 = time.perf_counter()
    for i in order:
        fr = frames[i]
        H, W = fr.image.shape
        hb, wb = -(-H // BLOCK), -(-W // BLOCK)
        pad = np.zeros((hb * BLOCK, wb * BLOCK), bool)
        pad[:H, :W] = fr.lost.astype(bool)
        nb = int(pad.reshape(hb, BLOCK, wb, BLOCK).any(axis=(1, 3)).sum())
        oracle.conceal(p, fr.image, fr.lost)
        blocks += nb
        used.append(f"{W}x{H}")
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": blocks / dt, "unit": "lost blocks/s", "cores": cores, "kind": "oracle",
            "cpu_model": model,
            "sample": f"{len(used)} whole frames of the batch ({', '.join(sorted(set(used)))}), "
                      f"{blocks} lost blocks, {dt:.1f} s, FP64, K={K_ITER}"}


def psnr_lost(out, ref, lost):
    m = lost.astype(bool)
    mse = np.mean((out[m].astype(np.float64) - ref[m].astype(np.float64)) ** 2)
    return float(10 * np.log10(255.0 ** 2 / mse)) if mse > 0 else float("inf")


def order_frames(synth, seeds=(0, 1, 2)):
    return [synth.config2(seed=s) for s in seeds]


def order_comparison_gpu(fse, frames, precision, reps=3):
    """512x512 polygon images with 16x16 blocks lost i.i.d. (p = 0.25), the
    optimized order (Algorithm 1) against the line scan on the GPU: PSNR on the
    lost samples against the ground truth, number of waves, lost blocks per
    second and wall time per frame (host buffers, one frame per call)."""
    res = {}
    for name, order in (("optimized", fse.FSE_ORDER_OPTIMIZED), ("line_scan", fse.FSE_ORDER_LINESCAN)):
        p = fse.Params(border_d=BORDER, iterations=K_ITER, precision=precision, order=order)
        with fse.Plan(p) as plan:
            psnrs, waves, blocks, times = [], [], 0, []
            for fr in frames:
                plan.fse_conceal_image([fr.image], [fr.lost])
                for _ in range(reps):
                    t0 = time.perf_counter()
                    r = plan.fse_conceal_image([fr.image], [fr.lost])[0]
                    times.append(time.perf_counter() - t0)
                psnrs.append(psnr_lost(r.out, fr.image, fr.lost))
                waves.append(r.waves)
                blocks += r.lost_blocks
        res[name] = {"psnr_db": psnrs, "mean_psnr_db": float(np.mean(psnrs)), "waves": waves,
                     "ms_per_frame": float(np.median(times) * 1e3),
                     "lost_blocks_per_s": blocks / (np.median(times) * len(frames))}
    res["gain_db"] = res["optimized"]["mean_psnr_db"] - res["line_scan"]["mean_psnr_db"]
    return res


def subblock_order_gpu(fse, synth, precision, size=512, seeds=(0, 1, 2, 3),
                       blocks=(16, 8, 4, 2)):
    """The paper's order experiment: 16-sample isolated, consecutive and mixed
    losses, each processed with blocks of 16, 8, 4 or 2 samples (d = 16, so
    blocks smaller than the border read their wave's snapshot), optimized
    order against line scan; PSNR on the lost samples per image and the mean
    gain over the images (GPU)."""
    res = {}
    for pname in ("isolated", "consecutive", "mixed"):
        rows = {f"{b}x{b}": {"gain_db": [], "line_scan_db": [], "optimized_db": [],
                             "waves": [], "line_scan_waves": []} for b in blocks}
        for seed in seeds:
            rng = np.random.default_rng(seed)
            img = synth.polygon_image(rng, size, size)
            lost = {"isolated": lambda: synth.isolated_block_loss(rng, size, size, 16, 0.25),
                    "consecutive": lambda: synth.consecutive_loss(rng, size, size),
                    "mixed": lambda: synth.mixed_loss(rng, size, size)}[pname]()
            for b in blocks:
                r = {}
                for oname, order in (("line_scan", fse.FSE_ORDER_LINESCAN),
                                     ("optimized", fse.FSE_ORDER_OPTIMIZED)):
                    p = fse.Params(block_w=b, block_h=b, border_d=16, iterations=K_ITER,
                                   precision=precision, order=order)
                    with fse.Plan(p) as plan:
                        out = plan.fse_conceal_image([img], [lost])[0]
                    r[oname] = (psnr_lost(out.out, img, lost), out.waves)
                row = rows[f"{b}x{b}"]
                row["line_scan_db"].append(r["line_scan"][0])
                row["optimized_db"].append(r["optimized"][0])
                row["gain_db"].append(r["optimized"][0] - r["line_scan"][0])
                row["waves"].append(r["optimized"][1])
                row["line_scan_waves"].append(r["line_scan"][1])
        for row in rows.values():
            row["mean_gain_db"] = float(np.mean(row["gain_db"]))
        res[pname] = rows
    return res


def refined_order_gpu(fse, synth, precision, size=512, seeds=(0, 1, 2, 3)):
    """The refined criterion (neighbours' unknown samples counted) against
    Algorithm 1 and the line scan, on losses that leave blocks partly known:
    "holes" = 300 unaligned holes of 1..12 x 1..12 samples plus isolated 16 x
    16 losses; "mixed_shifted" = the paper's mixed pattern with the 16 x 16
    block grid shifted by 8 samples both ways, so every lost block is partly
    known.  PSNR on the lost samples and waves per image (d = 16, GPU)."""
    res = {}
    for pname in ("holes", "mixed_shifted"):
        row = {o: {"psnr_db": [], "waves": []} for o in ("line_scan", "optimized", "refined")}
        for seed in seeds:
            rng = np.random.default_rng(seed)
            img = synth.polygon_image(rng, size, size)
            if pname == "holes":
                lost = np.maximum(synth.hole_loss(rng, size, size, 300),
                                  synth.isolated_block_loss(rng, size, size, 16, 0.12))
                off = 0
            else:
                lost = synth.mixed_loss(rng, size, size)
                off = 8
            for oname, order in (("line_scan", fse.FSE_ORDER_LINESCAN),
                                 ("optimized", fse.FSE_ORDER_OPTIMIZED),
                                 ("refined", fse.FSE_ORDER_REFINED)):
                p = fse.Params(border_d=16, iterations=K_ITER, precision=precision, order=order,
                               grid_off_x=off, grid_off_y=off)
                with fse.Plan(p) as plan:
                    out = plan.fse_conceal_image([img], [lost])[0]
                row[oname]["psnr_db"].append(psnr_lost(out.out, img, lost))
                row[oname]["waves"].append(out.waves)
        for v in row.values():
            v["mean_psnr_db"] = float(np.mean(v["psnr_db"]))
            v["mean_waves"] = float(np.mean(v["waves"]))
        row["refined_vs_optimized_db"] = (row["refined"]["mean_psnr_db"]
                                          - row["optimized"]["mean_psnr_db"])
        row["optimized_vs_line_scan_db"] = (row["optimized"]["mean_psnr_db"]
                                            - row["line_scan"]["mean_psnr_db"])
        res[pname] = row
    return res


def order_comparison_oracle(frames):
    """The same comparison computed by the FP64 oracle on all host cores
    (threads over the blocks of a wave, as in the paper's Section 3).  The
    line scan has one block per wave, so it runs on one core; the ratio of
    the two times is the paper's parallelization gain (its Fig. 4: up to 7.7
    on 8 cores) on this host."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    res = {}
    for name, order in (("optimized", 0), ("line_scan", 1)):
        p = oracle.Params(border_d=BORDER, iterations=K_ITER, nthreads=cores, order=order)
        psnrs, waves, dt = [], [], 0.0
        for fr in frames:
            t0 = time.perf_counter()
            o = oracle.conceal(p, fr.image, fr.lost)
            dt += time.perf_counter() - t0
            q = np.where(fr.lost.astype(bool), np.clip(np.rint(o.image), 0, 255), fr.image)
            psnrs.append(psnr_lost(q.astype(np.uint8), fr.image, fr.lost))
            waves.append(int(o.waves))
        res[name] = {"psnr_db": psnrs, "mean_psnr_db": float(np.mean(psnrs)), "waves": waves,
                     "s_per_frame": dt / len(frames)}
    res["gain_db"] = res["optimized"]["mean_psnr_db"] - res["line_scan"]["mean_psnr_db"]
    res["parallelization_gain"] = res["line_scan"]["s_per_frame"] / res["optimized"]["s_per_frame"]
    res["cores"] = cores
    return res


def end_to_end(fse, frames, precision, steps=2):
    """The 64-frame batch from and to host memory (PCIe copies included)."""
    p = fse.Params(border_d=BORDER, iterations=K_ITER, precision=precision)
    imgs = [f.image for f in frames]
    losts = [f.lost for f in frames]
    with fse.Plan(p) as plan:
        plan.fse_conceal_image(imgs, losts)
        blocks = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            res = plan.fse_conceal_image(imgs, losts)
            blocks += sum(r.lost_blocks for r in res)
        dt = time.perf_counter() - t0
    return {"value": blocks / dt, "unit": "lost blocks/s", "ms_per_step": dt / steps * 1e3,
            "form": "host uint8 frames in, host uint8 frames out, one call per step"}


def volume_run(fse, synth, frames=16, height=720, width=1280, p_loss=0.1, K=100, reps=3):
    """Three-dimensional FSE (FP64) of a 720p video volume of 16 frames with
    16 x 16 blocks of every frame lost i.i.d. with p = 0.1: blocks of one
    frame, areas over 2 frames before and after and 8 samples around, the
    8 x 32 x 32 basis grid, K = 100.  Device time per call from the
    library's events (host copies excluded) and wall time per call."""
    v = synth.video_volume(seed=0, frames=frames, height=height, width=width, p=p_loss)
    p = fse.Params3(iterations=K)
    dev_ms, wall_ms = [], []
    with fse.Plan3(p) as plan:
        plan.conceal_volume(v.volume, v.lost)
        for _ in range(reps):
            t0 = time.perf_counter()
            r = plan.conceal_volume(v.volume, v.lost)
            wall_ms.append((time.perf_counter() - t0) * 1e3)
            dev_ms.append(r.latency_ms)
    best = min(dev_ms)
    return {"value": r.lost_blocks / (best * 1e-3), "unit": "lost blocks/s",
            "device_ms": best, "wall_ms": min(wall_ms), "lost_blocks": r.lost_blocks,
            "waves": r.waves, "max_wave_blocks": r.max_wave_blocks,
            "workload": f"{frames} frames {width}x{height}, 16x16x1 blocks lost i.i.d. "
                        f"p = {p_loss}, border 2 frames / 8 samples, 8x32x32 grid, "
                        f"K = {K}, FP64"}


def serving_run(fse, synth, duration_s=10.0, warmup_s=1.0, rate_hz=240.0, seed=0,
                precision=None):
    """Poisson stream of drifting-texture frames (30 % 1280x720, 50 % 1920x1080,
    20 % 3840x2160, 2-15 % slice losses) submitted in real time for
    warmup_s + duration_s seconds; the frames are drawn from a pre-generated
    pool (12 drifting frames per resolution, 6 at 2160p, each arrival pairing
    one of them with one of 16 loss masks) so that generation does not pace
    the stream.  Latency is the library's submit -> result-on-host time."""
    import threading
    rng = np.random.default_rng(seed)
    scene = int(rng.integers(0, 2**31 - 1))
    pool = {}
    for (w, h), _ in synth.SERVING_MIX:
        n = 6 if w >= 3840 else 12
        imgs = [synth.drifting_frame(np.random.default_rng(scene), h, w, i / rate_hz, rng)
                for i in range(n)]
        masks = [synth.slice_loss(rng, h, w, BLOCK, (0.02, 0.15)) for _ in range(16)]
        pool[(w, h)] = (imgs, masks)
    sizes = [m[0] for m in synth.SERVING_MIX]
    probs = np.array([m[1] for m in synth.SERVING_MIX])
    total_s = warmup_s + duration_s
    arrivals, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= total_s:
            break
        imgs, masks = pool[sizes[int(rng.choice(len(sizes), p=probs))]]
        arrivals.append((t, (imgs[int(rng.integers(len(imgs)))],
                             masks[int(rng.integers(len(masks)))])))
    p = fse.Params(border_d=BORDER, iterations=K_ITER,
                   precision=fse.FSE_FP32_RERANK if precision is None else precision,
                   device_mem_budget=16 << 30, max_inflight_frames=256)
    plan = fse.Plan(p)
    tickets = []
    lock = threading.Lock()
    start = time.perf_counter()

    def submitter():
        for (ta, (img, lost)) in arrivals:
            delay = start + ta - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tk = plan.fse_submit(img, lost)
            with lock:
                tickets.append((tk, ta))

    th = threading.Thread(target=submitter)
    th.start()
    results = []
    i = 0
    while True:
        with lock:
            have = i < len(tickets)
            item = tickets[i] if have else None
        if not have:
            if not th.is_alive() and i >= len(tickets):
                break
            time.sleep(0.0005)
            continue
        r = plan.fse_poll(item[0], timeout_us=-1)
        results.append((item[1], r.latency_ms, r.lost_blocks, time.perf_counter() - start))
        i += 1
    th.join()
    plan.close()
    win = [x for x in results if x[0] >= warmup_s]
    lat = np.array([x[1] for x in win])
    done_blocks = sum(x[2] for x in win)
    t_end = max(x[3] for x in win)
    return {"frames": len(win), "rate_hz": rate_hz, "window_s": duration_s,
            "p50_frame_latency_ms": float(np.percentile(lat, 50)),
            "p99_frame_latency_ms": float(np.percentile(lat, 99)),
            "max_frame_latency_ms": float(lat.max()),
            "sustained_lost_blocks_per_s": done_blocks / (t_end - warmup_s),
            "offered_lost_blocks_per_s": done_blocks / duration_s,
            "precision": {fse.FSE_FP32: "fp32", fse.FSE_FP32_RERANK: "fp32_rerank",
                          fse.FSE_FP64: "fp64", fse.FSE_FP32_F16X3: "fp32_f16x3"}[p.precision],
            "mix": "30% 1280x720, 50% 1920x1080, 20% 3840x2160; 2-15% slice losses; K=200"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-order", action="store_true")
    ap.add_argument("--no-e2e", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--precision", choices=("fp32", "fp32_rerank", "fp32_f16x3"), default="fp32_rerank",
                    help="arithmetic of the headline batched run")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--hw-queues", type=int, default=8, choices=range(1, 33), metavar="1..32",
                    help="GPU_MAX_HW_QUEUES for this process (default 8)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device copy 3 times (HBM counter scale)")
    args = ap.parse_args()
    # hardware queues per process (HIP's default is 4): with 8 the re-rank
    # mode's frame groups take four streams besides the caller's; set before
    # anything initializes HIP
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(frames would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        src = torch.ones(512 << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel(), "copies": 3}), flush=True)
        return

    import paper_2207_00233_amd as fse
    from paper_2207_00233_amd import synth

    log("[bench] generating the 64-frame batch")
    frames = synth.config3(seed=args.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    imgs = [torch.from_numpy(f.image).to(dev) for f in frames]
    losts = [torch.from_numpy(f.lost).to(dev) for f in frames]
    outs = [torch.empty_like(t) for t in imgs]
    torch.cuda.synchronize()
    descs = [{"image": i.data_ptr(), "lost": l.data_ptr(), "out": o.data_ptr(),
              "width": i.shape[1], "height": i.shape[0]} for i, l, o in zip(imgs, losts, outs)]
    batch = fse.DeviceFrames(descs)  # the fse_frame array of the batch, built once
    stream = torch.cuda.current_stream().cuda_stream

    names = {fse.FSE_FP32: "fp32", fse.FSE_FP32_RERANK: "fp32_rerank", fse.FSE_FP64: "fp64",
             fse.FSE_FP32_F16X3: "fp32_f16x3"}

    def batched(precision, steps, warmup):
        p = fse.Params(border_d=BORDER, iterations=K_ITER, precision=precision,
                       flags=fse.FSE_FLAG_DEVICE_PTRS)
        plan = fse.Plan(p, hip_stream=stream)
        for _ in range(warmup):
            plan.conceal_device(batch)
        torch.cuda.synchronize()
        kms, busy, launches, blocks, rescored = 0.0, 0.0, 0, 0, 0
        step_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            plan.conceal_device(batch)  # synchronous: returns with the step done
            step_ms.append((time.perf_counter() - ts) * 1e3)
            cs = plan.last_call_stats()
            kms += cs["kernel_ms"]
            busy += cs["busy_ms"]
            launches += cs["launches"]
            blocks += cs["blocks"]
            rescored += cs["rescored"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plan.close()
        return {"value": blocks / dt, "ms_per_step": dt / steps * 1e3,
                "median_ms_per_step": float(np.median(step_ms)),
                "meets_parity_bar": MEETS_BAR[names[precision]],
                "rescored_iterations_per_step": rescored // steps,
                "kernel_ms_per_step": kms / steps,
                "kernel_busy_ms_per_step": busy / steps, "groups": cs["groups"],
                "launches_per_step": launches // steps,
                "blocks_per_step": blocks // steps, "avg_launch_ms": kms / max(1, launches),
                "blocks_per_launch": blocks / max(1, launches)}

    head_prec = {"fp32": fse.FSE_FP32, "fp32_rerank": fse.FSE_FP32_RERANK,
                 "fp32_f16x3": fse.FSE_FP32_F16X3}[args.precision]
    log(f"[bench] batched {args.precision}: {args.steps} timed steps")
    head = batched(head_prec, args.steps, args.warmup)
    log(f"[bench] batched {args.precision}: {head['value']:.0f} blocks/s, "
        f"{head['ms_per_step']:.1f} ms/step, kernel {head['kernel_ms_per_step']:.1f} ms/step")
    sweep = {names[head_prec]: head}
    if not args.no_sweep:
        for prec in (fse.FSE_FP32, fse.FSE_FP32_RERANK, fse.FSE_FP64, fse.FSE_FP32_F16X3):
            if prec == head_prec:
                continue
            r = batched(prec, 2, 1)
            sweep[names[prec]] = r
            log(f"[bench] batched {names[prec]}: {r['value']:.0f} blocks/s")
    value = head["value"]
    dt = head["ms_per_step"] * args.steps / 1e3
    lost_blocks = head["blocks_per_step"]
    launches = head["launches_per_step"] * args.steps
    avg_launch_ms = head["avg_launch_ms"]
    blocks_per_launch = head["blocks_per_launch"]
    # the dominant kernel is the per-block iteration kernel; in the re-rank
    # mode the transforms run in a separate FP64 pass
    kflops = (ITER_FLOPS + SYNTH_FLOPS if args.precision == "fp32_rerank"
              else FLOPS_PER_BLOCK)
    # launches of different frame groups overlap: the kernel's flops over the
    # time at least one of its launches ran (union of the launch intervals)
    # the frame groups' launches overlap, so a launch's duration includes the
    # time it shares the GPU: achieved = the step's flops over the union of
    # the kernel's launch intervals (HIP events on the launches' own streams);
    # beside it the per-launch figure: the flops of the blocks one launch
    # processes on average over the average launch duration
    busy_ms = head["kernel_busy_ms_per_step"]
    achieved = kflops * lost_blocks / (busy_ms * 1e-3) / 1e12
    achieved_launch = kflops * blocks_per_launch / (avg_launch_ms * 1e-3) / 1e12
    traffic = measured_traffic(args.precision)
    alg_bytes_launch = ALG_HBM_BYTES_PER_BLOCK * blocks_per_launch
    # the shifted read of W is the iteration's LDS traffic: 8 bytes (float
    # complex) per spectrum entry and iteration
    lds_tbps = LDS_BYTES_PER_BLOCK * lost_blocks / (busy_ms * 1e-3) / 1e12
    peaks = None
    if not args.no_peaks:
        log("[bench] measured peaks (FMA, LDS, HBM microbenchmarks)")
        peaks = fse.measure_peaks()
        log(f"[bench] peaks: FP32 FMA {peaks['fp32_fma_tflops']:.1f} TFLOP/s, FP64 FMA "
            f"{peaks['fp64_fma_tflops']:.1f}, LDS {peaks['lds_read_tbps']:.1f} TB/s, HBM copy "
            f"{peaks['hbm_copy_tbps']:.2f} TB/s")
    # VALU issue: the committed SQ_INSTS_VALU count of a step over the
    # kernel's busy time, against what 1024 SIMDs issue (a wave64 VALU
    # instruction occupies a 16-lane SIMD for 4 cycles)
    rec = measured_record(args.precision)
    valu = rec.get("valu_wave_insts_per_step") if rec else None
    valu_issue_frac = (valu / (busy_ms * 1e-3) / (SIMDS * CLOCK_HZ / 4.0)) if valu else None

    fp64 = None
    if not args.no_fp64:
        p64 = fse.Params(border_d=BORDER, iterations=K_ITER, precision=fse.FSE_FP64,
                         flags=fse.FSE_FLAG_DEVICE_PTRS)
        plan64 = fse.Plan(p64, hip_stream=stream)
        plan64.conceal_device(descs[:1])
        torch.cuda.synchronize()
        log("[bench] FP64 plain: one frame per call")
        t0 = time.perf_counter()
        lat = []
        for d in descs:
            t1 = time.perf_counter()
            plan64.conceal_device([d])
            lat.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        plan64.close()
        fp64 = {"value": lost_blocks / dt64, "unit": "lost blocks/s",
                "p50_frame_latency_ms": float(np.percentile(lat, 50)),
                "p99_frame_latency_ms": float(np.percentile(lat, 99)),
                "form": "FP64, one frame per call, one launch per wave"}
        log(f"[bench] FP64 plain: {fp64['value']:.0f} blocks/s")

    serving = None
    if not args.no_serving:
        log("[bench] serving: Poisson 240 frames/s")
        serving = serving_run(fse, synth)
        log(f"[bench] serving: p50 {serving['p50_frame_latency_ms']:.1f} ms, "
            f"p99 {serving['p99_frame_latency_ms']:.1f} ms over {serving['frames']} frames")

    volume = None
    if not args.no_volume:
        log("[bench] three-dimensional FSE, 720p video volume")
        volume = volume_run(fse, synth)
        log(f"[bench] 3-D: {volume['value']:.0f} lost blocks/s, {volume['device_ms']:.1f} ms "
            f"device, {volume['waves']} waves")

    e2e = None
    if not args.no_e2e:
        log("[bench] end to end from host memory")
        e2e = end_to_end(fse, frames, head_prec)
        log(f"[bench] end to end: {e2e['value']:.0f} blocks/s")

    order = None
    if not args.no_order:
        log("[bench] order comparison (512x512, p = 0.25)")
        oframes = order_frames(synth)
        order = {"gpu": order_comparison_gpu(fse, oframes, head_prec)}
        log(f"[bench] order comparison: gain {order['gpu']['gain_db']:.3f} dB (GPU)")
        log("[bench] order comparison with sub-blocks (isolated / consecutive / mixed)")
        order["subblocks"] = subblock_order_gpu(fse, synth, head_prec)
        for pn, v in order["subblocks"].items():
            log(f"[bench]   {pn}: " + ", ".join(f"{b} {r['mean_gain_db']:+.2f} dB"
                                              for b, r in v.items()))
        log("[bench] refined ordering criterion (partly known blocks)")
        order["refined"] = refined_order_gpu(fse, synth, head_prec)
        for pn, v in order["refined"].items():
            log(f"[bench]   {pn}: refined - optimized {v['refined_vs_optimized_db']:+.3f} dB, "
                f"waves {v['line_scan']['mean_waves']:.0f} / {v['optimized']['mean_waves']:.0f} / "
                f"{v['refined']['mean_waves']:.0f} (line scan / optimized / refined)")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(frames)
        if order is not None:
            # part of the CPU baseline leg: the oracle's order comparison (its
            # line scan is sequential, so one 256x256 frame), with the GPU
            # result on the same frame under order["gpu_256"]
            small = [synth.config2(seed=0, size=256)]
            cpu["order_comparison_256"] = {"frames": "one 256x256 frame (seed 0), p = 0.25",
                                           **order_comparison_oracle(small)}
            order["gpu_256"] = order_comparison_gpu(fse, small, head_prec, reps=1)
            oc = cpu["order_comparison_256"]
            log(f"[bench] order comparison: gain {oc['gain_db']:.3f} dB (oracle), "
                f"{order['gpu_256']['gain_db']:.3f} dB (GPU), 256x256; oracle parallelization "
                f"gain {oc['parallelization_gain']:.2f} on {oc['cores']} cores")

    line = {
        "metric": "lost blocks extrapolated/s (K=200) + p99 frame latency, FP32 batched vs FP64 plain",
        "value": value,
        "unit": "lost blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "median_ms_per_step": head["median_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision": args.precision,
        "data": "synthetic",
        "config": {"workload": "64 mixed-resolution frames (16 each 352x288, 704x576, "
                               "1280x720, 1920x1080), 5-30% slice losses, 16x16 blocks, "
                               "d=14, 64x64 DFT basis, K=200, FP32 iterations batched"
                               + (" with FP64 transforms and near-tie re-ranking"
                                  if args.precision == "fp32_rerank" else ""),
                   "lost_blocks_per_step": lost_blocks, "frames": len(frames),
                   "launches_per_step": launches // args.steps,
                   "hip_hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"])},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_PUBLISHED,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_PUBLISHED, "traffic": traffic,
                     "kernel": "fse_block_kernel<float>",
                     "flops_per_block": kflops, "blocks_per_launch": blocks_per_launch,
                     "avg_launch_ms": avg_launch_ms,
                     "achieved_note": "algorithmic flops of all blocks of a step over the "
                                      "union of the kernel's launch intervals (HIP events on "
                                      "the launches' streams): the launches of the frame "
                                      "groups overlap",
                     "peak_nonpacked": PEAK_FP32_TFLOPS,
                     "frac_nonpacked": achieved / PEAK_FP32_TFLOPS,
                     "peak_note": "published FP32 vector peak (counts packed FP32); this "
                                  "build compiles without packed FP32 instructions, so "
                                  "78.6 TFLOP/s (256 CU x 4 SIMD x 16 lanes x FMA x "
                                  "2.4 GHz) is what it can issue",
                     "kernel_busy_ms_per_step": busy_ms, "groups": head["groups"],
                     "achieved_per_launch": achieved_launch,
                     "frac_per_launch": achieved_launch / PEAK_FP32_PUBLISHED,
                     "per_launch_note": "the flops of the blocks one launch processes on "
                                        "average over the average launch duration; a launch "
                                        "shares the GPU with the other groups' launches "
                                        "(overlap_factor = summed launch time over the union "
                                        "of the launch intervals)",
                     "overlap_factor": avg_launch_ms * launches / args.steps / busy_ms,
                     "algorithmic_hbm_bytes_per_launch": alg_bytes_launch,
                     "traffic_over_algorithmic": (traffic / alg_bytes_launch if traffic else None),
                     "traffic_note": "HBM bytes of one launch on average (the step's launches) "
                                     "from rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0 (copy-"
                                     "calibrated), taken on this kernel source and launch "
                                     "configuration; null when either changed since",
                     "measured_peaks": peaks,
                     "frac_of_measured_fp32_fma": (achieved / peaks["fp32_fma_tflops"]
                                                   if peaks else None),
                     "lds_tbps": lds_tbps,
                     "lds_frac_of_measured": (lds_tbps / peaks["lds_read_tbps"]
                                              if peaks else None),
                     "lds_note": "the iteration's shifted reads of W (K x 4096 x 8 bytes per "
                                 "block) over the kernel's busy time, against the measured "
                                 "LDS read bandwidth",
                     "valu_issue_frac": valu_issue_frac,
                     "valu_issue_note": "VALU wavefront-instructions of a step (rocprofv3 "
                                        "SQ_INSTS_VALU, same source and launch configuration; "
                                        "null otherwise) x 4 cycles over 1024 SIMDs x 2.4 GHz "
                                        "x the kernel's busy time"},
        "fp64_plain": fp64,
        "precision_sweep": sweep,
        "p99_frame_latency_ms": serving["p99_frame_latency_ms"] if serving else None,
        "serving": serving,
        "end_to_end": e2e,
        "volume_3d": volume,
        "order_comparison": order,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
