"""Parity helpers: compare the GPU path with the oracle.

Nothing here computes the method itself: the oracle does, through
``oracle.extract_area`` / ``oracle.block``; these helpers only rebuild the
snapshot a block saw, and score indices, samples and PSNR.
"""
import numpy as np

import oracle

KNOWN, PENDING, RECON = 0, 1, 2


def psnr(out_u8, truth_u8, lost):
    m = lost.astype(bool)
    if not m.any():
        return float("inf")
    err = out_u8[m].astype(np.float64) - truth_u8[m].astype(np.float64)
    mse = float(np.mean(err * err))
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def mirror(k, nf=64, mf=64):
    k = np.asarray(k)
    return ((-(k // nf)) % mf) * nf + ((-(k % nf)) % nf)


def index_agreement(u_a, u_b):
    """Fraction of iterations whose selected indices agree, scored modulo one
    global mirror applied from the first exact mirror tie on; also the first
    iteration where the two disagree even modulo the mirror (-1 = never)."""
    u_a = np.asarray(u_a)
    u_b = np.asarray(u_b)
    n = len(u_a)
    same = u_a == u_b
    if same.all():
        return 1.0, -1
    first = int(np.argmin(same))
    flipped = np.where(np.arange(n) >= first, mirror(u_a), u_a)
    agree = np.maximum(same, flipped == u_b)
    bad = np.flatnonzero(~agree)
    return float(agree.mean()), int(bad[0]) if len(bad) else -1


def snapshot_for_block(image_u8, lost, gpu_float, wave_of, params, bi, bj):
    """Working image and state map that block (bi, bj) read at the start of
    its wave, rebuilt from the GPU's final unquantized image: samples of
    blocks from earlier waves are reconstructed, the rest still pending."""
    H, W = image_u8.shape
    Bh, Bw = params.block_h, params.block_w
    goy, gox = params.grid_off_y, params.grid_off_x
    yy = (np.arange(H) + goy) // Bh
    xx = (np.arange(W) + gox) // Bw
    blk_wave = wave_of[yy[:, None], xx[None, :]]
    w = wave_of[bi, bj]
    lost_b = lost.astype(bool)
    done = lost_b & (blk_wave >= 0) & (blk_wave < w)
    work = np.where(lost_b, 0.0, image_u8.astype(np.float64))
    work[done] = gpu_float[done]
    state = np.where(lost_b, PENDING, KNOWN).astype(np.uint8)
    state[done] = RECON
    return work, state


def teacher_forced_block(image_u8, lost, gpu_float, wave_of, params, bi, bj):
    """Oracle samples of block (bi, bj) from exactly the input the GPU block
    saw, and the GPU's samples there: (oracle values, gpu values, mask)."""
    work, state = snapshot_for_block(image_u8, lost, gpu_float, wave_of, params, bi, bj)
    f, cls = oracle.extract_area(params, work, state, bi, bj)
    res = oracle.block(params, f, cls)
    d = params.border_d
    H, W = image_u8.shape
    y0 = bi * params.block_h - params.grid_off_y
    x0 = bj * params.block_w - params.grid_off_x
    o_vals, g_vals = [], []
    for m in range(params.M):
        for n in range(params.N):
            if cls[m, n] == oracle.CLS_BI:
                y, x = y0 - d + m, x0 - d + n
                o_vals.append(res.g[m, n])
                g_vals.append(gpu_float[y, x])
    return np.array(o_vals), np.array(g_vals), res
