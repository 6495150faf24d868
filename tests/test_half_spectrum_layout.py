"""The layout of the re-rank mode's FP64 half-spectrum transforms (the block
kernel's rerank_transforms), emulated task by task in numpy: the row stage's
8 x 4 factorization, the real pairs (Z[k], Z[32 - k]) with results written
back into each task's own slots, the slot table kHalfSlot read from the
kernel source, the 8 x 8 column stage and the read-out of columns 0..32
(columns 0 and 32 from their shared slot) must give numpy's 2-D DFT of a
real 64 x 64 area, and exact zeros for a zero area.  A check of the index
logic only; the kernel itself is tested against the oracle on the GPU."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TW = np.exp(-2j * np.pi * np.arange(64) / 64)


def kernel_slot_table():
    src = open(os.path.join(ROOT, "paper_2207_00233_amd", "csrc", "fse_kernels.hip")).read()
    m = re.search(r"kHalfSlot\[kHalf\]\s*=\s*\{([^}]*)\}", src)
    assert m, "slot table not found"
    return [int(v) for v in m.group(1).replace("\n", " ").split(",")]


def dft(v):
    n = len(v)
    return np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) @ np.asarray(v)


def real_pair(zk, zp, k):
    e = (zk + np.conj(zp)) / 2
    o = -1j * (zk - np.conj(zp)) / 2
    to = o * TW[k]
    return e + to, np.conj(e - to)


def transform(x, M):
    """Rows m < M of x hold the area (the rest is zero)."""
    G = np.full((64, 33), np.nan + 0j)
    for m in range(M):  # gather: slot p holds the sample pair (x[2p], x[2p+1])
        G[m, :32] = x[m, 0::2] + 1j * x[m, 1::2]
    for m in range(M):  # task (m, n2): 8-point DFT over n1 of slot 4 n1 + n2
        for n2 in range(4):
            v = dft(G[m, n2:32:4])
            G[m, n2:32:4] = v * TW[(2 * n2 * np.arange(8)) % 64]
    for m in range(M):  # task (m, tau): 4-point DFTs ka, kb, real pairs, own slots
        for tau in range(4):
            t0 = tau == 0
            ka, kb = (0, 4) if t0 else (tau, 8 - tau)
            za, zb = dft(G[m, 4 * ka:4 * ka + 4]), dft(G[m, 4 * kb:4 * kb + 4])
            kA, kB = (8, 4) if t0 else (tau, tau + 8)
            kC, kD = (12 if t0 else 16 - tau), 8 - tau
            o = [*real_pair(za[1] if t0 else za[0], za[3] if t0 else zb[3], kA),
                 *real_pair(zb[0] if t0 else za[1], zb[3] if t0 else zb[2], kB),
                 *real_pair(zb[1], zb[2] if t0 else za[2], kC),
                 *real_pair(zb[0], za[3], kD)]
            if t0:
                o[6] = complex(za[0].real + za[0].imag, za[0].real - za[0].imag)
                o[7] = np.conj(za[2])
            G[m, 4 * ka:4 * ka + 4] = o[:4]
            G[m, 4 * kb:4 * kb + 4] = o[4:]
    col = np.where(np.arange(64)[:, None] < M, G[:, :32], 0)
    for m2 in range(8):  # task (s, m2): 8-point DFT over m1 of row 8 m1 + m2
        v = np.array([dft(col[m2::8, s]) for s in range(32)]).T
        col[m2::8, :] = v * TW[(m2 * np.arange(8)) % 64][:, None]
    for k1 in range(8):  # task (s, k1): 8-point DFT over the rows 8 k1 ..
        col[8 * k1:8 * k1 + 8, :] = np.array([dft(col[8 * k1:8 * k1 + 8, s]) for s in range(32)]).T
    return col


def read_out(G, slot):
    """Entry (K, k2) as the kernel reads it from the grid."""
    pos = lambda K: 8 * (K & 7) + (K >> 3)
    out = np.zeros((64, 64), complex)
    for K in range(64):
        Km = (64 - K) & 63
        for k2 in range(64):
            hi = k2 > 32
            c = 64 - k2 if hi else k2
            v = G[pos(Km if hi else K), slot[c]]
            if c in (0, 32):
                vm = G[pos(Km), slot[c]]
                v = (complex((v.real + vm.real) / 2, (v.imag - vm.imag) / 2) if c == 0 else
                     complex((v.imag + vm.imag) / 2, -(v.real - vm.real) / 2))
            elif hi:
                v = np.conj(v)
            out[K, k2] = v
    return out


def test_slot_table_inverts_the_row_stage():
    slot = kernel_slot_table()
    assert len(slot) == 33 and slot[0] == slot[32]
    held = {}
    for tau in range(4):  # the frequencies each task writes into its slots
        t0 = tau == 0
        ka, kb = (0, 4) if t0 else (tau, 8 - tau)
        ks = [8, 24, 4, 28, 12, 20, 0, 16] if t0 else \
            [tau, 32 - tau, tau + 8, 24 - tau, 16 - tau, 16 + tau, 8 - tau, 24 + tau]
        for i, k in enumerate(ks):
            held[4 * ka + i if i < 4 else 4 * kb + i - 4] = k
    assert sorted(held) == list(range(32)) and sorted(held.values()) == list(range(32))
    for s, k in held.items():
        assert slot[k] == s


@pytest.mark.parametrize("M,N", [(44, 44), (64, 64), (17, 30), (1, 1)])
def test_half_spectrum_transform_is_the_2d_dft(M, N):
    rng = np.random.default_rng(M * 100 + N)
    x = np.zeros((64, 64))
    x[:M, :N] = rng.standard_normal((M, N))
    S = read_out(transform(x, M), kernel_slot_table())
    np.testing.assert_allclose(S, np.fft.fft2(x), atol=1e-10 * max(1.0, np.abs(x).sum()))


def test_zero_area_gives_exact_zeros():
    S = read_out(transform(np.zeros((64, 64)), 44), kernel_slot_table())
    assert (S == 0).all()
