"""Accuracy against the number of pyramids (the experiment of Sec. IV, Fig. 4),
on four seeded synthetic 128x128 grayscale images: PSNR to naive LLF (the FP64
oracle with the exact remap) of Fourier LLF (2K + 1 pyramids) and of the fast
LLF comparator (n + 1 pyramids, Sec. II-C), both run by this library's GPU
kernels, for 2, 3 and 4 layers, sigma_r = 30/256 and T = 405.9/256 (the paper's
values on a 256-level scale, here on [0, 1]) and boost m = 2.  Checks the
paper's claims: Fourier LLF is more accurate at every equal pyramid count, its
PSNR grows with K, and at 25 pyramids it is above the 59 dB at which 8-bit
outputs agree.  The naive LLF of each image is computed once (its level-l
coefficients do not depend on the number of layers) in parallel processes.
Run with -s to see the table."""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from oracle import fourier_llf_ref as ref
from paper_2206_04681_amd.synth import synth_image

pytestmark = pytest.mark.gpu

SIGMA, T, M = 30.0 / 256.0, 405.9 / 256.0, 2.0
PYRAMIDS = (5, 9, 13, 17, 21, 25)
SEEDS = (11, 12, 13, 14)
SIZE = 128
LAYERS = (2, 3, 4)


def _remap(i, g):
    return ref.remap_exact(i, g, SIGMA, M)


def _naive_pyramid(seed):
    I = synth_image(SIZE, SIZE, 1, seed=seed)[0].astype(np.float64)
    return ref.naive_llf_pyramid(I, max(LAYERS), _remap)


@pytest.fixture(scope="module")
def truths():
    """seed -> {layers: naive LLF output}."""
    n = min(len(SEEDS), 16, os.cpu_count() or 1)
    with ProcessPoolExecutor(n, mp_context=mp.get_context("spawn")) as ex:
        pyrs = dict(zip(SEEDS, ex.map(_naive_pyramid, SEEDS)))
    out = {}
    for s, LO in pyrs.items():
        I = synth_image(SIZE, SIZE, 1, seed=s)[0].astype(np.float64)
        G = ref.gaussian_pyramid(I, max(LAYERS))
        out[s] = {L: ref.collapse(LO[:L - 1] + [G[L - 1]]) for L in LAYERS}
    return out


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("levels", LAYERS)
def test_fourier_beats_fast_llf_at_equal_pyramids(torch_dev, truths, levels):
    torch = torch_dev
    from paper_2206_04681_amd.fllf import FourierLLF
    llf = FourierLLF("f32")
    four = {p: [] for p in PYRAMIDS}
    fast = {p: [] for p in PYRAMIDS}
    for seed in SEEDS:
        I = synth_image(SIZE, SIZE, 1, seed=seed)
        truth = truths[seed][levels]
        x = torch.from_numpy(I).cuda()
        for p in PYRAMIDS:
            a = llf.run(x, levels, SIGMA, M, (p - 1) // 2, T=T)
            b = llf.run_fast(x, levels, SIGMA, M, p - 1)
            torch.cuda.synchronize()
            four[p].append(ref.psnr(a.cpu().numpy()[0], truth))
            fast[p].append(ref.psnr(b.cpu().numpy()[0], truth))
    rows = [(p, float(np.mean(four[p])), float(np.mean(fast[p]))) for p in PYRAMIDS]
    print(f"\nlayers {levels}: pyramids, mean PSNR to naive LLF of {len(SEEDS)} images: Fourier LLF, fast LLF (GPU)")
    for p, a, b in rows:
        print(f"  {p:3d}  {a:7.2f}  {b:7.2f}")
    for p, a, b in rows:
        assert a > b, (levels, p, a, b)
    f = [a for _, a, _ in rows]
    assert all(y > x for x, y in zip(f[:4], f[1:4])), f  # grows with K while FP32 does not limit it
    assert rows[-1][1] >= 59.0
    g = [b for _, _, b in rows]
    assert all(y > x for x, y in zip(g, g[1:])), g  # fast LLF improves with more samples too
