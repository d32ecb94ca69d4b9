"""Runs the FP64 oracle on the channels of an image in parallel processes (test
helper).  The oracle is single-threaded NumPy; the channels of an image are
independent, so a full-size RGB image is checked on every channel in about the
time of one.  Worker processes are spawned (they never touch the GPU)."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from oracle import fourier_llf_ref as ref


def _one(args):
    kind, plane, levels, sigma, m, K, T, mmap, smap = args
    if kind == "adaptive":
        return ref.fourier_llf_adaptive(plane, levels, sigma, mmap, K, T=T, sigma_map=smap, m=m)
    return ref.fourier_llf(plane, levels, sigma, m, K, T=T)


def oracle_channels(img, levels, sigma, m, K, T=None, m_map=None, workers=None, sigma_map=None):
    """Per-channel oracle output of a (C, H, W) image as a float64 (C, H, W)
    array; with m_map and/or sigma_map the pixel-by-pixel form (maps shared by
    the channels)."""
    img = np.asarray(img, dtype=np.float64)
    if img.ndim == 2:
        img = img[None]
    kind = "plain" if m_map is None and sigma_map is None else "adaptive"
    mm = None if m_map is None else np.asarray(m_map, dtype=np.float64)
    sm = None if sigma_map is None else np.asarray(sigma_map, dtype=np.float64)
    jobs = [(kind, img[c], levels, sigma, m, K, T, mm, sm) for c in range(img.shape[0])]
    n = workers or min(len(jobs), 16, os.cpu_count() or 1)
    if n <= 1 or len(jobs) == 1:
        return np.stack([_one(j) for j in jobs])
    with ProcessPoolExecutor(n, mp_context=mp.get_context("spawn")) as ex:
        return np.stack(list(ex.map(_one, jobs)))


def report(label, got, want, peak=1.0):
    """Per-channel max-abs and PSNR (printed; visible under -s); returns the
    lists of both."""
    errs = [ref.max_abs(got[c], want[c]) for c in range(want.shape[0])]
    ps = [ref.psnr(got[c], want[c], peak) for c in range(want.shape[0])]
    text = ", ".join(f"ch{c} {e:.3e} / {p:.1f} dB" for c, (e, p) in enumerate(zip(errs, ps)))
    print(f"\n{label}: max-abs / PSNR per channel: {text}", flush=True)
    return errs, ps
