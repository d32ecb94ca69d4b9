"""Pins of the oracle's error metrics (max-abs and PSNR with MAX = peak over all
pixels and channels), against closed forms: a uniform offset d gives
MSE = d^2 and PSNR = -20 log10(d / peak); an offset on a fraction f of the
samples gives MSE = f d^2.  Each case is chosen so that a plausible slip fails
one of them: 10 vs 20 log10, a sum instead of a mean, the peak not squared, or
a per-channel instead of a global mean."""
import math

import numpy as np

from oracle import fourier_llf_ref as ref


def test_psnr_uniform_offset_is_60_db():
    a = np.random.default_rng(0).random((3, 40, 50))
    assert abs(ref.psnr(a + 1e-3, a) - 60.0) < 1e-9
    assert abs(ref.psnr(a - 1e-2, a) - 40.0) < 1e-9


def test_psnr_uses_the_square_of_the_peak():
    a = np.zeros((8, 8))
    # offset 1 on a 255 scale: 20 log10(255) = 48.1308 dB
    assert abs(ref.psnr(a + 1.0, a, peak=255.0) - 20.0 * math.log10(255.0)) < 1e-9
    assert abs(ref.psnr(a + 1.0, a, peak=255.0) - 48.130803608679) < 1e-9


def test_psnr_mean_over_every_sample_and_channel():
    a = np.zeros((2, 10, 10))
    b = a.copy()
    b[0] += 1e-3  # one channel of two: MSE = 1e-6 / 2
    assert abs(ref.psnr(b, a) - (60.0 + 10.0 * math.log10(2.0))) < 1e-9
    c = a.copy()
    c[:, :5, :] = 2e-3  # half the rows of every channel: MSE = 4e-6 / 2
    assert abs(ref.psnr(c, a) - (10.0 * math.log10(1.0 / 2e-6))) < 1e-9


def test_psnr_of_identical_arrays_is_infinite_and_symmetric():
    a = np.random.default_rng(1).random((5, 7))
    assert ref.psnr(a, a) == float("inf")
    b = a + 0.01 * np.random.default_rng(2).standard_normal(a.shape)
    assert ref.psnr(a, b) == ref.psnr(b, a)


def test_max_abs_closed_forms():
    a = np.zeros((3, 4, 5))
    b = a.copy()
    b[2, 3, 4] = -0.25
    b[0, 0, 0] = 0.125
    assert ref.max_abs(a, b) == 0.25
    assert ref.max_abs(b, a) == 0.25
    assert ref.max_abs(a, a) == 0.0
