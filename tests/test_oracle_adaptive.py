"""Pins of the pixel-by-pixel oracle functions (Sec. III-B): per-pixel range scale
sigma_p (alpha~_{k,p}) and boost m_p, the period fitted to a range of scales, and
the variance-driven boost map (Sec. IV, Fig. 5)."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import fourier_llf_ref as ref


def _img(h, w, seed):
    return np.random.default_rng(seed).random((h, w))


# ---- one period for a range of scales ----------------------------------------
@pytest.mark.parametrize("s,K", [(0.1, 8), (0.2, 4), (0.05, 16)])
def test_fit_range_of_one_scale_is_eq12(s, K):
    assert abs(ref.fit_period_range(s, s, K) - ref.fit_period(s, K)) <= 1e-9 * ref.fit_period(s, K)


@pytest.mark.parametrize("lo,hi,K", [(0.05, 0.3, 8), (0.1, 0.2, 4), (0.08, 0.12, 16)])
def test_fit_range_lies_between_the_fits_of_its_ends_and_is_stationary(lo, hi, K):
    T = ref.fit_period_range(lo, hi, K)
    assert ref.fit_period(lo, K) <= T <= ref.fit_period(hi, K)
    E = lambda t: math.erfc(math.pi * lo * (2 * K + 1) / t) + math.erfc((t - 1.0) / hi)
    h = 1e-6 * T
    assert E(T) <= E(T - h) and E(T) <= E(T + h)


# ---- per-pixel alpha~_{k,p} -----------------------------------------------------
def test_alpha_tilde_of_matches_the_scalar_coefficients():
    T = 1.7
    for s in (0.05, 0.1, 0.3):
        got = ref.alpha_tilde_of(np.array([s, s]), 8, T)[:, 0]
        assert np.allclose(got, ref.fourier_coefficients(s, 8, T)[2], rtol=1e-14, atol=0)


def test_constant_sigma_map_reduces_to_the_fixed_filter():
    I = _img(33, 27, 1)
    T = ref.fit_period_range(0.1, 0.25, 6)
    got = ref.fourier_llf_adaptive(I, 4, 0.15, None, 6, T=T, sigma_map=np.full(I.shape, 0.15), m=2.0)
    want = ref.fourier_llf(I, 4, 0.15, 2.0, 6, T=T)
    assert ref.max_abs(got, want) <= 1e-13


@pytest.mark.parametrize("h,w,L,K", [(20, 17, 3, 4), (24, 20, 3, 6), (16, 16, 4, 8)])
def test_sigma_and_boost_maps_equal_brute_force_with_a_per_pixel_truncated_remap(h, w, L, K):
    """Fourier LLF with alpha~_{k,p} and m_p is naive LLF whose remap at level-l
    pixel p is r_K of Eq. (11) with sigma_p = G_l[sigma_map]_p, m_p = G_l[m_map]_p
    (exact by linearity, as in the fixed case)."""
    I = _img(h, w, h + w)
    yy, xx = np.mgrid[0:h, 0:w]
    smap = 0.08 + 0.2 * xx / (w - 1) + 0.04 * np.sin(yy)
    mmap = 1.0 + 2.0 * yy / (h - 1)
    T = ref.fit_period_range(float(smap.min()), float(smap.max()), K)
    got = ref.fourier_llf_adaptive(I, L, float(smap.min()), mmap, K, T=T, sigma_map=smap)
    remap = lambda img, g, m, s: ref.remap_fourier(img, g, s, m, K, T)
    want = ref.naive_llf_adaptive(I, L, remap, (mmap, smap))
    assert ref.max_abs(got, want) <= 1e-12


def test_sigma_map_error_to_the_exact_remap_falls_with_k():
    I = _img(20, 18, 7)
    smap = 0.12 + 0.12 * np.mgrid[0:20, 0:18][1] / 17
    exact = ref.naive_llf_adaptive(I, 3, lambda img, g, s: ref.remap_exact(img, g, s, 2.0), smap)
    errs = []
    for K in (4, 8, 16):
        T = ref.fit_period_range(float(smap.min()), float(smap.max()), K)
        errs.append(ref.max_abs(ref.fourier_llf_adaptive(I, 3, 0.12, None, K, T=T, sigma_map=smap, m=2.0), exact))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-7


def test_sigma_map_changes_the_output_where_the_scale_changes():
    I = _img(32, 32, 3)
    T = ref.fit_period_range(0.05, 0.3, 8)
    smap = np.full(I.shape, 0.05)
    smap[:, 16:] = 0.3
    a = ref.fourier_llf_adaptive(I, 4, 0.05, None, 8, T=T, sigma_map=smap, m=3.0)
    b = ref.fourier_llf_adaptive(I, 4, 0.05, None, 8, T=T, sigma_map=np.full(I.shape, 0.05), m=3.0)
    assert ref.max_abs(a[:, :8], b[:, :8]) < ref.max_abs(a[:, 24:], b[:, 24:])


# ---- variance-driven boost map ----------------------------------------------------
@pytest.mark.parametrize("r", [1, 2, 3])
def test_variance_map_equals_the_mirror_box_filter(r):
    I = _img(23, 31, r)
    n = 2 * r + 1
    mean = ndimage.uniform_filter(I, size=n, mode="mirror")
    mean2 = ndimage.uniform_filter(I * I, size=n, mode="mirror")
    v = mean2 - mean * mean
    want = 2.5 * v / (v + 0.01)
    assert np.allclose(ref.variance_boost_map(I, r, 2.5, 0.01), want, rtol=1e-9, atol=1e-12)


def test_variance_map_closed_forms():
    # flat image (a dyadic value, so the window mean is exact): zero variance, zero boost
    assert ref.max_abs(ref.variance_boost_map(np.full((9, 11), 0.375), 2, 3.0, 0.01), 0.0) == 0.0
    # vertical stripes 0/1: a (2r+1)-wide window holds r+1 of its own column's value
    # and r of the other, variance (r+1) r / (2r+1)^2 (interior and, by the mirror,
    # at the borders too)
    r = 2
    I = np.tile(np.array([0.0, 1.0]), (7, 6))
    v = (r + 1) * r / (2 * r + 1) ** 2
    got = ref.variance_boost_map(I, r, 4.0, v)  # v_half = v: half the maximum boost
    assert np.allclose(got, 2.0, rtol=1e-12)
