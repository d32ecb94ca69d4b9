"""Pins for the oracle's pyramid operators (Eq. (1), (2), (4)) against an
independent library (scipy.ndimage) and closed forms."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import fourier_llf_ref as ref

W5 = np.array([1, 4, 6, 4, 1], dtype=np.float64) / 16.0


def _rand(h, w, seed=0):
    return np.random.default_rng(seed).uniform(0, 1, size=(h, w))


@pytest.mark.parametrize("n,expect", [
    (1, [0, 0, 0, 0, 0, 0, 0]),
    (2, [0, 1, 0, 1, 0, 1, 0]),
    (3, [2, 1, 0, 1, 2, 1, 0]),
    (5, [2, 1, 0, 1, 2, 3, 4]),
])
def test_fold_index_reflect101(n, expect):
    # positions -2 .. 4 folded onto [0, n)
    got = [ref.fold_index(i, n) for i in range(-2, 5)]
    assert got == expect


@pytest.mark.parametrize("h,w", [(16, 16), (17, 23), (33, 8), (5, 9), (3, 3), (64, 37)])
def test_reduce_matches_scipy_mirror(h, w):
    # scipy's 'mirror' mode is reflect-101 (d c b | a b c d | c b a)
    X = _rand(h, w, seed=h * 100 + w)
    Y = ndimage.convolve1d(ndimage.convolve1d(X, W5, axis=0, mode="mirror"), W5, axis=1, mode="mirror")
    np.testing.assert_allclose(ref.reduce_(X), Y[0::2, 0::2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("h,w", [(16, 16), (17, 23), (33, 8), (5, 9), (4, 6), (64, 37)])
def test_expand_matches_scipy_mirror(h, w):
    hc, wc = (h + 1) // 2, (w + 1) // 2
    X = _rand(hc, wc, seed=7 + h + w)
    Z = np.zeros((h, w))
    Z[0::2, 0::2] = X
    Y = 4.0 * ndimage.convolve1d(ndimage.convolve1d(Z, W5, axis=0, mode="mirror"), W5, axis=1, mode="mirror")
    np.testing.assert_allclose(ref.expand(X, (h, w)), Y, rtol=0, atol=1e-15)


def test_reduce_length2_and_length1_closed_form():
    # n = 2: every output is the mean of the two samples along that axis
    X = np.array([[1.0, 3.0], [5.0, 11.0]])
    assert np.allclose(ref.reduce_(X), [[(1 + 3 + 5 + 11) / 4.0]], atol=1e-15)
    # n = 1: identity
    assert np.allclose(ref.reduce_(np.array([[2.5]])), [[2.5]])


@pytest.mark.parametrize("h,w", [(2, 2), (2, 7), (3, 5), (8, 8), (9, 17), (30, 17)])
def test_expand_preserves_constants(h, w):
    X = np.full(((h + 1) // 2, (w + 1) // 2), 0.37)
    np.testing.assert_allclose(ref.expand(X, (h, w)), 0.37, rtol=0, atol=1e-15)


def test_expand_preserves_linear_ramp_interior():
    hc, wc = 12, 14
    yy, xx = np.mgrid[0:hc, 0:wc].astype(np.float64)
    X = 0.3 * xx - 0.2 * yy + 1.0
    E = ref.expand(X, (2 * hc, 2 * wc))
    fy, fx = np.mgrid[0:2 * hc, 0:2 * wc].astype(np.float64)
    want = 0.3 * fx / 2 - 0.2 * fy / 2 + 1.0
    np.testing.assert_allclose(E[2:-3, 2:-3], want[2:-3, 2:-3], atol=1e-13)


@pytest.mark.parametrize("h,w,levels", [(32, 32, 5), (33, 17, 4), (24, 20, 3), (7, 5, 3)])
def test_collapse_inverts_laplacian_pyramid(h, w, levels):
    X = _rand(h, w, seed=3)
    np.testing.assert_allclose(ref.collapse(ref.laplacian_pyramid(X, levels)), X, atol=1e-13)


def test_pyramid_linearity():
    X, Y = _rand(29, 31, 1), _rand(29, 31, 2)
    a, b = 0.7, -1.9
    GX, GY, GZ = (ref.gaussian_pyramid(Z, 4) for Z in (X, Y, a * X + b * Y))
    for gx, gy, gz in zip(GX, GY, GZ):
        np.testing.assert_allclose(gz, a * gx + b * gy, atol=1e-14)


def test_level_sizes_are_ceil_half():
    G = ref.gaussian_pyramid(_rand(2160, 17), 5)
    assert [g.shape for g in G] == [(2160, 17), (1080, 9), (540, 5), (270, 3), (135, 2)]


def test_max_levels_keeps_upsampled_levels_at_least_two():
    for h, w in [(2, 2), (3, 9), (17, 5), (512, 512), (2160, 3840), (33, 4097)]:
        L = ref.max_levels(h, w)
        for l in range(L - 1):
            assert -(-h // 2 ** l) >= 2 and -(-w // 2 ** l) >= 2
