"""Pins for the series fit (Eq. (9)-(12)) and the remap (Eq. (5)-(11))."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fourier_llf_ref as ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_period_matches_paper_printed_value():
    g = json.load(open(os.path.join(GOLDEN, "paper_period.json")))
    T = ref.fit_period(g["sigma_r"], g["K"], g["R"])
    assert abs(T - g["T_printed"]) / g["T_printed"] < g["rel_tol"]
    assert 404.0 <= T <= 407.0


@pytest.mark.parametrize("sigma,K,R", [(0.2, 4, 1.0), (0.1, 8, 1.0), (0.1, 16, 1.0),
                                       (0.05, 4, 1.0), (0.3, 16, 1.0), (30.0, 10, 256.0)])
def test_period_is_a_local_minimum_of_eq12(sigma, K, R):
    T = ref.fit_period(sigma, K, R)
    E0 = ref.period_error(T, sigma, K, R)
    for d in (1e-3, 1e-2):
        assert ref.period_error(T * (1 + d), sigma, K, R) >= E0
        assert ref.period_error(T * (1 - d), sigma, K, R) >= E0
    # stationarity: the two erfc terms have opposite, equal-magnitude slopes
    a = math.pi * sigma * (2 * K + 1)
    s1 = (a / T ** 2) * math.exp(-(a / T) ** 2)
    s2 = math.exp(-((T - R) / sigma) ** 2) / sigma
    assert abs(s1 - s2) <= 1e-6 * max(s1, s2)


def test_period_values_for_workloads():
    # 512^2 gray (sigma 0.2, K 4) and 4K RGB (sigma 0.1, K 8), K 16 variant
    assert abs(ref.fit_period(0.2, 4) - 1.694720) < 2e-6
    assert abs(ref.fit_period(0.1, 8) - 1.398517) < 2e-6
    assert abs(ref.fit_period(0.1, 16) - 1.639742) < 2e-6


def test_period_scale_invariance():
    # only sigma/R matters: T(s*sigma, K, s*R) = s * T(sigma, K, R)
    t1 = ref.fit_period(0.1, 8, 1.0)
    t2 = ref.fit_period(25.6, 8, 256.0)
    assert abs(t2 / 256.0 - t1) < 1e-7


@pytest.mark.parametrize("sigma", [0.05, 0.1, 0.2, 0.3])
def test_cosine_series_reconstructs_gaussian(sigma):
    # Eq. (9): the truncated Fourier series of the periodised Gaussian;
    # error on [-R, R] falls with K (Poisson summation + truncation).
    x = np.linspace(-1.0, 1.0, 2001)
    exact = np.exp(-x ** 2 / (2 * sigma ** 2))
    errs = []
    for K in (2, 4, 8, 16):
        T = ref.fit_period(sigma, K)
        errs.append(np.max(np.abs(ref.gaussian_series(x, sigma, K, T) - exact)))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-3


def test_derivative_series_and_remap():
    # Eq. (10)-(11): sum_k at_k sin(w_k x) ~ x exp(-x^2 / 2 sigma^2) on [-1, 1]
    sigma, m = 0.2, 2.0
    x = np.linspace(-1.0, 1.0, 4001)
    prev = None
    for K in (2, 4, 8, 12):
        T = ref.fit_period(sigma, K)
        omega, _, at, _ = ref.fourier_coefficients(sigma, K, T)
        ser = np.sum(at[:, None] * np.sin(omega[:, None] * x[None, :]), axis=0)
        err = np.max(np.abs(ser - x * np.exp(-x ** 2 / (2 * sigma ** 2))))
        if prev is not None:
            assert err < prev
        prev = err
        # Eq. (11) term by term equals i + m * series(i - g)
        i = np.linspace(0, 1, 101)
        g = 0.37
        rk = ref.remap_fourier(i, g, sigma, m, K, T)
        series_i = np.sum(at[:, None] * np.sin(omega[:, None] * (i - g)[None, :]), axis=0)
        np.testing.assert_allclose(rk, i + m * series_i, atol=1e-13)
    assert prev < 1e-8


def test_remap_fixes_reference_intensity():
    # r(g, g) = g for both the exact and the Fourier remap (used in Eq. (14), l = 0)
    g = np.linspace(0, 1, 11)
    np.testing.assert_allclose(ref.remap_exact(g, g, 0.2, 3.0), g, atol=0)
    T = ref.fit_period(0.2, 6)
    np.testing.assert_allclose(ref.remap_fourier(g, g, 0.2, 3.0, 6, T), g, atol=1e-15)


def test_remap_sign_enhances_for_positive_m():
    # m > 0 pushes i away from g near g (enhance); m < 0 pulls it toward g
    g, i = 0.5, 0.55
    assert ref.remap_exact(i, g, 0.1, 2.0) > i
    assert ref.remap_exact(i, g, 0.1, -0.5) < i
    # far from g (edges) the remap is ~identity: halos are not created
    assert abs(ref.remap_exact(0.95, 0.05, 0.1, 2.0) - 0.95) < 1e-12
