"""Pins of the oracle's fast LLF (the comparator of Sec. II-C) against facts that
do not depend on its code: linear interpolation in g is exact for remaps whose
Laplacian coefficients are affine in g; with two samples the nodes are 0 and R;
the identity remap returns the input; more samples approach naive LLF."""
import numpy as np
import pytest

from oracle import fourier_llf_ref as ref


def _img(h, w, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(h, w))


@pytest.mark.parametrize("n", [2, 3, 7])
def test_exact_for_remaps_affine_in_g(n):
    # r(i, g) = i (1 + c g) + d g: L_l[r(I, g)] = (1 + c g) L_l[I] below the top
    # (the d g term is a constant image), so interpolating in g is exact.
    I = _img(12, 10, 1)
    remap = lambda i, g: i * (1.0 + 0.7 * g) + 0.3 * g
    want = ref.naive_llf(I, 3, remap)
    got = ref.fast_llf(I, 3, remap, n)
    assert ref.max_abs(got, want) <= 1e-12


def test_two_samples_sit_at_zero_and_R():
    # r(i, g) = i (1 + c g^2): with nodes {0, R} the interpolated coefficient is
    # (1 + c g R) L_l[I]_p (chord of g^2 between 0 and R), residual G_top[I].
    I = _img(16, 12, 2)
    c, R, L = 0.5, 1.0, 3
    got = ref.fast_llf(I, L, lambda i, g: i * (1.0 + c * g * g), 2, R=R)
    G = ref.gaussian_pyramid(I, L)
    LI = ref.laplacian_pyramid(I, L)
    want = ref.collapse([(1.0 + c * G[l] * R) * LI[l] for l in range(L - 1)] + [G[L - 1]])
    assert ref.max_abs(got, want) <= 1e-12


def test_identity_remap_returns_input():
    I = _img(20, 17, 3)
    assert ref.max_abs(ref.fast_llf(I, 4, lambda i, g: i, 5), I) <= 1e-12


def test_converges_to_naive_with_more_samples():
    I = _img(16, 16, 4)
    remap = lambda i, g: ref.remap_exact(i, g, 0.15, 2.0)
    want = ref.naive_llf(I, 3, remap)
    errs = [ref.max_abs(ref.fast_llf(I, 3, remap, n), want) for n in (3, 5, 9, 17, 33)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.1 * errs[0]


def test_needs_two_samples():
    with pytest.raises(ValueError):
        ref.fast_llf(_img(8, 8, 5), 2, lambda i, g: i, 1)
