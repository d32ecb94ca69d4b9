"""FP64 CPU oracle for the Fourier local Laplacian filter (Gaussian Fourier pyramid).

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the HIP
path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
GPU library (``paper_2206_04681_amd``) and imports nothing from it.

Everything is float64 NumPy.  Each function names the passage of the paper
("Gaussian Fourier Pyramid for Local Laplacian Filter", Sumiya et al., IEEE SPL)
that it follows.  Readings taken where the paper is silent or inconsistent:

* Remap sign (Sec. II-D vs. Sec. III-A): the Fourier remap is used exactly as
  printed in Eq. (11) and the per-level formula exactly as in Eq. (14).  Eq. (11)
  equals ``i + m * sum_k at_k sin(w_k (i - g))``, which approximates
  ``i + m (i - g) exp(-(i - g)^2 / (2 sigma_r^2))``; that is the form whose
  ``m > 0`` enhances detail as the text around Eq. (6) states.  ``remap_exact``
  below is that reading.
* Eq. (12) writes ``sigma``; it is ``sigma_r``.  ``R`` is the intensity range
  (``R = 1`` for images in [0, 1]).  Eq. (12) is minimised literally (no sqrt(2)).
* The 5-tap filter is the binomial [1, 4, 6, 4, 1] / 16 (Sec. II-A, "binomial,
  five taps, sigma ~ 1"); upsampling uses the same kernel with gain 4 in 2-D
  applied to the zero-inserted grid (Eq. (2) and the sentence after it).
* Borders (the paper is silent): reflect-101, i.e. ``... c b | a b c d | c b ...``,
  applied as a general fold so that it also covers length-2 and length-1 axes.
  Decimation keeps even indices; level sizes are ``ceil(n / 2)``.
* ``levels`` = |L| = l_max + 1 counts the residual (top) level.
* Collapse of Eq. (4) is the usual recursive upsample-and-add.
* No clipping of the output.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import math
from typing import Callable, List, Sequence

import numpy as np

# Binomial 5-tap filter of Sec. II-A (Eq. (1)); weights are dyadic, exact in FP.
BINOMIAL5 = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


# --------------------------------------------------------------------------- #
# Series fit: Eq. (9), (10), (11), (12)
# --------------------------------------------------------------------------- #
def period_error(T: float, sigma_r: float, K: int, R: float) -> float:
    """E_K(T) of Eq. (12): erfc(pi sigma (2K+1) / T) + erfc((T - R) / sigma)."""
    return math.erfc(math.pi * sigma_r * (2 * K + 1) / T) + math.erfc((T - R) / sigma_r)


def fit_period(sigma_r: float, K: int, R: float = 1.0) -> float:
    """T = argmin_{T > R} E_K(T) (Eq. (12)).

    Plain search: a uniform scan of (R, R + 20 sigma_r + 4 pi sigma_r (2K+1)]
    brackets the minimum, then golden-section search refines it in float64.
    """
    if sigma_r <= 0 or K < 1 or R <= 0:
        raise ValueError("sigma_r > 0, K >= 1 and R > 0 are required")
    lo = R
    hi = R + 20.0 * sigma_r + 4.0 * math.pi * sigma_r * (2 * K + 1)
    n = 20000
    grid = [lo + (hi - lo) * (i + 1) / n for i in range(n)]
    vals = [period_error(t, sigma_r, K, R) for t in grid]
    i = int(np.argmin(vals))
    a = grid[max(i - 1, 0)] if i > 0 else lo
    b = grid[min(i + 1, n - 1)]
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(300):
        c = b - g * (b - a)
        d = a + g * (b - a)
        if period_error(c, sigma_r, K, R) < period_error(d, sigma_r, K, R):
            b = d
        else:
            a = c
    return 0.5 * (a + b)


def fit_period_range(sigma_lo: float, sigma_hi: float, K: int, R: float = 1.0) -> float:
    """One period for every range scale in [sigma_lo, sigma_hi] (pixel-by-pixel
    alpha~_{k,p}, Sec. III-B, where one T must serve all pixels).  Each term of
    Eq. (12) is taken at the scale where it is largest: the truncation term
    erfc(pi sigma (2K+1) / T) grows as sigma falls, the aliasing term
    erfc((T - R) / sigma) as sigma rises, so
        T = argmin_{T > R} erfc(pi sigma_lo (2K+1) / T) + erfc((T - R) / sigma_hi).
    Same plain scan and golden-section search as fit_period; with
    sigma_lo = sigma_hi it is Eq. (12) itself."""
    if not (0 < sigma_lo <= sigma_hi) or K < 1 or R <= 0:
        raise ValueError("0 < sigma_lo <= sigma_hi, K >= 1 and R > 0 are required")

    def E(T):
        return math.erfc(math.pi * sigma_lo * (2 * K + 1) / T) + math.erfc((T - R) / sigma_hi)

    lo = R
    hi = R + 20.0 * sigma_hi + 4.0 * math.pi * sigma_lo * (2 * K + 1)
    n = 20000
    grid = [lo + (hi - lo) * (i + 1) / n for i in range(n)]
    i = int(np.argmin([E(t) for t in grid]))
    a = grid[max(i - 1, 0)] if i > 0 else lo
    b = grid[min(i + 1, n - 1)]
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(300):
        c = b - g * (b - a)
        d = a + g * (b - a)
        if E(c) < E(d):
            b = d
        else:
            a = c
    return 0.5 * (a + b)


def fourier_coefficients(sigma_r: float, K: int, T: float):
    """omega_k, alpha_k and alpha~_k for k = 1..K (Eq. (9) and Eq. (11)).

    omega_k = 2 pi k / T
    alpha_k = sigma_r sqrt(2 pi) / T * exp(-(omega_k sigma_r)^2 / 2)
    alpha~_k = 2 sigma_r^2 alpha_k omega_k
    Returns three float64 arrays of length K, plus alpha_0.
    """
    k = np.arange(1, K + 1, dtype=np.float64)
    omega = 2.0 * math.pi * k / T
    alpha = sigma_r * math.sqrt(2.0 * math.pi) / T * np.exp(-0.5 * (omega * sigma_r) ** 2)
    alpha0 = sigma_r * math.sqrt(2.0 * math.pi) / T
    alpha_t = 2.0 * sigma_r ** 2 * alpha * omega
    return omega, alpha, alpha_t, alpha0


def gaussian_series(x, sigma_r: float, K: int, T: float):
    """Cosine series of exp(-x^2 / (2 sigma_r^2)) (Eq. (9) with m = 1)."""
    omega, alpha, _, alpha0 = fourier_coefficients(sigma_r, K, T)
    x = np.asarray(x, dtype=np.float64)
    return alpha0 + 2.0 * np.sum(alpha[:, None] * np.cos(omega[:, None] * x.ravel()[None, :]), axis=0).reshape(x.shape)


def remap_exact(i, g, sigma_r: float, m: float):
    """Detail remap r(i, g) = i + m (i - g) exp(-(i - g)^2 / (2 sigma_r^2)).

    This is the reading of Eq. (5)-(6) that agrees with Eq. (11) and with the
    enhance/smooth statement for the sign of m (Sec. II-D).
    """
    d = np.asarray(i, dtype=np.float64) - g
    return np.asarray(i, dtype=np.float64) + m * d * np.exp(-(d * d) / (2.0 * sigma_r ** 2))


def remap_fourier(i, g, sigma_r: float, m: float, K: int, T: float):
    """Fourier remap r_K(i, g) of Eq. (11), written term by term as printed:

        i - m sum_k at_k ( sin(w_k g) cos(w_k i) - cos(w_k g) sin(w_k i) ).
    """
    omega, _, alpha_t, _ = fourier_coefficients(sigma_r, K, T)
    i = np.asarray(i, dtype=np.float64)
    out = i.copy()
    for k in range(K):
        out = out - m * alpha_t[k] * (np.sin(omega[k] * g) * np.cos(omega[k] * i)
                                      - np.cos(omega[k] * g) * np.sin(omega[k] * i))
    return out


# --------------------------------------------------------------------------- #
# Pyramids: Eq. (1), (2), (4)
# --------------------------------------------------------------------------- #
def fold_index(i: int, n: int) -> int:
    """Reflect-101 border fold onto [0, n): ... 2 1 | 0 1 2 ... n-1 | n-2 ..."""
    if n == 1:
        return 0
    p = 2 * n - 2
    i = i % p
    return p - i if i > n - 1 else i


def _filter_axis(X: np.ndarray, axis: int) -> np.ndarray:
    """5-tap binomial along one axis with reflect-101 borders (full resolution)."""
    n = X.shape[axis]
    out = np.zeros_like(X)
    for d in range(-2, 3):
        idx = [fold_index(j + d, n) for j in range(n)]
        out += BINOMIAL5[d + 2] * np.take(X, idx, axis=axis)
    return out


def reduce_(X: np.ndarray) -> np.ndarray:
    """REDUCE of Eq. (1): blur with the binomial kernel, keep even rows/columns."""
    Y = _filter_axis(_filter_axis(X, 0), 1)
    return Y[0::2, 0::2]


def expand(X: np.ndarray, shape: Sequence[int]) -> np.ndarray:
    """Upsampling of Eq. (2): zero-insert to ``shape`` then blur with 4 (w x w)."""
    Z = np.zeros(tuple(shape), dtype=np.float64)
    Z[0::2, 0::2] = X
    return 4.0 * _filter_axis(_filter_axis(Z, 0), 1)


def gaussian_pyramid(X: np.ndarray, levels: int) -> List[np.ndarray]:
    """G_0 = X, G_{l+1} = REDUCE(G_l) for l < levels - 1 (Eq. (1))."""
    pyr = [np.asarray(X, dtype=np.float64)]
    for _ in range(levels - 1):
        pyr.append(reduce_(pyr[-1]))
    return pyr


def laplacian_pyramid(X: np.ndarray, levels: int) -> List[np.ndarray]:
    """L_l = G_l - EXPAND(G_{l+1}); the top level is G_lmax (Eq. (2))."""
    G = gaussian_pyramid(X, levels)
    out = [G[l] - expand(G[l + 1], G[l].shape) for l in range(levels - 1)]
    out.append(G[-1])
    return out


def collapse(Lp: List[np.ndarray]) -> np.ndarray:
    """Collapse of Eq. (4), recursively: O_l = L_l + EXPAND(O_{l+1})."""
    O = Lp[-1]
    for l in range(len(Lp) - 2, -1, -1):
        O = Lp[l] + expand(O, Lp[l].shape)
    return O


def max_levels(height: int, width: int) -> int:
    """Largest |L| such that every level that is upsampled has both sides >= 2."""
    return 1 + int(math.floor(math.log2(min(height, width))))


# --------------------------------------------------------------------------- #
# The method: Eq. (13)-(14), Fig. 2
# --------------------------------------------------------------------------- #
def fourier_llf(I: np.ndarray, levels: int, sigma_r: float, m: float, K: int,
                R: float = 1.0, T: float | None = None) -> np.ndarray:
    """Fourier LLF of one grayscale plane, Eq. (14) case by case, then Eq. (4).

    C~_{l,k} = G_l[cos(w_k I)], S~_{l,k} = G_l[sin(w_k I)]: the 2K Gaussian
    Fourier pyramids; plus G_l[I].  For l = 0 the level-0 Fourier terms drop out
    because r(I, I_p) = I (first case of Eq. (14)); for 1 <= l < l_max both the
    level-l and the upsampled level-(l+1) terms appear; L_lmax[O] = G_lmax[I].
    """
    I = np.asarray(I, dtype=np.float64)
    if T is None:
        T = fit_period(sigma_r, K, R)
    omega, _, alpha_t, _ = fourier_coefficients(sigma_r, K, T)
    G = gaussian_pyramid(I, levels)
    Ct = [gaussian_pyramid(np.cos(omega[k] * I), levels) for k in range(K)]
    St = [gaussian_pyramid(np.sin(omega[k] * I), levels) for k in range(K)]

    LO: List[np.ndarray] = []
    for l in range(levels - 1):
        shape = G[l].shape
        g = G[l]
        up_sum = np.zeros(shape)
        for k in range(K):
            up_sum += alpha_t[k] * (np.sin(omega[k] * g) * expand(Ct[k][l + 1], shape)
                                    - np.cos(omega[k] * g) * expand(St[k][l + 1], shape))
        if l == 0:
            Lo = I - expand(G[1], shape) + m * up_sum
        else:
            here_sum = np.zeros(shape)
            for k in range(K):
                here_sum += alpha_t[k] * (np.sin(omega[k] * g) * Ct[k][l]
                                          - np.cos(omega[k] * g) * St[k][l])
            Lo = G[l] - m * here_sum - expand(G[l + 1], shape) + m * up_sum
        LO.append(Lo)
    LO.append(G[levels - 1])
    return collapse(LO)


def fourier_llf_image(img: np.ndarray, levels: int, sigma_r: float, m: float, K: int,
                      R: float = 1.0, T: float | None = None) -> np.ndarray:
    """Per-channel Fourier LLF of a (C, H, W) or (H, W) array."""
    img = np.asarray(img, dtype=np.float64)
    if img.ndim == 2:
        return fourier_llf(img, levels, sigma_r, m, K, R, T)
    return np.stack([fourier_llf(c, levels, sigma_r, m, K, R, T) for c in img])


def alpha_tilde_of(sigma, K: int, T: float) -> np.ndarray:
    """alpha~_k = 2 sigma^2 alpha_k omega_k (Eq. (9), Eq. (11)) for an array of
    range scales: shape (K,) + sigma.shape, written out from Eq. (9) at each sigma."""
    sigma = np.asarray(sigma, dtype=np.float64)
    k = np.arange(1, K + 1, dtype=np.float64).reshape((K,) + (1,) * sigma.ndim)
    omega = 2.0 * math.pi * k / T
    alpha = sigma * math.sqrt(2.0 * math.pi) / T * np.exp(-0.5 * (omega * sigma) ** 2)
    return 2.0 * sigma ** 2 * alpha * omega


def fourier_llf_adaptive(I: np.ndarray, levels: int, sigma_r: float, m_map: np.ndarray | None,
                         K: int, R: float = 1.0, T: float | None = None,
                         sigma_map: np.ndarray | None = None, m: float | None = None) -> np.ndarray:
    """Pixel-by-pixel Fourier LLF (Sec. III-B): alpha~_k replaced by alpha~_{k,p}
    and/or m by m_p, pixel by pixel, in Eq. (14).

    The maps are given at level 0 and brought to level l by the Gaussian pyramid
    (their value at the level-l pixel p): sigma_p = G_l[sigma_map]_p gives
    alpha~_{k,p} through Eq. (9) and (11), m_p = G_l[m_map]_p.  The Fourier
    pyramids depend on the remap only through omega_k = 2 pi k / T, so they are
    those of the fixed case; a sigma map therefore needs one T for every pixel
    (given, or fitted to the map's range by fit_period_range).  Without a map
    the scalar (sigma_r, or m -- m_map None needs m) is used.
    """
    I = np.asarray(I, dtype=np.float64)
    if sigma_map is not None:
        sigma_map = np.asarray(sigma_map, dtype=np.float64)
        if T is None:
            T = fit_period_range(float(sigma_map.min()), float(sigma_map.max()), K, R)
    elif T is None:
        T = fit_period(sigma_r, K, R)
    omega = 2.0 * math.pi * np.arange(1, K + 1) / T
    G = gaussian_pyramid(I, levels)
    if m_map is not None:
        M = gaussian_pyramid(np.asarray(m_map, dtype=np.float64), levels)
    else:
        if m is None:
            raise ValueError("without m_map the scalar m is needed")
        M = [np.full(g.shape, float(m)) for g in G]
    if sigma_map is not None:
        SG = gaussian_pyramid(sigma_map, levels)
    else:
        SG = [np.full(g.shape, float(sigma_r)) for g in G]
    Ct = [gaussian_pyramid(np.cos(omega[k] * I), levels) for k in range(K)]
    St = [gaussian_pyramid(np.sin(omega[k] * I), levels) for k in range(K)]
    LO: List[np.ndarray] = []
    for l in range(levels - 1):
        shape = G[l].shape
        g = G[l]
        mp = M[l]
        at_p = alpha_tilde_of(SG[l], K, T)  # alpha~_{k,p} at every level-l pixel
        up_sum = np.zeros(shape)
        for k in range(K):
            up_sum += at_p[k] * (np.sin(omega[k] * g) * expand(Ct[k][l + 1], shape)
                                 - np.cos(omega[k] * g) * expand(St[k][l + 1], shape))
        if l == 0:
            Lo = I - expand(G[1], shape) + mp * up_sum
        else:
            here_sum = np.zeros(shape)
            for k in range(K):
                here_sum += at_p[k] * (np.sin(omega[k] * g) * Ct[k][l]
                                       - np.cos(omega[k] * g) * St[k][l])
            Lo = G[l] - mp * here_sum - expand(G[l + 1], shape) + mp * up_sum
        LO.append(Lo)
    LO.append(G[levels - 1])
    return collapse(LO)


# --------------------------------------------------------------------------- #
# Brute force: the definition of LLF (Sec. II-C, Eq. (13))
# --------------------------------------------------------------------------- #
def naive_llf_pyramid(I: np.ndarray, levels: int,
                      remap: Callable[[np.ndarray, float], np.ndarray]) -> List[np.ndarray]:
    """The output Laplacian pyramid of naive LLF (Eq. (13)): for every level
    l < l_max and every level-l pixel p, remap the whole input with
    g = G_l[I]_p, build its pyramid to level l+1 and keep L_l[r(I, g)]_p;
    L_lmax[O] = G_lmax[I].  Level l < l_max does not depend on |L|.

    O(N^2) per level: tiny images only.
    """
    I = np.asarray(I, dtype=np.float64)
    G = gaussian_pyramid(I, levels)
    LO: List[np.ndarray] = []
    for l in range(levels - 1):
        out = np.empty_like(G[l])
        for y in range(G[l].shape[0]):
            for x in range(G[l].shape[1]):
                g = G[l][y, x]
                Gr = gaussian_pyramid(remap(I, g), l + 2)
                lap = Gr[l] - expand(Gr[l + 1], Gr[l].shape)
                out[y, x] = lap[y, x]
        LO.append(out)
    LO.append(G[levels - 1])
    return LO


def naive_llf(I: np.ndarray, levels: int,
              remap: Callable[[np.ndarray, float], np.ndarray]) -> np.ndarray:
    """Naive LLF: the collapse (Eq. (4)) of naive_llf_pyramid."""
    return collapse(naive_llf_pyramid(I, levels, remap))


def naive_llf_adaptive(I: np.ndarray, levels: int, remap: Callable[..., np.ndarray],
                       m_map) -> np.ndarray:
    """Naive LLF whose remap at level-l pixel p takes the per-pixel parameters
    G_l[map]_p: remap(I, g, v) for one map, remap(I, g, v1, v2, ...) when m_map is
    a tuple of maps."""
    I = np.asarray(I, dtype=np.float64)
    G = gaussian_pyramid(I, levels)
    maps = m_map if isinstance(m_map, (tuple, list)) else (m_map,)
    P = [gaussian_pyramid(np.asarray(mm, dtype=np.float64), levels) for mm in maps]
    LO: List[np.ndarray] = []
    for l in range(levels - 1):
        out = np.empty_like(G[l])
        for y in range(G[l].shape[0]):
            for x in range(G[l].shape[1]):
                vals = [Pm[l][y, x] for Pm in P]
                Gr = gaussian_pyramid(remap(I, G[l][y, x], *vals), l + 2)
                lap = Gr[l] - expand(Gr[l + 1], Gr[l].shape)
                out[y, x] = lap[y, x]
        LO.append(out)
    LO.append(G[levels - 1])
    return collapse(LO)


def fast_llf(I: np.ndarray, levels: int, remap: Callable[[np.ndarray, float], np.ndarray],
             n_samples: int, R: float = 1.0) -> np.ndarray:
    """Fast LLF, the comparator of Sec. II-C (Aubry et al.), step by step:
    sample n intensities tau k, k = 0 .. n-1, at equal intervals tau = R / (n-1)
    over [0, R]; build the Laplacian pyramids of the remapped images
    R_k = r(I, tau k); at every level l < l_max and level-l pixel p write
    g = G_l[I]_p = tau ((1-a) k + a (k+1)) with k = floor(g / tau) and take
    L_l[O]_p = (1-a) L_l[R_k]_p + a L_l[R_{k+1}]_p; the residual level is G_lmax[I]
    as in naive LLF; collapse (Eq. (4)).  It uses n + 1 pyramids."""
    if n_samples < 2:
        raise ValueError("fast LLF needs at least 2 sampled intensities")
    I = np.asarray(I, dtype=np.float64)
    G = gaussian_pyramid(I, levels)
    tau = R / (n_samples - 1)
    LR = [laplacian_pyramid(remap(I, tau * k), levels) for k in range(n_samples)]
    LO: List[np.ndarray] = []
    for l in range(levels - 1):
        t = np.clip(G[l] / tau, 0.0, n_samples - 1.0)
        k = np.minimum(np.floor(t).astype(np.int64), n_samples - 2)
        a = t - k
        stack = np.stack([LR[j][l] for j in range(n_samples)])
        lo = np.take_along_axis(stack, k[None], axis=0)[0]
        hi = np.take_along_axis(stack, (k + 1)[None], axis=0)[0]
        LO.append((1.0 - a) * lo + a * hi)
    LO.append(G[levels - 1])
    return collapse(LO)


def variance_boost_map(I: np.ndarray, radius: int, m_max: float, v_half: float) -> np.ndarray:
    """Boost map for pixel-by-pixel enhancement driven by local variance (Sec. IV,
    Fig. 5: the enhancement follows the variance of the pixels in a local
    window, small where the variance is low).  Reading: the window is the
    (2 radius + 1)^2 square around p with reflect-101 borders, v_p its population
    variance, and m_p = m_max v_p / (v_p + v_half): 0 on flat areas, m_max / 2 at
    v_p = v_half, approaching m_max on strong texture.  Plain loops: the mean of
    the window first, then the mean squared deviation from it."""
    I = np.asarray(I, dtype=np.float64)
    H, W = I.shape
    out = np.empty_like(I)
    for y in range(H):
        rows = [fold_index(y + d, H) for d in range(-radius, radius + 1)]
        for x in range(W):
            cols = [fold_index(x + d, W) for d in range(-radius, radius + 1)]
            win = I[np.ix_(rows, cols)]
            mean = win.sum() / win.size
            v = ((win - mean) ** 2).sum() / win.size
            out[y, x] = m_max * v / (v + v_half)
    return out


# --------------------------------------------------------------------------- #
# Metrics
# --------------------------------------------------------------------------- #
def max_abs(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))))


def psnr(a, b, peak: float = 1.0) -> float:
    """PSNR in dB with MAX = peak over all pixels and channels."""
    mse = float(np.mean((np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) ** 2))
    if mse == 0.0:
        return float("inf")
    return 10.0 * math.log10(peak * peak / mse)
