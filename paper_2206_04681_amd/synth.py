"""Seeded synthetic test images (input generation only; none of the filter's arithmetic).

The paper evaluates on natural 512x512 grayscale photographs that are not part
of this project.  These generators stand in for them: piecewise-constant shapes
give strong edges (the case local Laplacian filtering is built for: detail is
boosted without halos at edges), a low-frequency sinusoid gives smooth shading,
and Gaussian noise gives fine detail to enhance.

Recipe (all float64, cast to float32 at the end, values in [0, 1] after clipping):

* background ``0.5 + amp * sin(2 pi (fx x / W + fy y / H) + phi)``,
  ``fx, fy ~ U[0.5, 2]``, ``phi ~ U[0, 2 pi)``, ``amp = 0.2``;
* ``n_rect`` axis-aligned rectangles with integer corners uniform over the image;
* ``n_disk`` disks, centre uniform, radius ``~ U[min(W,H)/32, min(W,H)/6]``;
* shapes painted in order, each with intensity ``~ U[0, 1]``;
* additive Gaussian noise of std ``noise``, then clip to [0, 1].

Multi-channel images use one shape geometry per image and independent
intensities, background phase and noise per channel.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np


def synth_image(height: int, width: int, channels: int = 1, seed: int = 0,
                n_rect: int = 6, n_disk: int = 4, noise: float = 0.02,
                amp: float = 0.2) -> np.ndarray:
    """Return a float32 array of shape (channels, height, width) in [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = int(height), int(width)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    fx, fy = rng.uniform(0.5, 2.0, size=2)
    rects = []
    for _ in range(n_rect):
        x0, x1 = np.sort(rng.integers(0, W + 1, size=2))
        y0, y1 = np.sort(rng.integers(0, H + 1, size=2))
        rects.append((int(y0), int(y1), int(x0), int(x1)))
    mn = min(H, W)
    disks = []
    for _ in range(n_disk):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        r = rng.uniform(mn / 32.0, mn / 6.0)
        disks.append((cy, cx, r))
    out = np.empty((channels, H, W), dtype=np.float32)
    for c in range(channels):
        phi = rng.uniform(0.0, 2.0 * np.pi)
        img = 0.5 + amp * np.sin(2.0 * np.pi * (fx * xx / W + fy * yy / H) + phi)
        # paint in order: rectangles then disks, interleaved by index
        shapes: List[Tuple[str, tuple]] = []
        for i in range(max(n_rect, n_disk)):
            if i < n_rect:
                shapes.append(("r", rects[i]))
            if i < n_disk:
                shapes.append(("d", disks[i]))
        for kind, s in shapes:
            v = rng.uniform(0.0, 1.0)
            if kind == "r":
                y0, y1, x0, x1 = s
                img[y0:y1, x0:x1] = v
            else:
                cy, cx, r = s
                img[(yy - cy) ** 2 + (xx - cx) ** 2 <= r * r] = v
        img = img + rng.normal(0.0, noise, size=(H, W))
        out[c] = np.clip(img, 0.0, 1.0).astype(np.float32)
    return out


@dataclass(frozen=True)
class Workload:
    """One filter invocation: image shape and filter parameters."""
    height: int
    width: int
    channels: int
    levels: int
    K: int
    sigma_r: float
    m: float
    seed: int
    n_rect: int = 6
    n_disk: int = 4
    noise: float = 0.02

    def image(self) -> np.ndarray:
        return synth_image(self.height, self.width, self.channels, self.seed,
                           self.n_rect, self.n_disk, self.noise)

    @property
    def megapixels(self) -> float:
        return self.height * self.width / 1e6


# 512x512 grayscale, 6 rectangles + 4 disks, noise 0.02; 6 levels, K = 4,
# sigma_r = 0.2, detail boost m = 2.
SMALL_GRAY = Workload(512, 512, 1, 6, 4, 0.2, 2.0, seed=0)
# 3840x2160 RGB, 20 rectangles + 20 disks, noise 0.01; 8 levels, K = 8,
# sigma_r = 0.1, detail boost m = 3.
UHD_RGB = Workload(2160, 3840, 3, 8, 8, 0.1, 3.0, seed=1, n_rect=20, n_disk=20, noise=0.01)


def levels_for_size(height: int, width: int) -> int:
    """Level count for uneven batches: 8 if min side >= 1024 else 7."""
    return 8 if min(height, width) >= 1024 else 7


def batch_workloads(n: int = 64, seed: int = 3, K: int = 8, m: float = 2.0) -> List[Workload]:
    """Uneven batch: W ~ U{480..4096}, H ~ U{320..2160}; half gray, half RGB
    (seeded permutation); sigma_r ~ U[0.05, 0.3]; content as SMALL_GRAY."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = rng.integers(480, 4097, size=n)
    H = rng.integers(320, 2161, size=n)
    ch = np.array([1] * (n // 2) + [3] * (n - n // 2))
    ch = ch[rng.permutation(n)]
    sig = rng.uniform(0.05, 0.3, size=n)
    return [Workload(int(H[i]), int(W[i]), int(ch[i]), levels_for_size(int(H[i]), int(W[i])),
                     K, float(sig[i]), m, seed=1000 * seed + i) for i in range(n)]


# Request stream of the serving form: RGB sizes with their probabilities.
SERVE_SIZES = ((720, 1280), (1080, 1920), (2160, 3840), (4320, 7680))
SERVE_WEIGHTS = (0.4, 0.3, 0.25, 0.05)


@dataclass(frozen=True)
class Request:
    """One request of the serving form: arrival time (s) and its job."""
    arrival: float
    work: Workload


def serve_requests(rate: float = 200.0, seconds: float = 60.0, seed: int = 4, m: float = 2.0,
                   sizes=SERVE_SIZES, weights=SERVE_WEIGHTS, Ks=(4, 8, 16),
                   content_variants: int = 4) -> List[Request]:
    """Open-loop Poisson arrivals at `rate` per second for `seconds`: RGB sizes
    drawn with `weights`, K uniform over `Ks`, sigma_r ~ U[0.05, 0.3], levels by
    size (levels_for_size).  Image content cycles through `content_variants`
    seeds per size (the content does not change the work)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    p = np.asarray(weights, dtype=np.float64)
    p = p / p.sum()
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        h, w = sizes[int(rng.choice(len(sizes), p=p))]
        K = int(Ks[int(rng.integers(0, len(Ks)))])
        sig = float(rng.uniform(0.05, 0.3))
        variant = int(rng.integers(0, content_variants))
        out.append(Request(t, Workload(h, w, 3, levels_for_size(h, w), K, sig, m,
                                       seed=100000 * seed + 1000 * variant + h % 997)))
    return out
