"""GPU parity of the pixel-by-pixel forms (Sec. III-B): per-pixel range scale
sigma_p (alpha~_{k,p}) and boost m_p against the FP64 oracle's
fourier_llf_adaptive, element by element on every channel, at sizes that span
several strips and ragged tails and at a size whose levels 1 and 2 take the
fused path; the variance-driven boost map of Sec. IV against the oracle's
variance_boost_map; and the pipeline map -> filter."""
import numpy as np
import pytest

from oracle import fourier_llf_ref as ref
from oracle_pool import oracle_channels, report
from paper_2206_04681_amd.synth import synth_image

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-4, "f16": 2e-4, "bf16": 2e-3}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


_CTX = {}


def llf(storage="f32"):
    from paper_2206_04681_amd.fllf import FourierLLF
    if storage not in _CTX:
        _CTX[storage] = FourierLLF(storage)
    return _CTX[storage]


def sigma_field(h, w, seed, lo=0.05, hi=0.3):
    """A smooth range-scale map in [lo, hi] (two low-frequency waves), float32."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:h, 0:w]
    fx, fy, ph = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0), rng.uniform(0, 2 * np.pi)
    u = 0.5 + 0.25 * np.sin(2 * np.pi * fx * xx / w + ph) + 0.25 * np.cos(2 * np.pi * fy * yy / h)
    return (lo + (hi - lo) * u).astype(np.float32)


def run_gpu(torch, img, L, smap, K, m=2.0, mmap=None, storage="f32"):
    x = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    sm = torch.from_numpy(smap).cuda()
    mm = None if mmap is None else torch.from_numpy(np.ascontiguousarray(mmap, dtype=np.float32)).cuda()
    lo, hi = float(smap.min()), float(smap.max())
    out = llf(storage).run(x, L, lo, m, K, m_map=mm, sigma_map=sm, sigma_max=hi)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def oracle(img, L, smap, K, m=2.0, mmap=None):
    img = np.asarray(img, dtype=np.float64)
    if img.ndim == 2:
        img = img[None]
    s = smap.astype(np.float64)
    mm = None if mmap is None else np.asarray(mmap, dtype=np.float64)
    return np.stack([ref.fourier_llf_adaptive(c, L, float(s.min()), mm, K, sigma_map=s, m=m) for c in img])


@pytest.mark.parametrize("h,w,L,K", [(64, 64, 5, 8), (70, 45, 4, 4), (33, 130, 5, 8), (129, 97, 6, 16),
                                     (5, 9, 3, 5)])
def test_sigma_map_against_oracle(torch_dev, h, w, L, K):
    img = synth_image(h, w, 1, seed=h * w)
    smap = sigma_field(h, w, seed=h + w)
    got = run_gpu(torch_dev, img, L, smap, K)
    want = oracle(img, L, smap, K)
    assert ref.max_abs(got[0] if got.ndim == 3 else got, want[0]) <= TOL["f32"]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("K", [9, 12, 15])
def test_maps_with_9_to_15_terms(torch_dev, K, storage):
    """Both maps with 9 to 15 terms: the job runs the exact 16-term loop with the
    extra terms' weights zero.  Every channel against the oracle with K terms."""
    h, w, L = 150, 210, 6
    img = synth_image(h, w, 3, seed=K)
    smap = sigma_field(h, w, seed=K + 1, lo=0.08, hi=0.25)
    mmap = (1.0 + 2.0 * synth_image(h, w, 1, seed=K + 2)[0]).astype(np.float32)
    got = run_gpu(torch_dev, img, L, smap, K, m=0.0, mmap=mmap, storage=storage)
    want = oracle(img, L, smap, K, m=0.0, mmap=mmap)
    errs, _ = report(f"150x210 RGB, both maps, K={K}, {storage}", got, want)
    assert max(errs) <= TOL[storage]


def test_sigma_and_boost_maps_together(torch_dev):
    h, w, L, K = 96, 110, 5, 8
    img = synth_image(h, w, 3, seed=4)
    smap = sigma_field(h, w, seed=5, lo=0.08, hi=0.25)
    mmap = (1.0 + 2.0 * synth_image(h, w, 1, seed=6)[0]).astype(np.float32)
    got = run_gpu(torch_dev, img, L, smap, K, m=0.0, mmap=mmap)
    want = oracle(img, L, smap, K, m=0.0, mmap=mmap)
    errs, _ = report("96x110 RGB, sigma and boost maps", got, want)
    assert max(errs) <= TOL["f32"]


@pytest.mark.parametrize("storage,K", [("f32", 8), ("f16", 8), ("bf16", 16)])
def test_sigma_map_at_fused_size_every_channel(torch_dev, storage, K):
    # 1100 x 1500 RGB: level 1 (550 x 750 x 3 channels) above the fusion threshold
    # of 2^19 samples (fused down(1), the level-1 collapse folded into up(0))
    h, w, L = 1100, 1500, 7
    img = synth_image(h, w, 3, seed=31, n_rect=20, n_disk=20, noise=0.01)
    smap = sigma_field(h, w, seed=32)
    got = run_gpu(torch_dev, img, L, smap, K, m=3.0, storage=storage)
    want = oracle_channels(img, L, float(smap.min()), 3.0, K,
                           T=ref.fit_period_range(float(smap.min()), float(smap.max()), K),
                           sigma_map=smap.astype(np.float64))
    errs, ps = report(f"1100x1500 RGB with a sigma map, K={K}, {storage} pyramids", got, want)
    assert max(errs) <= TOL[storage]


def test_constant_sigma_map_matches_the_plain_filter(torch_dev):
    torch = torch_dev
    h, w = 200, 300
    img = synth_image(h, w, 3, seed=9)
    x = torch.from_numpy(img).cuda()
    sm = torch.full((h, w), 0.15, device="cuda")
    a = llf().run(x, 6, 0.15, 2.0, 8, sigma_map=sm, sigma_max=0.15)
    b = llf().run(x, 6, 0.15, 2.0, 8)
    torch.cuda.synchronize()
    assert float((a - b).abs().max()) <= 2e-6


def test_sigma_map_batch_equals_single_runs(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd.fllf import Job
    specs = [((3, 150, 220), 6, 8), ((1, 77, 300), 5, 4), ((3, 1100, 1000), 7, 8)]
    jobs, singles = [], []
    for i, ((c, h, w), L, K) in enumerate(specs):
        x = torch.from_numpy(synth_image(h, w, c, seed=50 + i)).cuda()
        smap = sigma_field(h, w, seed=60 + i)
        sm = torch.from_numpy(smap).cuda()
        kw = dict(sigma_map=sm, sigma_max=float(smap.max()))
        jobs.append(Job(x, L, float(smap.min()), 2.0, K, **kw))
        singles.append(llf().run(x, L, float(smap.min()), 2.0, K, **kw))
    outs = llf().run_batch(jobs)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)


# ---- variance-driven boost map --------------------------------------------------
@pytest.mark.parametrize("h,w,r", [(23, 31, 1), (64, 64, 2), (100, 130, 3), (17, 300, 5), (3, 2, 2), (1, 7, 1)])
def test_boost_map_against_oracle(torch_dev, h, w, r):
    torch = torch_dev
    img = synth_image(h, w, 1, seed=h + 7 * w)[0]
    got = llf().boost_map(torch.from_numpy(img).cuda(), r, 3.0, 0.002)
    torch.cuda.synchronize()
    want = ref.variance_boost_map(img.astype(np.float64), r, 3.0, 0.002)
    assert ref.max_abs(got.cpu().numpy(), want) <= 1e-5


def test_boost_map_of_a_channel_view(torch_dev):
    torch = torch_dev
    img = synth_image(90, 120, 3, seed=12)
    x = torch.from_numpy(img).cuda()
    got = llf().boost_map(x[1, 5:85, 7:107], 2, 2.0, 0.001)
    torch.cuda.synchronize()
    want = ref.variance_boost_map(img[1, 5:85, 7:107].astype(np.float64), 2, 2.0, 0.001)
    assert ref.max_abs(got.cpu().numpy(), want) <= 1e-5


def test_variance_driven_enhancement_pipeline(torch_dev):
    """The boost map from the input's local variance, then the pixel-by-pixel
    filter with it (Sec. IV): against the oracle's map and filter."""
    torch = torch_dev
    h, w, L, K = 256, 320, 6, 8
    img = synth_image(h, w, 1, seed=77, noise=0.02)[0]
    x = torch.from_numpy(img).cuda()
    mm = llf().boost_map(x, 3, 4.0, 0.002)
    out = llf().run(x, L, 0.2, 0.0, K, m_map=mm)
    torch.cuda.synchronize()
    mref = ref.variance_boost_map(img.astype(np.float64), 3, 4.0, 0.002)
    want = ref.fourier_llf_adaptive(img.astype(np.float64), L, 0.2, mref, K)
    assert ref.max_abs(out.cpu().numpy(), want) <= 1e-4
    # flat areas are enhanced less than textured ones: the map follows the variance
    assert float(mm.min()) < 0.5 * float(mm.max())
