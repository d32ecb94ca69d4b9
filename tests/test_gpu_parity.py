"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by
element, on seeded synthetic images that span several tiles and ragged tails."""
import numpy as np
import pytest

from oracle import fourier_llf_ref as ref
from oracle_pool import oracle_channels, report
from paper_2206_04681_amd.synth import SMALL_GRAY, synth_image

pytestmark = pytest.mark.gpu

# float32 arithmetic with float32 pyramids: max-abs tolerance against float64
TOL_F32 = 1e-4
# 16-bit pyramid storage, float32 filtering and accumulation
TOL_F16, PSNR_F16 = 2e-4, 90.0
TOL_BF16, PSNR_BF16 = 2e-3, 75.0


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


def gpu_run(torch, img, levels, sigma, m, K, storage="f32", m_map=None, T=0.0):
    x = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    mm = None if m_map is None else torch.from_numpy(np.ascontiguousarray(m_map, dtype=np.float32)).cuda()
    out = llf(storage).run(x, levels, sigma, m, K, T=T, m_map=mm)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def oracle_run(img, levels, sigma, m, K, T=None):
    return ref.fourier_llf_image(np.asarray(img, dtype=np.float64), levels, sigma, m, K, T=T)


def _img(h, w, c=1, seed=0):
    return synth_image(h, w, c, seed=seed)


def test_small_gray_workload(torch_dev):
    w = SMALL_GRAY
    img = w.image()
    got = gpu_run(torch_dev, img, w.levels, w.sigma_r, w.m, w.K)
    want = oracle_run(img, w.levels, w.sigma_r, w.m, w.K)
    assert ref.max_abs(got, want) <= TOL_F32


@pytest.mark.parametrize("h,w", [(33, 17), (17, 33), (70, 45), (2, 2), (3, 2), (5, 9)])
def test_every_level_count(torch_dev, h, w):
    img = _img(h, w, seed=h * 7 + w)
    for L in range(1, ref.max_levels(h, w) + 1):
        got = gpu_run(torch_dev, img, L, 0.2, 2.0, 4)
        want = oracle_run(img, L, 0.2, 2.0, 4)
        assert ref.max_abs(got, want) <= TOL_F32, (h, w, L)


@pytest.mark.parametrize("h,w,L", [(1001, 777, 7), (4097, 3, 2), (3, 4097, 2), (1, 1, 1), (1, 300, 1),
                                   (257, 129, 8), (130, 500, 6)])
def test_ragged_sizes(torch_dev, h, w, L):
    img = _img(h, w, seed=h + 3 * w)
    got = gpu_run(torch_dev, img, L, 0.1, 3.0, 8)
    want = oracle_run(img, L, 0.1, 3.0, 8)
    assert ref.max_abs(got, want) <= TOL_F32


@pytest.mark.parametrize("K", [1, 2, 4, 5, 8, 16, 32])
def test_term_counts(torch_dev, K):
    img = _img(96, 80, seed=K)
    got = gpu_run(torch_dev, img, 5, 0.15, 2.5, K)
    want = oracle_run(img, 5, 0.15, 2.5, K)
    assert ref.max_abs(got, want) <= TOL_F32


def test_multichannel_and_negative_boost(torch_dev):
    img = _img(130, 97, c=3, seed=5)
    for m in (3.0, -0.7):
        got = gpu_run(torch_dev, img, 6, 0.1, m, 8)
        want = oracle_run(img, 6, 0.1, m, 8)
        assert ref.max_abs(got, want) <= TOL_F32


def test_given_period_and_range(torch_dev):
    img = 255.0 * _img(64, 72, seed=9)
    got = gpu_run(torch_dev, img, 4, 30.0, 2.0, 10, T=405.9)
    want = ref.fourier_llf_image(img.astype(np.float64), 4, 30.0, 2.0, 10, R=256.0, T=405.9)
    assert ref.max_abs(got, want) <= 255.0 * TOL_F32


def test_zero_boost_returns_input(torch_dev):
    img = _img(120, 88, seed=11)
    got = gpu_run(torch_dev, img, 6, 0.2, 0.0, 8)
    assert ref.max_abs(got, img) <= 1e-5


def test_constant_image_is_fixed(torch_dev):
    img = np.full((1, 77, 51), 0.3, dtype=np.float32)
    got = gpu_run(torch_dev, img, 6, 0.1, 3.0, 8)
    assert ref.max_abs(got, img) <= 1e-5


@pytest.mark.parametrize("storage,tol,min_psnr", [("f16", TOL_F16, PSNR_F16), ("bf16", TOL_BF16, PSNR_BF16)])
@pytest.mark.parametrize("K", [8, 16])
def test_reduced_precision_storage(torch_dev, storage, tol, min_psnr, K):
    img = synth_image(512, 512, 1, seed=1, n_rect=20, n_disk=20, noise=0.01)
    got = gpu_run(torch_dev, img, 8, 0.1, 3.0, K, storage=storage)
    want = oracle_run(img, 8, 0.1, 3.0, K)
    assert ref.max_abs(got, want) <= tol
    assert ref.psnr(got, want) >= min_psnr


def test_pixel_adaptive_boost(torch_dev):
    img = _img(90, 70, seed=12)
    yy, xx = np.mgrid[0:90, 0:70]
    mmap = (0.5 + 2.5 * xx / 69.0).astype(np.float32)
    got = gpu_run(torch_dev, img, 5, 0.2, 0.0, 6, m_map=mmap)
    want = ref.fourier_llf_adaptive(img[0].astype(np.float64), 5, 0.2, mmap.astype(np.float64), 6)
    assert ref.max_abs(got[0], want) <= TOL_F32


def test_batch_matches_individual_runs(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd.fllf import Job
    specs = [((1, 200, 150), 6, 0.2, 2.0, 4), ((3, 64, 99), 5, 0.1, 3.0, 8), ((1, 31, 257), 4, 0.3, -0.5, 16)]
    xs = [torch.from_numpy(_img(h, w, c, seed=i)).cuda() for i, ((c, h, w), *_) in enumerate(specs)]
    outs = llf().run_batch([Job(x, L, s, m, K) for x, (_, L, s, m, K) in zip(xs, specs)])
    torch.cuda.synchronize()
    for x, o, (_, L, s, m, K) in zip(xs, outs, specs):
        alone = llf().run(x, L, s, m, K)
        torch.cuda.synchronize()
        assert torch.equal(alone, o)
        want = oracle_run(x.cpu().numpy(), L, s, m, K)
        assert ref.max_abs(o.cpu().numpy(), want) <= TOL_F32


def test_small_workspace_is_rejected_before_launch(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd import fllf
    ctx = llf()
    x = torch.from_numpy(_img(64, 64)).cuda()
    out = torch.full_like(x, -7.0)
    fj, _ = ctx._prepare(fllf.Job(x, 4, 0.2, 2.0, 4, out=out))
    need = ctx.workspace_size([fj])
    ws = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(fllf.FourierLLFError) as e:
        ctx.run_jobs([fj], workspace=ws)
    assert e.value.status == fllf.FLLF_ENOMEM
    torch.cuda.synchronize()
    assert bool((out == -7.0).all())


def test_input_inside_the_workspace_is_rejected(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd import fllf
    ctx = llf()
    h, w = 64, 64
    probe = fllf.make_job(0x1000, 0x100000000, w, h, 1, 4, 0.2, 2.0, 4)
    need = ctx.workspace_size([probe])
    ws = torch.empty(need + h * w * 4, dtype=torch.uint8, device="cuda")
    x = ws[:h * w * 4].view(torch.float32).view(1, h, w)  # the input lives in the workspace
    x.copy_(torch.from_numpy(_img(h, w)).cuda())
    out = torch.full_like(x, -3.0)
    fj, _ = ctx._prepare(fllf.Job(x, 4, 0.2, 2.0, 4, out=out))
    with pytest.raises(fllf.FourierLLFError) as e:
        ctx.run_jobs([fj], workspace=ws)
    assert e.value.status == fllf.FLLF_EINVAL and "input overlaps" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == -3.0).all())


@pytest.mark.parametrize("L", [2, 3, 4])
def test_fused_level1_shallow_pyramids(torch_dev, L):
    """1500x1100 RGB: level 1 takes the fused form.  With 3 levels, level 2 is
    the top and up(0) folds in the collapse from G_2; with 2 levels, level 1
    is the top and nothing is fused."""
    img = _img(1100, 1500, c=3, seed=40 + L)
    got = gpu_run(torch_dev, img, L, 0.15, 2.5, 8)
    want = oracle_channels(img, L, 0.15, 2.5, 8)
    errs, _ = report(f"1500x1100 RGB, {L} levels", got, want)
    assert max(errs) <= TOL_F32


@pytest.mark.parametrize("h,w", [(65536, 4), (4, 65536)])
def test_fused_levels_on_thin_images(torch_dev, h, w):
    """16 channels, 4 samples across at the 65536-sample side limit: level 1 is
    2 wide with 2^20 samples over the channels (fused: at least 2^19) and level 2
    one sample: the fused level-1 pass with one strip or over a thousand, the
    folded collapse reading a one-sample level 2.  Every channel against the oracle."""
    img = _img(h, w, c=16, seed=h % 97 + w % 89)
    got = gpu_run(torch_dev, img, 3, 0.2, 2.0, 4)
    want = oracle_channels(img, 3, 0.2, 2.0, 4)
    errs, _ = report(f"{w}x{h}, 16 channels", got, want)
    assert max(errs) <= TOL_F32


@pytest.mark.parametrize("storage,tol", [("f32", TOL_F32), ("f16", TOL_F16)])
@pytest.mark.parametrize("w", [961, 963, 966])
def test_fused_level1_last_strip_widths(torch_dev, w, storage, tol):
    """800 x w RGB, level 1 fused: its last strip holds 5, 6 or 7 in-bounds fine
    columns (w = 961, 963, 966), on both sides of the 6 from which a border strip
    reads its record rows as a span and picks the folded columns (below it the
    records are loaded per lane).  Every channel against the oracle."""
    img = _img(800, w, c=3, seed=w)
    got = gpu_run(torch_dev, img, 5, 0.15, 2.5, 8, storage=storage)
    want = oracle_channels(img, 5, 0.15, 2.5, 8)
    errs, _ = report(f"800x{w} RGB, {storage}", got, want)
    assert max(errs) <= tol
