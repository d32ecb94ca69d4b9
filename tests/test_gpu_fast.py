"""GPU parity of the fast LLF comparator (Sec. II-C; FLLF_FLAG_FAST_LLF): the
library's kernels with the sampled remaps r(I, tau j) in place of the Fourier
pairs, against the FP64 oracle's fast_llf element by element (every channel),
at sizes that span several strips and ragged tails, sample counts from 2 to 32,
and reduced-precision storage; plus its degenerate cases."""
import numpy as np
import pytest

from oracle import fourier_llf_ref as ref
from paper_2206_04681_amd.synth import synth_image

pytestmark = pytest.mark.gpu


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


def oracle(img, L, sigma, m, n):
    remap = lambda i, g: ref.remap_exact(i, g, sigma, m)
    img = np.asarray(img, dtype=np.float64)
    return np.stack([ref.fast_llf(c, L, remap, n) for c in img])


@pytest.mark.parametrize("c,h,w,L,n,sigma,m", [
    (1, 64, 64, 5, 8, 0.2, 2.0), (1, 70, 45, 4, 4, 0.15, 3.0), (1, 129, 97, 6, 16, 0.1, 2.0),
    (1, 33, 17, 3, 2, 0.2, 2.0), (1, 5, 9, 3, 6, 0.3, -1.0), (3, 300, 400, 7, 12, 30 / 256, 2.0),
    (2, 151, 260, 6, 32, 0.12, 2.5), (1, 2, 2, 2, 10, 0.2, 2.0)])
def test_fast_llf_against_oracle(torch_dev, c, h, w, L, n, sigma, m):
    torch = torch_dev
    img = synth_image(h, w, c, seed=h + 3 * w + n)
    out = llf().run_fast(torch.from_numpy(img).cuda(), L, sigma, m, n)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(c, h, w)
    want = oracle(img, L, sigma, m, n)
    errs = [ref.max_abs(got[i], want[i]) for i in range(c)]
    print(f"\nfast LLF {c}x{h}x{w}, {L} levels, n={n}: max-abs per channel {['%.2e' % e for e in errs]}")
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("storage,tol", [("f16", 1e-3), ("bf16", 8e-3)])
def test_fast_llf_reduced_storage(torch_dev, storage, tol):
    torch = torch_dev
    img = synth_image(200, 260, 1, seed=3)
    out = llf(storage).run_fast(torch.from_numpy(img).cuda(), 6, 0.15, 2.0, 8)
    torch.cuda.synchronize()
    want = oracle(img, 6, 0.15, 2.0, 8)[0]
    got = out.cpu().numpy()[0]
    assert ref.max_abs(got, want) <= tol
    assert ref.psnr(got, want) >= (70.0 if storage == "f16" else 55.0)


def test_fast_llf_degenerate_cases(torch_dev):
    torch = torch_dev
    # a constant image is fixed (every Laplacian level of a constant is zero)
    x = torch.full((1, 40, 50), 0.375, device="cuda")
    out = llf().run_fast(x, 5, 0.2, 3.0, 8)
    torch.cuda.synchronize()
    assert float((out - 0.375).abs().max()) <= 1e-6
    # m = 0: every sampled remap is the identity, the output is the input
    img = torch.from_numpy(synth_image(77, 91, 1, seed=8)).cuda()
    out = llf().run_fast(img, 5, 0.2, 0.0, 6)
    torch.cuda.synchronize()
    assert float((out - img).abs().max()) <= 1e-5
    # one level: the output is the input
    out = llf().run_fast(img, 1, 0.2, 3.0, 6)
    torch.cuda.synchronize()
    assert torch.equal(out, img)


def test_fast_llf_rejections(torch_dev):
    from paper_2206_04681_amd import fllf
    torch = torch_dev
    img = torch.from_numpy(synth_image(40, 40, 1, seed=1)).cuda()
    for n in (3, 1, 34):
        with pytest.raises(fllf.FourierLLFError) as e:
            llf().run_fast(img, 4, 0.2, 2.0, n)
        assert e.value.status == fllf.FLLF_EINVAL
