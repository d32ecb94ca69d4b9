"""GPU tests of re-parameterisation from resident pyramids: a new boost m and/or
range scale sigma_r with the period T kept, computed from the pyramids a
previous run left in its workspace, against a full run with the new parameters
(and that T) and against the FP64 oracle."""
import numpy as np
import pytest

from oracle import fourier_llf_ref as ref
from oracle_pool import oracle_channels, report
from paper_2206_04681_amd.synth import synth_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _setup(torch, storage, shape=(3, 300, 400), L=7, K=8, sigma=0.1, m=3.0, seed=5):
    from paper_2206_04681_amd import fllf
    ctx = fllf.FourierLLF(storage)
    x = torch.from_numpy(synth_image(shape[1], shape[2], shape[0], seed=seed)).cuda()
    out = torch.empty_like(x)
    prev, _ = ctx._prepare(fllf.Job(x, L, sigma, m, K, out=out))
    ws = torch.empty(ctx.workspace_size([prev]), dtype=torch.uint8, device="cuda")
    ctx.run_jobs([prev], workspace=ws)
    T = fllf.fit(sigma, K)[0]
    return fllf, ctx, x, prev, ws, T


def _full(torch, fllf, storage, x, L, sigma, m, K, T):
    return fllf.FourierLLF(storage).run(x, L, sigma, m, K, T=T)


@pytest.mark.parametrize("sigma2,m2", [(0.15, 2.0), (0.1, -1.5), (0.06, 4.0)])
def test_reparam_matches_full_run(torch_dev, sigma2, m2):
    torch = torch_dev
    fllf, ctx, x, prev, ws, T = _setup(torch, "f32")
    out2 = torch.full_like(x, -9.0)
    nxt, _ = ctx._prepare(fllf.Job(x, 7, sigma2, m2, 8, out=out2))
    ctx.reparam(prev, nxt, ws)
    full = _full(torch, fllf, "f32", x, 7, sigma2, m2, 8, T)
    torch.cuda.synchronize()
    assert float((out2 - full).abs().max()) <= 2e-5
    want = ref.fourier_llf_image(x.cpu().numpy().astype(np.float64), 7, sigma2, m2, 8, T=T)
    assert ref.max_abs(out2.cpu().numpy(), want) <= 1e-4


def test_reparam_chain_from_same_pyramids(torch_dev):
    torch = torch_dev
    fllf, ctx, x, prev, ws, T = _setup(torch, "f32", shape=(1, 257, 129), L=6, K=16, sigma=0.2, m=2.0)
    for sigma2, m2 in [(0.25, 1.0), (0.12, 3.0), (0.2, 2.0)]:
        out2 = torch.empty_like(x)
        nxt, _ = ctx._prepare(fllf.Job(x, 6, sigma2, m2, 16, out=out2))
        ctx.reparam(prev, nxt, ws)
        torch.cuda.synchronize()
        want = ref.fourier_llf_image(x.cpu().numpy().astype(np.float64), 6, sigma2, m2, 16, T=T)
        assert ref.max_abs(out2.cpu().numpy(), want) <= 1e-4, (sigma2, m2)


def test_reparam_after_a_fused_run(torch_dev):
    """1500x1100 RGB: the first run takes the fused form at level 1; the
    re-parameterised passes read the same resident pyramids."""
    torch = torch_dev
    fllf, ctx, x, prev, ws, T = _setup(torch, "f32", shape=(3, 1100, 1500), L=7, K=8, sigma=0.12, m=2.0)
    out2 = torch.empty_like(x)
    nxt, _ = ctx._prepare(fllf.Job(x, 7, 0.2, 3.0, 8, out=out2))
    ctx.reparam(prev, nxt, ws)
    full = _full(torch, fllf, "f32", x, 7, 0.2, 3.0, 8, T)
    torch.cuda.synchronize()
    assert float((out2 - full).abs().max()) <= 2e-5
    want = oracle_channels(x.cpu().numpy(), 7, 0.2, 3.0, 8, T=T)
    errs, _ = report("re-parameterised 1500x1100 RGB", out2.cpu().numpy(), want)
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("storage,tol", [("f16", 2e-4), ("bf16", 2e-3)])
def test_reparam_reduced_storage(torch_dev, storage, tol):
    torch = torch_dev
    fllf, ctx, x, prev, ws, T = _setup(torch, storage, K=4, sigma=0.2, m=2.0)
    out2 = torch.empty_like(x)
    nxt, _ = ctx._prepare(fllf.Job(x, 7, 0.25, 1.5, 4, out=out2))
    ctx.reparam(prev, nxt, ws)
    torch.cuda.synchronize()
    want = ref.fourier_llf_image(x.cpu().numpy().astype(np.float64), 7, 0.25, 1.5, 4, T=T)
    assert ref.max_abs(out2.cpu().numpy(), want) <= tol


def test_reparam_rejects_mismatches(torch_dev):
    torch = torch_dev
    fllf, ctx, x, prev, ws, T = _setup(torch, "f32", shape=(1, 64, 80), L=5, K=8)
    out2 = torch.empty_like(x)
    cases = [(dict(K=4), fllf.FLLF_EINVAL), (dict(levels=4), fllf.FLLF_EINVAL),
             (dict(T=T * 1.01), fllf.FLLF_EINVAL)]
    for kw, status in cases:
        args = dict(levels=5, K=8, T=0.0)
        args.update(kw)
        nxt, _ = ctx._prepare(fllf.Job(x, args["levels"], 0.15, 2.0, args["K"], T=args["T"], out=out2))
        with pytest.raises(fllf.FourierLLFError) as e:
            ctx.reparam(prev, nxt, ws)
        assert e.value.status == status, kw
    # K = 5 pyramids cannot be re-parameterised
    _, ctx5, x5, prev5, ws5, _ = _setup(torch, "f32", shape=(1, 64, 80), L=5, K=5)
    nxt5, _ = ctx5._prepare(fllf.Job(x5, 5, 0.15, 2.0, 5, out=torch.empty_like(x5)))
    with pytest.raises(fllf.FourierLLFError) as e:
        ctx5.reparam(prev5, nxt5, ws5)
    assert e.value.status == fllf.FLLF_EUNSUPPORTED
