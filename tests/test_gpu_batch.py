"""GPU tests of the batched form (one launch per pass over many jobs), of the
persistent grid cap, of captured schedules (HIP graphs) and of the autotuner.
Every batched result is compared with the single-job run of the same job (bit
for bit: the same wave bodies run the same arithmetic) and, where cheap, with
the FP64 oracle."""
import numpy as np
import pytest

from oracle import fourier_llf_ref as ref
from oracle_pool import oracle_channels, report
from paper_2206_04681_amd.synth import batch_workloads, synth_image

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-4


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _ctx(storage="f32"):
    from paper_2206_04681_amd.fllf import FourierLLF
    return FourierLLF(storage)


# (channels, height, width), levels, sigma_r, m, K, with boost map
MIXED = [((1, 200, 150), 6, 0.2, 2.0, 4, False),
         ((3, 64, 99), 5, 0.1, 3.0, 8, False),
         ((1, 31, 257), 4, 0.3, -0.5, 16, False),
         ((1, 1, 1), 1, 0.2, 2.0, 8, False),      # single level: a copy
         ((3, 45, 70), 6, 0.15, 1.5, 5, False),   # guarded K loop
         ((1, 130, 77), 7, 0.1, 2.0, 32, False),
         ((1, 90, 70), 5, 0.2, 0.0, 6, True),     # pixel-adaptive boost
         ((3, 129, 257), 8, 0.25, 2.0, 8, False),
         ((1, 5, 9), 2, 0.2, 2.0, 3, False)]


def _mixed_jobs(torch, ctx, specs=MIXED, seed=0):
    from paper_2206_04681_amd.fllf import Job
    jobs, fjobs, outs = [], [], []
    for i, ((c, h, w), L, s, m, K, use_map) in enumerate(specs):
        x = torch.from_numpy(synth_image(h, w, c, seed=seed + i)).cuda()
        mm = None
        if use_map:
            xx = np.mgrid[0:h, 0:w][1]
            mm = torch.from_numpy((0.5 + 2.5 * xx / max(w - 1, 1)).astype(np.float32)).cuda()
        j = Job(x, L, s, m, K, m_map=mm)
        fj, out = ctx._prepare(j)
        jobs.append(j)
        fjobs.append(fj)
        outs.append(out)
    return jobs, fjobs, outs


def _alone(torch, ctx, job):
    out = ctx.run(job.x, job.levels, job.sigma_r, job.m, job.K, m_map=job.m_map)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_batch_equals_single_runs(torch_dev, storage):
    torch = torch_dev
    ctx = _ctx(storage)
    jobs, fjobs, outs = _mixed_jobs(torch, ctx)
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    for i, (j, o) in enumerate(zip(jobs, outs)):
        assert torch.equal(_alone(torch, ctx, j), o), i
    if storage == "f32":
        for i in (0, 2, 3, 4, 6, 8):
            j, o = jobs[i], outs[i]
            img = j.x.cpu().numpy().astype(np.float64)
            if j.m_map is not None:
                want = ref.fourier_llf_adaptive(img[0] if img.ndim == 3 else img, j.levels, j.sigma_r,
                                                j.m_map.cpu().numpy().astype(np.float64), j.K)
                got = o.cpu().numpy()
                got = got[0] if got.ndim == 3 else got
            else:
                want = ref.fourier_llf_image(img, j.levels, j.sigma_r, j.m, j.K)
                got = o.cpu().numpy()
            assert ref.max_abs(got, want) <= TOL_F32, i


@pytest.mark.parametrize("cap", [1, 2])
def test_persistent_grid_cap(torch_dev, cap):
    torch = torch_dev
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, seed=20)
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    ref_outs = [o.clone() for o in outs]
    for o in outs:
        o.fill_(-1.0)
    # few waves per pass: every wave walks many work items
    ctx.set_tuning([0, 0, 0, 0, cap, -1])
    assert ctx.get_tuning()[4] == cap
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    ctx.set_tuning(None)
    for a, b in zip(ref_outs, outs):
        assert torch.equal(a, b)


def test_graph_replays_match_eager(torch_dev):
    torch = torch_dev
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, seed=40)
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    g = ctx.graph(fjobs)
    other = torch.from_numpy(synth_image(300, 200, 3, seed=99)).cuda()
    try:
        for rep in range(3):
            for o in outs:
                o.zero_()
            # unrelated eager work between replays, on the same stream
            ctx.run(other, 6, 0.1, 2.0, 8)
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(eager, outs)):
                assert torch.equal(a, b), (rep, i)
    finally:
        g.close()


def test_single_job_graph(torch_dev):
    torch = torch_dev
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, specs=MIXED[:1], seed=60)
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    eager = outs[0].clone()
    g = ctx.graph(fjobs)
    try:
        for _ in range(2):
            outs[0].zero_()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(eager, outs[0])
    finally:
        g.close()


def test_autotune_keeps_results(torch_dev):
    torch = torch_dev
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, seed=80)
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    before = [o.clone() for o in outs]
    chosen = ctx.autotune(fjobs, reps=1)
    assert chosen == ctx.get_tuning()
    assert all(v in (512, 1024, 1536, 3072, 6144, 12288, 24576) for v in chosen[:4])
    assert chosen[4] in (0, 1, 2, 4)
    assert 0 <= chosen[5] <= 31
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    for a, b in zip(before, outs):
        assert float((a - b).abs().max()) <= 1e-6


def test_autotune_cache_round_trip(torch_dev, tmp_path):
    torch = torch_dev
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, seed=90)
    path = str(tmp_path / "tuning.txt")
    first = ctx.autotune(fjobs, reps=1, cache=path)  # times, then appends one line
    assert first == ctx.get_tuning()
    assert len(open(path).read().strip().splitlines()) == 1
    ctx.set_tuning(None)
    assert ctx.autotune(fjobs, reps=1, cache=path) == first  # read back, nothing appended
    assert ctx.get_tuning() == first
    assert len(open(path).read().strip().splitlines()) == 1
    # an entry written by hand is honoured; lines that are not entries are skipped
    key = open(path).read().split()[0]
    with open(path, "w") as f:
        f.write("# launch shapes\nnot an entry\n" + f"{key} 1024 2048 3072 6144 2 9\n")
    assert ctx.autotune(fjobs, reps=1, cache=path) == [1024, 2048, 3072, 6144, 2, 9]
    # another job set has another key: timed and appended
    other = ctx.autotune(fjobs[:3], reps=1, cache=path)
    assert len(open(path).read().strip().splitlines()) == 4 and other == ctx.get_tuning()
    ctx.set_tuning(None)


def test_uneven_batch_of_64_full_size(torch_dev):
    """The 64-image uneven batch at full size: batched == single-job runs for every
    image; the two smallest images, and every channel of the largest RGB image
    (fused levels in the batched kernels), against the oracle."""
    torch = torch_dev
    from paper_2206_04681_amd.fllf import Job
    ctx = _ctx()
    ws = batch_workloads()
    xs = [torch.from_numpy(w.image()).cuda() for w in ws]
    jobs = [Job(x, w.levels, w.sigma_r, w.m, w.K) for x, w in zip(xs, ws)]
    prepared = [ctx._prepare(j) for j in jobs]
    ctx.run_jobs([p[0] for p in prepared])
    torch.cuda.synchronize()
    for i, (j, (_, o)) in enumerate(zip(jobs, prepared)):
        assert torch.equal(_alone(torch, ctx, j), o), i
    order = sorted(range(len(ws)), key=lambda i: ws[i].height * ws[i].width * ws[i].channels)
    for i in order[:2]:
        w = ws[i]
        want = ref.fourier_llf_image(xs[i].cpu().numpy().astype(np.float64), w.levels, w.sigma_r, w.m, w.K)
        assert ref.max_abs(prepared[i][1].cpu().numpy(), want) <= TOL_F32, i
    big = max((i for i in range(len(ws)) if ws[i].channels == 3), key=lambda i: ws[i].height * ws[i].width)
    w = ws[big]
    want = oracle_channels(xs[big].cpu().numpy(), w.levels, w.sigma_r, w.m, w.K)
    errs, _ = report(f"batched {w.width}x{w.height} RGB", prepared[big][1].cpu().numpy(), want)
    assert max(errs) <= TOL_F32


def test_batch_with_one_invalid_job_launches_nothing(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd import fllf
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, specs=MIXED[:3], seed=90)
    for o in outs:
        o.fill_(-5.0)
    bad = fllf.make_job(fjobs[1].in_, outs[1].data_ptr(), fjobs[1].width, fjobs[1].height, fjobs[1].channels,
                        fjobs[1].levels, 0.1, 2.0, 40)  # K above the maximum
    ws = torch.empty(ctx.workspace_size(fjobs), dtype=torch.uint8, device="cuda")
    with pytest.raises(fllf.FourierLLFError) as e:
        ctx.run_jobs([fjobs[0], bad, fjobs[2]], workspace=ws)
    assert e.value.status == fllf.FLLF_EINVAL
    torch.cuda.synchronize()
    for o in outs:
        assert bool((o == -5.0).all())


def test_batch_with_fused_jobs_and_a_boost_map(torch_dev):
    """Jobs large enough for the fused levels (one of them with a boost map and
    its level-1 collapse folded into up(0)) batched with small ones: every
    batched result equals its single-job run bit for bit."""
    torch = torch_dev
    specs = [((1, 2200, 2000), 7, 0.2, 2.0, 8, True),   # fused levels 1-2, boost map
             ((3, 1100, 1500), 3, 0.12, 2.0, 8, False),  # fused level 1, level 2 the top
             ((3, 1100, 1500), 6, 0.1, 3.0, 4, False),
             ((1, 90, 70), 5, 0.2, 0.0, 6, True),
             ((3, 64, 99), 5, 0.1, 3.0, 8, False)]
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, specs=specs, seed=120)
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    for i, (j, o) in enumerate(zip(jobs, outs)):
        assert torch.equal(_alone(torch, ctx, j), o), i


def test_results_do_not_depend_on_the_launch_shape(torch_dev):
    """Segment lengths and block shapes change which wave computes which row,
    never the arithmetic of a sample: two very different tunings give the same
    outputs bit for bit (small jobs and fused-size ones, batched)."""
    torch = torch_dev
    specs = MIXED + [((3, 1100, 1500), 6, 0.12, 2.0, 8, False), ((1, 1300, 1700), 7, 0.2, 2.0, 8, True)]
    ctx = _ctx()
    jobs, fjobs, outs = _mixed_jobs(torch, ctx, specs=specs, seed=140)
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    for o in outs:
        o.fill_(-3.0)
    ctx.set_tuning([512, 24576, 512, 512, 0, 31 - ctx.get_tuning()[5]])  # the other store policy too
    ctx.run_jobs(fjobs)
    torch.cuda.synchronize()
    ctx.set_tuning(None)
    for i, (a, b) in enumerate(zip(first, outs)):
        assert torch.equal(a, b), i
