"""GPU tests of the serving form (continuous batching over a device arena):
every result equals the same job run alone, whatever arrives around it;
admission never exceeds the arena; oversized jobs are refused up front."""
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


# (channels, height, width), levels, sigma_r, m, K
REQS = [((3, 240, 320), 7, 0.1, 2.0, 8), ((1, 100, 130), 6, 0.2, 2.0, 4),
        ((3, 480, 640), 7, 0.3, 2.0, 16), ((1, 33, 47), 5, 0.05, 3.0, 8),
        ((3, 200, 300), 6, 0.15, -1.0, 5), ((1, 1, 1), 1, 0.2, 2.0, 4),
        ((3, 360, 480), 7, 0.25, 2.0, 4), ((1, 512, 512), 6, 0.2, 2.0, 4),
        ((3, 129, 257), 8, 0.12, 2.0, 16), ((1, 64, 64), 7, 0.2, 1.0, 8),
        ((3, 300, 200), 6, 0.08, 2.0, 8), ((1, 700, 90), 7, 0.2, 2.0, 32),
        # large enough for the fused form at level 1 (the second with float16 pairs only)
        ((3, 1100, 1500), 7, 0.12, 2.0, 8), ((1, 2200, 2000), 8, 0.2, 2.0, 16)]
# step index at which each request arrives: several join while others are mid-flight
ARRIVE = [0, 0, 1, 3, 3, 4, 6, 9, 9, 10, 15, 22, 2, 12]


def _inputs(torch, seed):
    hosts = []
    for i, ((c, h, w), *_rest) in enumerate(REQS):
        hosts.append(torch.from_numpy(synth_image(h, w, c, seed=seed + i)).pin_memory())
    return hosts


def _serve(torch, storage, arena_bytes, hosts, max_active=64):
    """Drive a server: uploads on a side stream, submits at their arrival
    step, steps until everything is reported.  Returns outputs and stats."""
    from paper_2206_04681_amd.fllf import FourierLLF, Job, Server
    llf = FourierLLF(storage)
    srv = Server(llf, arena_bytes, max_active=max_active)
    side = torch.cuda.Stream()
    outs, done, step, peak_queued = {}, set(), 0, 0
    try:
        while len(done) < len(REQS):
            for i, a in enumerate(ARRIVE):
                if a == step:
                    with torch.cuda.stream(side):
                        x = hosts[i].to("cuda", non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(side)
                    _, L, s, m, K = REQS[i]
                    outs[i] = (x, srv.submit(Job(x, L, s, m, K), tag=i, ready_event=ev))
            srv.step()
            peak_queued = max(peak_queued, srv.stats()["queued"])
            done.update(srv.poll())
            step += 1
            assert step < 10000, "server made no progress"
        torch.cuda.synchronize()
        stats = srv.stats()
    finally:
        srv.close()
    return outs, stats, peak_queued, llf


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mix_equals_alone(torch_dev, storage):
    torch = torch_dev
    hosts = _inputs(torch, 500)
    outs, stats, _, llf = _serve(torch, storage, 1 << 30, hosts)
    assert stats["completed"] == len(REQS)
    assert stats["arena_used"] == 0 and 0 < stats["arena_peak"] <= stats["arena_bytes"]
    assert stats["active"] == stats["queued"] == stats["finishing"] == 0
    # every pass of every job was enqueued once; jobs in flight together shared
    # steps and launches (continuous batching, not a queue)
    assert stats["passes"] == sum(1 if L == 1 else 2 * (L - 1) for _, L, *_ in REQS)
    assert stats["max_step_jobs"] >= 3
    assert stats["launches"] < stats["passes"]
    for i, (x, o) in outs.items():
        _, L, s, m, K = REQS[i]
        alone = llf.run(x, L, s, m, K)
        torch.cuda.synchronize()
        assert torch.equal(alone, o), i
    if storage == "f32":
        for i in (1, 3, 5, 9):
            x, o = outs[i]
            _, L, s, m, K = REQS[i]
            want = ref.fourier_llf_image(x.cpu().numpy().astype(np.float64), L, s, m, K)
            assert ref.max_abs(o.cpu().numpy(), want) <= 1e-4, i


def test_small_arena_queues_and_stays_within_budget(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd import fllf
    hosts = _inputs(torch, 600)
    # room for the largest workspace and a little more: jobs must wait their turn
    fps = []
    for (c, h, w), L, s, m, K in REQS:
        j = fllf.make_job(0x1000, 0x100000000, w, h, c, L, s, m, K)
        fps.append(fllf.footprint([j], "f32"))
    arena = max(fps) + max(fps) // 2 + (8 << 20)
    outs, stats, peak_queued, llf = _serve(torch, "f32", arena, hosts)
    assert stats["completed"] == len(REQS)
    assert stats["arena_peak"] <= stats["arena_bytes"]
    assert peak_queued > 0
    for i, (x, o) in outs.items():
        _, L, s, m, K = REQS[i]
        alone = llf.run(x, L, s, m, K)
        torch.cuda.synchronize()
        assert torch.equal(alone, o), i


def test_max_active_one_serialises(torch_dev):
    torch = torch_dev
    hosts = _inputs(torch, 700)
    outs, stats, peak_queued, llf = _serve(torch, "f32", 1 << 30, hosts, max_active=1)
    assert stats["completed"] == len(REQS) and peak_queued > 0
    assert stats["max_step_jobs"] == 1
    for i, (x, o) in outs.items():
        _, L, s, m, K = REQS[i]
        assert torch.equal(llf.run(x, L, s, m, K), o), i


def test_oversized_job_is_refused(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd.fllf import FourierLLF, FourierLLFError, Job, Server, FLLF_ENOMEM
    llf = FourierLLF("f32")
    srv = Server(llf, 64 << 20, max_active=8)
    try:
        big = torch.zeros(3, 1080, 1920, device="cuda")
        with pytest.raises(FourierLLFError) as e:
            srv.submit(Job(big, 8, 0.1, 2.0, 8), tag=1)
        assert e.value.status == FLLF_ENOMEM
        small = torch.from_numpy(synth_image(64, 80, 1, seed=3)).cuda()
        out = srv.submit(Job(small, 5, 0.2, 2.0, 4), tag=2)
        done = []
        for _ in range(100):
            srv.step()
            done += srv.poll()
            if done:
                break
        assert done == [2]
        torch.cuda.synchronize()
        assert torch.equal(llf.run(small, 5, 0.2, 2.0, 4), out)
    finally:
        srv.close()


def test_images_inside_the_arena_are_refused(torch_dev):
    torch = torch_dev
    from paper_2206_04681_amd.fllf import FourierLLF, FourierLLFError, Job, Server, FLLF_EINVAL
    llf = FourierLLF("f32")
    srv = Server(llf, 64 << 20, max_active=4)
    try:
        x = srv.arena[-(64 * 80 * 4):].view(torch.float32).view(1, 64, 80)  # input inside the arena
        with pytest.raises(FourierLLFError) as e:
            srv.submit(Job(x, 5, 0.2, 2.0, 4), tag=1)
        assert e.value.status == FLLF_EINVAL
    finally:
        srv.close()


def test_maps_and_views_in_a_served_mix(torch_dev):
    """Jobs with per-pixel boost and range-scale maps and strided input views,
    served together with plain jobs: each equals the same job run alone; fast
    LLF jobs are refused (single runs only)."""
    torch = torch_dev
    from paper_2206_04681_amd.fllf import (FourierLLF, FourierLLFError, Job, Server, FLLF_EUNSUPPORTED,
                                           FLLF_FLAG_FAST_LLF)
    llf = FourierLLF("f32")
    srv = Server(llf, 1 << 30, max_active=16)
    big = torch.from_numpy(synth_image(700, 900, 3, seed=41)).cuda()
    yy, xx = np.mgrid[0:300, 0:400]
    smap = torch.from_numpy((0.08 + 0.2 * xx / 399).astype(np.float32)).cuda()
    mmap = torch.from_numpy((1.0 + 2.0 * yy / 299).astype(np.float32)).cuda()
    jobs = [Job(big[:, 100:400, 200:600], 7, 0.08, 2.0, 8, sigma_map=smap, sigma_max=0.28),
            Job(big[1, 50:350, 0:400], 6, 0.2, 0.0, 4, m_map=mmap),
            Job(big[:, 0:300, 500:900], 6, 0.08, 0.0, 16, m_map=mmap, sigma_map=smap, sigma_max=0.28),
            Job(big, 8, 0.1, 3.0, 8),
            Job(big[2], 7, 0.15, 2.0, 5)]
    try:
        outs = [srv.submit(j, tag=i) for i, j in enumerate(jobs)]
        done = set()
        for _ in range(10000):
            srv.step()
            done.update(srv.poll())
            if len(done) == len(jobs):
                break
        assert len(done) == len(jobs)
        torch.cuda.synchronize()
        for j, o in zip(jobs, outs):
            alone = llf.run(j.x, j.levels, j.sigma_r, j.m, j.K, m_map=j.m_map, sigma_map=j.sigma_map,
                            sigma_max=j.sigma_max)
            torch.cuda.synchronize()
            assert torch.equal(alone, o)
        fj, _ = llf._prepare(Job(big[0], 5, 0.2, 2.0, 8))
        fj.flags = FLLF_FLAG_FAST_LLF
        from paper_2206_04681_amd.fllf import lib
        import ctypes
        st = lib().fourier_llf_server_submit(srv._s, ctypes.byref(fj), 99, None)
        assert st == FLLF_EUNSUPPORTED
    finally:
        srv.close()
