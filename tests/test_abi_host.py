"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
declared entry point, and its validation, float64 fit and footprint agree with
the oracle and the documented layout."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import fourier_llf_ref as ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fourier_llf.h")


@pytest.fixture(scope="session")
def F():
    from paper_2206_04681_amd import fllf
    if not os.path.exists(fllf.LIB_PATH):
        from paper_2206_04681_amd import build
        build.build()
    fllf.lib()
    return fllf


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fourier_llf_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(F):
    names = _declared()
    assert len(names) >= 9
    raw = ctypes.CDLL(F.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(F.EXPORTED)


@pytest.mark.parametrize("sigma,K,R", [(0.2, 4, 1.0), (0.1, 8, 1.0), (0.1, 16, 1.0), (0.05, 32, 1.0),
                                       (0.3, 1, 1.0), (30.0, 10, 256.0)])
def test_fit_matches_oracle(F, sigma, K, R):
    T, om, at = F.fit(sigma, K, R)
    Tr = ref.fit_period(sigma, K, R)
    assert abs(T - Tr) / Tr < 1e-7
    omr, _, atr, _ = ref.fourier_coefficients(sigma, K, T)
    np.testing.assert_allclose(om, omr, rtol=1e-13)
    np.testing.assert_allclose(at, atr, rtol=1e-12, atol=1e-300)


def test_fit_given_period_is_used(F):
    T, om, _ = F.fit(30.0, 10, 256.0, 405.9)
    assert T == 405.9 and abs(om[0] - 2 * math.pi / 405.9) < 1e-15


@pytest.mark.parametrize("h,w", [(1, 1), (2, 2), (3, 9), (512, 512), (2160, 3840), (33, 4097), (70000, 70000)])
def test_max_levels(F, h, w):
    assert F.max_levels(h, w) == min(ref.max_levels(h, w), F.FLLF_MAX_LEVELS)


def _job(F, **kw):
    base = dict(in_ptr=0x1000, out_ptr=0x100000000, width=64, height=48, channels=1, levels=4,
                sigma_r=0.2, m=2.0, K=4)
    base.update(kw)
    return F.make_job(**base)


def test_validate_accepts_good_job(F):
    assert F.validate([_job(F)]) == F.FLLF_OK
    other = dict(in_ptr=0x200000000, out_ptr=0x300000000)
    assert F.validate([_job(F), _job(F, width=3, height=2, levels=2, K=32, **other)], "bf16") == F.FLLF_OK


def test_validate_rejects_batch_overlap(F):
    # a batch where one job writes into another job's input or output
    assert F.validate([_job(F), _job(F, in_ptr=0x200000000)]) == F.FLLF_EINVAL
    assert "overlaps" in F.last_error()
    assert F.validate([_job(F), _job(F, out_ptr=0x200000000, in_ptr=0x100000000 + 64)]) == F.FLLF_EINVAL


@pytest.mark.parametrize("bad", [
    dict(in_ptr=0), dict(out_ptr=0), dict(width=0), dict(height=-1), dict(channels=0),
    dict(levels=0), dict(levels=7), dict(K=0), dict(K=33), dict(sigma_r=0.0), dict(sigma_r=float("nan")),
    dict(m=float("inf")), dict(R=0.0), dict(T=0.5), dict(T=float("nan")),
    dict(out_ptr=0x1000 + 64 * 48 * 4 - 4),  # overlaps in
])
def test_validate_rejects(F, bad):
    assert F.validate([_job(F, **bad)]) == F.FLLF_EINVAL
    assert F.last_error()


def test_validate_rejects_bad_storage_and_empty(F):
    assert F.lib().fourier_llf_validate(F._job_array([_job(F)]), 1, 7) == F.FLLF_EINVAL
    assert F.lib().fourier_llf_validate(F._job_array([_job(F)]), 0, 0) == F.FLLF_EINVAL


def _expected_footprint(w, h, C, L, K, pair_bytes, has_map=False):
    al = lambda x: (x + 255) // 256 * 256
    tot = 0
    for l in range(1, L):
        wl, hl = -(-w // 2 ** l), -(-h // 2 ** l)
        n = (wl + 63) // 64 * 64 * hl  # rows padded to 64 elements
        tot += al(4 * n) * C + al(pair_bytes * n * K) * C  # K pairs per pixel record
        if l < L - 1:
            tot += al(4 * n) * C + (al(4 * n) if has_map else 0)
    return tot


@pytest.mark.parametrize("storage,pb", [("f32", 8), ("f16", 4), ("bf16", 4)])
def test_footprint_matches_layout(F, storage, pb):
    j = _job(F, width=3840, height=2160, channels=3, levels=8, K=8)
    assert F.footprint([j], storage) == _expected_footprint(3840, 2160, 3, 8, 8, pb)
    j2 = _job(F, width=1001, height=777, channels=1, levels=5, K=3, m_map_ptr=0x5000,
              in_ptr=0x200000000, out_ptr=0x300000000)
    assert F.footprint([j2], storage) == _expected_footprint(1001, 777, 1, 5, 3, pb, True)
    # two jobs: both workspaces plus the batch launch table in front of them
    table = F.footprint([j, j2], storage) - (_expected_footprint(3840, 2160, 3, 8, 8, pb)
                                             + _expected_footprint(1001, 777, 1, 5, 3, pb, True))
    assert table > 0 and table % 256 == 0 and table < 2 * 32 * 1024


def test_footprint_of_4k_rgb_k8(F):
    # levels >= 1 hold ~N/3 pixels per channel: (4 + 2K*4 + 4) bytes each with float32
    # pyramids (~0.6 GB), (4 + 2K*2 + 4) with 16-bit ones (~0.33 GB)
    j = _job(F, width=3840, height=2160, channels=3, levels=8, K=8)
    assert 0.55e9 < F.footprint([j], "f32") < 0.65e9
    assert 0.30e9 < F.footprint([j], "f16") < 0.36e9


def test_create_without_device_reports_edevice(F):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    st = F.lib().fourier_llf_create(ctypes.byref(ctx), 0, 0)
    assert st == F.FLLF_EDEVICE and not ctx.value
    assert "device" in F.last_error()


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2206_04681_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in txt.replace("oracle-free", ""), fn


def test_struct_mirrors_match_the_header(F):
    # fllf_job: 2 pointers, 6 int32, 4 doubles, 1 pointer, 4 int64, 1 pointer, 1 double;
    # fllf_server_stats: 4 int32, 4 int64, 2 int32, 3 uint64; fllf_kernel_time:
    # char[32], int32, 2 doubles
    assert ctypes.sizeof(F.FllfJob) == 2 * 8 + 6 * 4 + 4 * 8 + 8 + 4 * 8 + 8 + 8
    assert ctypes.sizeof(F.FllfServerStats) == 4 * 4 + 4 * 8 + 2 * 4 + 3 * 8
    assert ctypes.sizeof(F.FllfKernelTime) == 32 + 4 + 4 + 2 * 8


def test_validate_rejects_record_planes_past_32bit_offsets(F):
    # kernels address one channel's level-1 record plane with 32-bit byte offsets:
    # 16384 x 16384, K = 8 needs 8192 x 8192 x 8 pairs x 8 bytes = 4 GiB in float32
    big = dict(width=16384, height=16384, levels=2, K=8, out_ptr=0x10000000000)
    assert F.validate([_job(F, **big)], "f32") == F.FLLF_EINVAL
    assert "4 GiB" in F.last_error()
    # the same image with 16-bit pairs (2 GiB) is accepted
    assert F.validate([_job(F, **big)], "f16") == F.FLLF_OK


# --- strided images: row and plane pitches (0 = dense) ---------------------------

def test_validate_accepts_strided_views(F):
    # a crop of a 3 x 100 x 90 tensor (rows of 90, planes of 9000) into a dense output
    assert F.validate([_job(F, channels=3, pitches=(90, 9000, 0, 0))]) == F.FLLF_OK
    # output rows inside a wider tensor; row-interleaved output channels (an H x C x W tensor viewed as C x H x W)
    assert F.validate([_job(F, channels=3, pitches=(0, 0, 200, 200 * 48))]) == F.FLLF_OK
    assert F.validate([_job(F, channels=3, pitches=(0, 0, 3 * 64, 64))]) == F.FLLF_OK
    # any input plane pitch is fine (the input is only read), even planes that share rows
    assert F.validate([_job(F, channels=3, pitches=(64, 64, 0, 0))]) == F.FLLF_OK


@pytest.mark.parametrize("pitches,why", [
    ((63, 0, 0, 0), "pitches"),              # input rows shorter than the image
    ((0, 0, 50, 0), "pitches"),              # output rows shorter than the image
    ((-64, 0, 0, 0), "pitches"),
    ((0, -1, 0, 0), "pitches"),
    ((0, 0, 0, 64 * 47), "overlap"),         # output planes one row too close
    ((0, 0, 2 * 64, 64), "overlap"),         # interleaved output rows too short for 3 channels
])
def test_validate_rejects_bad_pitches(F, pitches, why):
    assert F.validate([_job(F, channels=3, pitches=pitches)]) == F.FLLF_EINVAL
    assert why in F.last_error()


def test_validate_span_of_strided_images(F):
    # with a row pitch of 1000, the input (0x1000 + 4 x (47 x 1000 + 64) bytes) reaches
    # an output placed 100 KB further: overlap; dense it does not
    out = 0x1000 + 100 * 1024
    assert F.validate([_job(F, out_ptr=out)]) == F.FLLF_OK
    assert F.validate([_job(F, out_ptr=out, pitches=(1000, 0, 0, 0))]) == F.FLLF_EINVAL
    assert "overlap" in F.last_error()


def test_validate_rejects_planes_past_32bit_offsets(F):
    # rows of 2^20 elements: 1100 rows exceed the 2^30-element plane limit
    big = dict(width=64, height=1100, levels=2, out_ptr=0x100000000000)
    assert F.validate([_job(F, **big, pitches=(1 << 20, 0, 0, 0))]) == F.FLLF_EINVAL
    assert "2^30" in F.last_error()
    assert F.validate([_job(F, **big, pitches=(1 << 19, 0, 0, 0))]) == F.FLLF_OK


def test_footprint_does_not_depend_on_pitches(F):
    a = F.footprint([_job(F, channels=3)])
    b = F.footprint([_job(F, channels=3, pitches=(100, 10000, 128, 128 * 48))])
    assert a == b


# --- pixel-by-pixel range scale (sigma_map) ---------------------------------------

@pytest.mark.parametrize("lo,hi,K", [(0.05, 0.3, 8), (0.1, 0.2, 4), (0.08, 0.12, 16), (0.15, 0.15, 8)])
def test_fit_range_matches_oracle(F, lo, hi, K):
    T = F.fit_range(lo, hi, K)
    Tr = ref.fit_period_range(lo, hi, K)
    assert abs(T - Tr) / Tr < 1e-7
    if lo == hi:
        assert abs(T - F.fit(lo, K)[0]) <= 1e-12 * T


def test_fit_range_rejects_bad_ranges(F):
    with pytest.raises(F.FourierLLFError):
        F.fit_range(0.2, 0.1, 8)
    with pytest.raises(F.FourierLLFError):
        F.fit_range(0.0, 0.1, 8)


def test_validate_sigma_map(F):
    ok = _job(F, sigma_map_ptr=0x700000000, sigma_max=0.3)
    assert F.validate([ok]) == F.FLLF_OK
    # sigma_max must bound the map from above (sigma_r is its smallest value)
    assert F.validate([_job(F, sigma_map_ptr=0x700000000, sigma_max=0.1)]) == F.FLLF_EINVAL
    assert "sigma_max" in F.last_error()
    # the map must not overlap the output
    assert F.validate([_job(F, sigma_map_ptr=0x100000000 + 64, sigma_max=0.3)]) == F.FLLF_EINVAL


def test_footprint_of_maps(F):
    # each map adds one float32 plane per level 1 .. top-1, shared by the channels
    plain = F.footprint([_job(F, channels=3)])
    one = F.footprint([_job(F, channels=3, m_map_ptr=0x700000000)])
    two = F.footprint([_job(F, channels=3, m_map_ptr=0x700000000, sigma_map_ptr=0x800000000, sigma_max=0.3)])
    assert one > plain and two - one == one - plain


# --- the fast LLF comparator (FLLF_FLAG_FAST_LLF) -----------------------------------

def test_validate_fast_llf_jobs(F):
    fast = dict(flags=F.FLLF_FLAG_FAST_LLF)
    assert F.validate([_job(F, K=8, **fast)]) == F.FLLF_OK
    assert F.validate([_job(F, K=32, **fast)]) == F.FLLF_OK
    for K in (1, 7, 34):  # an even number of samples in [2, 32]
        assert F.validate([_job(F, K=K, **fast)]) == F.FLLF_EINVAL
    assert F.validate([_job(F, K=8, T=2.0, **fast)]) == F.FLLF_EINVAL  # no period
    assert F.validate([_job(F, K=8, m_map_ptr=0x700000000, **fast)]) == F.FLLF_EUNSUPPORTED
    other = dict(in_ptr=0x200000000, out_ptr=0x300000000)
    assert F.validate([_job(F, K=8, **fast), _job(F, **other)]) == F.FLLF_EUNSUPPORTED  # single jobs only
    assert F.validate([_job(F, flags=2)]) == F.FLLF_EINVAL
    assert "flags" in F.last_error()


def test_fast_llf_footprint_is_that_of_half_as_many_terms(F):
    # n samples are stored as n / 2 pairs: the footprint of a Fourier job with K = n / 2
    a = F.footprint([_job(F, K=12, flags=F.FLLF_FLAG_FAST_LLF)])
    b = F.footprint([_job(F, K=6)])
    assert a == b


def test_binding_pitches_of_views(F):
    torch = pytest.importorskip("torch")
    x = torch.zeros(3, 100, 90)
    assert F._pitches(x) == (90, 9000)
    assert F._pitches(x[:, 10:60, 5:80]) == (90, 9000)
    assert F._pitches(x[1, 10:60, 5:80]) == (90, 0)
    assert F._pitches(x.permute(1, 0, 2)[:, :3, :].permute(1, 0, 2)) == (90, 9000)
    assert F._pitches(torch.zeros(100, 3, 90).permute(1, 0, 2)) == (270, 90)   # row-interleaved channels
    with pytest.raises(ValueError):
        F._pitches(x[:, :, ::2])                                     # rows not contiguous
    with pytest.raises(ValueError):
        F._pitches(torch.zeros(100, 90).expand(3, 100, 90))           # channels share their memory
    with pytest.raises(ValueError):
        F._pitches(torch.zeros(1, 90).expand(100, 90))                # rows share their memory
