"""A host program (tests/c_client.cpp, built by __graft_entry__.build()) that uses
the library through its C interface only: argument and error handling on the
CPU, and on the GPU its output against the FP64 oracle."""
import os
import subprocess

import numpy as np
import pytest

from oracle import fourier_llf_ref as ref
from paper_2206_04681_amd.synth import synth_image

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_client")


def _run(args, timeout=120):
    assert os.path.exists(EXE), "tests/c_client is built by __graft_entry__.build()"
    return subprocess.run([EXE] + [str(a) for a in args], capture_output=True, text=True, timeout=timeout)


def _has_gpu():
    import torch
    return torch.cuda.device_count() > 0  # counts devices without initialising one


def test_c_client_rejects_bad_arguments():
    r = _run(["only", "two"])
    assert r.returncode == 2 and "usage" in r.stderr
    r = _run(["/nonexistent/in.bin", "/tmp/out.bin", 8, 8, 1, 3, 0.2, 2.0, 4, "f32"])
    assert r.returncode == 2 and "cannot read" in r.stderr
    r = _run(["/nonexistent/in.bin", "/tmp/out.bin", 8, 8, 1, 3, 0.2, 2.0, 4, "f64"])
    assert r.returncode == 2 and "unknown storage" in r.stderr


@pytest.mark.skipif(_has_gpu(), reason="checks the report of a missing device")
def test_c_client_reports_missing_device(tmp_path):
    src = tmp_path / "in.bin"
    np.zeros((1, 8, 8), np.float32).tofile(src)
    r = _run([src, tmp_path / "out.bin", 8, 8, 1, 3, 0.2, 2.0, 4, "f32"])
    assert r.returncode == 3 and "status -3" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("storage,tol", [("f32", 1e-4), ("f16", 2e-4)])
def test_c_client_against_oracle(tmp_path, storage, tol):
    c, h, w, L, sigma, m, K = 3, 200, 300, 6, 0.15, 2.0, 8
    img = synth_image(h, w, c, seed=7)
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    img.astype(np.float32).tofile(src)
    print(f"c_client {w}x{h}x{c} L={L} K={K} {storage}", flush=True)
    r = _run([src, dst, w, h, c, L, sigma, m, K, storage])
    assert r.returncode == 0, r.stderr
    got = np.fromfile(dst, dtype=np.float32).reshape(c, h, w)
    want = ref.fourier_llf_image(img.astype(np.float64), L, sigma, m, K)
    assert ref.max_abs(got, want) <= tol


@pytest.mark.gpu
def test_c_client_reports_library_errors(tmp_path):
    src = tmp_path / "in.bin"
    np.zeros((1, 16, 16), np.float32).tofile(src)
    r = _run([src, tmp_path / "out.bin", 16, 16, 1, 3, 0.2, 2.0, 40, "f32"])  # K above the maximum
    assert r.returncode == 3 and "status -1" in r.stderr
