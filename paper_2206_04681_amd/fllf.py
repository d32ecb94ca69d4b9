"""Python binding of libfourier_llf.so (argument marshalling only).

Every step of the filter runs in the library's HIP kernels; PyTorch provides
device memory (inputs, outputs, workspace) and the stream.  Names mirror the C
ABI declared in ``include/fourier_llf.h``.  There is no CPU fallback: if the
library is missing or no device is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfourier_llf.so")

FLLF_OK, FLLF_EINVAL, FLLF_ENOMEM, FLLF_EDEVICE, FLLF_EUNSUPPORTED = 0, -1, -2, -3, -4
FLLF_MAX_K = 32
FLLF_FLAG_FAST_LLF = 1
FLLF_MAX_LEVELS = 16
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}

# Every symbol the public header declares (checked by the CPU test suite).
EXPORTED = ("fourier_llf_create", "fourier_llf_workspace_size", "fourier_llf_run",
            "fourier_llf_destroy", "fourier_llf_last_error", "fourier_llf_fit",
            "fourier_llf_max_levels", "fourier_llf_validate", "fourier_llf_footprint",
            "fourier_llf_version", "fourier_llf_timing_enable", "fourier_llf_timing_read",
            "fourier_llf_set_tuning", "fourier_llf_get_tuning", "fourier_llf_autotune",
            "fourier_llf_graph_create", "fourier_llf_graph_launch", "fourier_llf_graph_destroy",
            "fourier_llf_server_create", "fourier_llf_server_submit", "fourier_llf_server_step",
            "fourier_llf_server_poll", "fourier_llf_server_stats", "fourier_llf_server_destroy",
            "fourier_llf_reparam", "fourier_llf_run_static", "fourier_llf_fit_range",
            "fourier_llf_boost_map", "fourier_llf_autotune_cached")

# Launch-shape parameters (FLLF_TUNE_*): target waves of the REDUCE pass from
# level 0 and from levels >= 1, of the up passes that evaluate the product-sum
# (not the re-parameterised ones), and of the one-plane collapse of the fused
# levels; then the grid cap and the pass kinds with non-temporal stores (bits).
TUNE_NAMES = ("down0", "down", "up0", "up", "grid_cap", "nt_stores")


class FourierLLFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fourier_llf status {status}: {message}")
        self.status = status


class FllfKernelTime(ctypes.Structure):
    """Mirror of ``fllf_kernel_time``."""
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class FllfJob(ctypes.Structure):
    """Mirror of ``fllf_job``."""
    _fields_ = [
        ("in_", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("channels", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("sigma_r", ctypes.c_double),
        ("m", ctypes.c_double),
        ("range_R", ctypes.c_double),
        ("period_T", ctypes.c_double),
        ("m_map", ctypes.c_void_p),
        ("row_pitch", ctypes.c_int64),
        ("plane_pitch", ctypes.c_int64),
        ("out_row_pitch", ctypes.c_int64),
        ("out_plane_pitch", ctypes.c_int64),
        ("sigma_map", ctypes.c_void_p),
        ("sigma_max", ctypes.c_double),
    ]


class FllfServerStats(ctypes.Structure):
    """Mirror of ``fllf_server_stats``."""
    _fields_ = [("queued", ctypes.c_int32), ("active", ctypes.c_int32), ("finishing", ctypes.c_int32),
                ("max_active", ctypes.c_int32), ("steps", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("passes", ctypes.c_int64), ("max_step_jobs", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("arena_bytes", ctypes.c_uint64),
                ("arena_used", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64)]


_LIB = None


def lib() -> ctypes.CDLL:
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_04681_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        jp = ctypes.POINTER(FllfJob)
        L.fourier_llf_create.argtypes = [ctypes.POINTER(vp), i32, i32]
        L.fourier_llf_create.restype = i32
        L.fourier_llf_workspace_size.argtypes = [vp, jp, i32, ctypes.POINTER(sz)]
        L.fourier_llf_workspace_size.restype = i32
        L.fourier_llf_run.argtypes = [vp, jp, i32, vp, sz, vp]
        L.fourier_llf_run.restype = i32
        L.fourier_llf_destroy.argtypes = [vp]
        L.fourier_llf_destroy.restype = None
        L.fourier_llf_last_error.argtypes = [vp]
        L.fourier_llf_last_error.restype = ctypes.c_char_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.fourier_llf_fit.argtypes = [dbl, i32, dbl, dbl, dp, dp, dp]
        L.fourier_llf_fit.restype = i32
        L.fourier_llf_max_levels.argtypes = [i32, i32]
        L.fourier_llf_max_levels.restype = i32
        L.fourier_llf_validate.argtypes = [jp, i32, i32]
        L.fourier_llf_validate.restype = i32
        L.fourier_llf_footprint.argtypes = [jp, i32, i32, ctypes.POINTER(sz)]
        L.fourier_llf_footprint.restype = i32
        L.fourier_llf_timing_enable.argtypes = [vp, i32]
        L.fourier_llf_timing_enable.restype = i32
        L.fourier_llf_timing_read.argtypes = [vp, ctypes.POINTER(FllfKernelTime), i32, ctypes.POINTER(i32)]
        L.fourier_llf_timing_read.restype = i32
        L.fourier_llf_version.argtypes = []
        L.fourier_llf_version.restype = i32
        ip = ctypes.POINTER(ctypes.c_int32)
        L.fourier_llf_set_tuning.argtypes = [vp, ip]
        L.fourier_llf_set_tuning.restype = i32
        L.fourier_llf_get_tuning.argtypes = [vp, ip]
        L.fourier_llf_get_tuning.restype = i32
        L.fourier_llf_autotune.argtypes = [vp, jp, i32, vp, sz, vp, i32, ip]
        L.fourier_llf_autotune.restype = i32
        L.fourier_llf_autotune_cached.argtypes = [vp, jp, i32, vp, sz, vp, i32, ctypes.c_char_p, ip]
        L.fourier_llf_autotune_cached.restype = i32
        L.fourier_llf_graph_create.argtypes = [vp, jp, i32, vp, sz, ctypes.POINTER(vp)]
        L.fourier_llf_graph_create.restype = i32
        L.fourier_llf_graph_launch.argtypes = [vp, vp]
        L.fourier_llf_graph_launch.restype = i32
        L.fourier_llf_graph_destroy.argtypes = [vp]
        L.fourier_llf_graph_destroy.restype = None
        u64 = ctypes.c_uint64
        L.fourier_llf_server_create.argtypes = [vp, vp, sz, i32, ctypes.POINTER(vp)]
        L.fourier_llf_server_create.restype = i32
        L.fourier_llf_server_submit.argtypes = [vp, jp, u64, vp]
        L.fourier_llf_server_submit.restype = i32
        L.fourier_llf_server_step.argtypes = [vp, vp, ctypes.POINTER(i32)]
        L.fourier_llf_server_step.restype = i32
        L.fourier_llf_server_poll.argtypes = [vp, ctypes.POINTER(u64), i32, ctypes.POINTER(i32)]
        L.fourier_llf_server_poll.restype = i32
        L.fourier_llf_server_stats.argtypes = [vp, ctypes.POINTER(FllfServerStats)]
        L.fourier_llf_server_stats.restype = i32
        L.fourier_llf_server_destroy.argtypes = [vp]
        L.fourier_llf_server_destroy.restype = None
        L.fourier_llf_reparam.argtypes = [vp, jp, jp, vp, sz, vp]
        L.fourier_llf_reparam.restype = i32
        L.fourier_llf_run_static.argtypes = [vp, jp, vp]
        L.fourier_llf_run_static.restype = i32
        L.fourier_llf_fit_range.argtypes = [dbl, dbl, i32, dbl, dp]
        L.fourier_llf_fit_range.restype = i32
        L.fourier_llf_boost_map.argtypes = [vp, vp, i32, i32, ctypes.c_int64, i32, dbl, dbl, vp, vp]
        L.fourier_llf_boost_map.restype = i32
        _LIB = L
    return _LIB


def last_error(ctx=None) -> str:
    s = lib().fourier_llf_last_error(ctx)
    return s.decode() if s else ""


def _check(status: int, ctx=None) -> None:
    if status != FLLF_OK:
        raise FourierLLFError(status, last_error(ctx))


def fit(sigma_r: float, K: int, R: float = 1.0, T: float = 0.0) -> Tuple[float, np.ndarray, np.ndarray]:
    """Host float64 series fit: (T, omega_k, alpha~_k) for k = 1..K."""
    Tout = ctypes.c_double()
    om = (ctypes.c_double * max(K, 1))()
    at = (ctypes.c_double * max(K, 1))()
    _check(lib().fourier_llf_fit(float(sigma_r), int(K), float(R), float(T), ctypes.byref(Tout), om, at))
    return Tout.value, np.array(om[:K]), np.array(at[:K])


def fit_range(sigma_lo: float, sigma_hi: float, K: int, R: float = 1.0) -> float:
    """Host float64 period shared by the range scales [sigma_lo, sigma_hi]."""
    T = ctypes.c_double()
    _check(lib().fourier_llf_fit_range(float(sigma_lo), float(sigma_hi), int(K), float(R), ctypes.byref(T)))
    return T.value


def max_levels(height: int, width: int) -> int:
    return int(lib().fourier_llf_max_levels(int(height), int(width)))


def version() -> int:
    return int(lib().fourier_llf_version())


def _job_array(jobs: Sequence[FllfJob]):
    arr = (FllfJob * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j
    return arr


def validate(jobs: Sequence[FllfJob], storage: str = "f32") -> int:
    """Host-only parameter check; returns the status code (0 = OK)."""
    return int(lib().fourier_llf_validate(_job_array(jobs), len(jobs), STORAGE[storage]))


def footprint(jobs: Sequence[FllfJob], storage: str = "f32") -> int:
    """Workspace bytes for these jobs (host-only; no device needed)."""
    n = ctypes.c_size_t()
    _check(lib().fourier_llf_footprint(_job_array(jobs), len(jobs), STORAGE[storage], ctypes.byref(n)))
    return int(n.value)


@dataclass
class Job:
    """One image to filter: x is a CUDA float32 tensor (C, H, W) or (H, W)."""
    x: "object"
    levels: int
    sigma_r: float
    m: float
    K: int
    R: float = 1.0
    T: float = 0.0
    out: Optional["object"] = None
    m_map: Optional["object"] = None
    sigma_map: Optional["object"] = None
    sigma_max: float = 0.0


def make_job(in_ptr: int, out_ptr: int, width: int, height: int, channels: int, levels: int,
             sigma_r: float, m: float, K: int, R: float = 1.0, T: float = 0.0,
             m_map_ptr: int = 0, pitches: Sequence[int] = (0, 0, 0, 0), sigma_map_ptr: int = 0,
             sigma_max: float = 0.0, flags: int = 0) -> FllfJob:
    """pitches = (row_pitch, plane_pitch, out_row_pitch, out_plane_pitch) in
    elements, 0 = dense."""
    j = FllfJob()
    j.in_ = in_ptr
    j.out = out_ptr
    j.width, j.height, j.channels = int(width), int(height), int(channels)
    j.levels, j.K, j.flags = int(levels), int(K), int(flags)
    j.sigma_r, j.m, j.range_R, j.period_T = float(sigma_r), float(m), float(R), float(T)
    j.m_map = m_map_ptr or None
    j.row_pitch, j.plane_pitch, j.out_row_pitch, j.out_plane_pitch = (int(p) for p in pitches)
    j.sigma_map = sigma_map_ptr or None
    j.sigma_max = float(sigma_max)
    return j


def _pitches(t) -> Tuple[int, int]:
    """(row, plane) element pitches of a (C, H, W) or (H, W) float32 view whose
    rows are contiguous; raises for other layouts."""
    if t.dim() not in (2, 3):
        raise ValueError("images must be (H, W) or (C, H, W)")
    if t.stride(-1) != 1 and t.shape[-1] > 1:
        raise ValueError("image rows must be contiguous (last stride 1)")
    row = t.stride(-2) if t.shape[-2] > 1 else t.shape[-1]
    plane = t.stride(0) if t.dim() == 3 and t.shape[0] > 1 else 0
    # a pitch of 0 means "dense" to the library: an expanded view (stride 0) must
    # be materialised by the caller
    if (t.shape[-2] > 1 and row == 0) or (t.dim() == 3 and t.shape[0] > 1 and plane == 0):
        raise ValueError("image has a zero stride (an expanded view); pass a tensor with its own rows and planes")
    return int(row), int(plane)


class FourierLLF:
    """A library context (one per stream / host thread) with a cached workspace."""

    def __init__(self, storage: str = "f32", device: int = 0):
        import torch  # memory and streams only
        if storage not in STORAGE:
            raise ValueError(f"storage must be one of {sorted(STORAGE)}")
        self.storage = storage
        self.device = torch.device("cuda", device)
        ctx = ctypes.c_void_p()
        _check(lib().fourier_llf_create(ctypes.byref(ctx), int(device), STORAGE[storage]))
        self._ctx = ctx
        self._ws = None

    def close(self) -> None:
        if getattr(self, "_ctx", None):
            lib().fourier_llf_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- marshalling ---------------------------------------------------------
    def _prepare(self, job: Job) -> Tuple[FllfJob, "object"]:
        import torch
        x = job.x
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32):
            raise TypeError("x must be a CUDA float32 tensor")
        if x.dim() == 2:
            C, H, W = 1, x.shape[0], x.shape[1]
        elif x.dim() == 3:
            C, H, W = x.shape
        else:
            raise ValueError("x must be (H, W) or (C, H, W)")
        out = job.out if job.out is not None else torch.empty(x.shape, dtype=torch.float32, device=x.device)
        if out.shape != x.shape or out.dtype != torch.float32 or not out.is_cuda:
            raise ValueError("out must be a CUDA float32 tensor shaped like x")
        irp, ipp = _pitches(x)
        orp, opp = _pitches(out)
        mptr = 0
        if job.m_map is not None:
            mm = job.m_map
            if tuple(mm.shape) != (H, W) or mm.dtype != torch.float32 or not mm.is_contiguous() or not mm.is_cuda:
                raise ValueError("m_map must be a contiguous CUDA float32 (H, W) tensor")
            mptr = mm.data_ptr()
        sptr = 0
        if job.sigma_map is not None:
            sm = job.sigma_map
            if tuple(sm.shape) != (H, W) or sm.dtype != torch.float32 or not sm.is_contiguous() or not sm.is_cuda:
                raise ValueError("sigma_map must be a contiguous CUDA float32 (H, W) tensor")
            sptr = sm.data_ptr()
        fj = make_job(x.data_ptr(), out.data_ptr(), W, H, C, job.levels, job.sigma_r, job.m, job.K,
                      job.R, job.T, mptr, (irp, ipp, orp, opp), sptr, job.sigma_max)
        return fj, out

    def workspace_size(self, jobs: Sequence[FllfJob]) -> int:
        n = ctypes.c_size_t()
        arr = _job_array(jobs)
        _check(lib().fourier_llf_workspace_size(self._ctx, arr, len(jobs), ctypes.byref(n)), self._ctx)
        return int(n.value)

    def workspace(self, nbytes: int):
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def run_jobs(self, fjobs: Sequence[FllfJob], workspace=None, stream=None, keep=()) -> None:
        """Enqueue already-marshalled jobs on `stream` (default: torch's current
        stream).  On another stream than the current one, the cached workspace and
        the tensors in `keep` are marked as used by that stream, so that torch's
        allocator does not hand their memory out again before its work is done."""
        import torch
        arr = _job_array(fjobs)
        need = self.workspace_size(fjobs)
        ws = workspace if workspace is not None else self.workspace(need)
        current = torch.cuda.current_stream(self.device)
        if stream is None:
            stream = current
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().fourier_llf_run(self._ctx, arr, len(fjobs), ws.data_ptr(), ws.numel(), sptr), self._ctx)
        if isinstance(stream, torch.cuda.Stream) and stream != current:
            for t in (ws,) + tuple(keep):
                if t is not None:
                    t.record_stream(stream)

    def timing(self, enable: bool) -> None:
        """Bracket every kernel launch with hipEvents on the run's stream."""
        _check(lib().fourier_llf_timing_enable(self._ctx, 1 if enable else 0), self._ctx)

    def timing_read(self) -> List[dict]:
        """Per kernel class: launches, total ms and algorithmic bytes since the last read."""
        cap = 128
        buf = (FllfKernelTime * cap)()
        n = ctypes.c_int()
        _check(lib().fourier_llf_timing_read(self._ctx, buf, cap, ctypes.byref(n)), self._ctx)
        return [dict(name=buf[i].name.decode(), launches=buf[i].launches, total_ms=buf[i].total_ms,
                     bytes=buf[i].bytes) for i in range(min(n.value, cap))]

    def reparam(self, prev: FllfJob, nxt: FllfJob, workspace, stream=None) -> None:
        """Filter `nxt` (new m / sigma_r, same T) from the pyramids `prev` left in `workspace`."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().fourier_llf_reparam(self._ctx, ctypes.byref(prev), ctypes.byref(nxt), workspace.data_ptr(),
                                         workspace.numel(), sptr), self._ctx)

    # -- launch shape ----------------------------------------------------------
    def set_tuning(self, params: Optional[Sequence[int]] = None) -> None:
        """Set (FLLF_TUNE_*) launch-shape parameters; None restores the built-in ones."""
        if params is None:
            _check(lib().fourier_llf_set_tuning(self._ctx, None), self._ctx)
            return
        arr = (ctypes.c_int32 * len(TUNE_NAMES))(*[int(v) for v in params])
        _check(lib().fourier_llf_set_tuning(self._ctx, arr), self._ctx)

    def get_tuning(self) -> List[int]:
        arr = (ctypes.c_int32 * len(TUNE_NAMES))()
        _check(lib().fourier_llf_get_tuning(self._ctx, arr), self._ctx)
        return list(arr)

    def autotune(self, fjobs: Sequence[FllfJob], workspace=None, stream=None, reps: int = 3,
                 cache: Optional[str] = None) -> List[int]:
        """Time candidate launch shapes on these jobs and keep the fastest
        (synchronous).  With `cache` (a file path) a stored result for the same
        device, storage and job shapes is reused, and a new one is appended."""
        import torch
        arr = _job_array(fjobs)
        ws = workspace if workspace is not None else self.workspace(self.workspace_size(fjobs))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        out = (ctypes.c_int32 * len(TUNE_NAMES))()
        if cache is None:
            _check(lib().fourier_llf_autotune(self._ctx, arr, len(fjobs), ws.data_ptr(), ws.numel(), sptr,
                                              int(reps), out), self._ctx)
        else:
            _check(lib().fourier_llf_autotune_cached(self._ctx, arr, len(fjobs), ws.data_ptr(), ws.numel(), sptr,
                                                     int(reps), os.fsencode(cache), out), self._ctx)
        return list(out)

    def graph(self, fjobs: Sequence[FllfJob], workspace=None) -> "Graph":
        """Capture the launches of these jobs into a replayable HIP graph with its own workspace."""
        import torch
        need = self.workspace_size(fjobs)
        ws = workspace if workspace is not None else torch.empty(max(need, 256), dtype=torch.uint8,
                                                                 device=self.device)
        arr = _job_array(fjobs)
        g = ctypes.c_void_p()
        _check(lib().fourier_llf_graph_create(self._ctx, arr, len(fjobs), ws.data_ptr(), ws.numel(),
                                              ctypes.byref(g)), self._ctx)
        return Graph(g, ws)

    def run(self, x, levels: int, sigma_r: float, m: float, K: int, R: float = 1.0, T: float = 0.0,
            out=None, m_map=None, stream=None, sigma_map=None, sigma_max: float = 0.0):
        """Filter one (C, H, W) or (H, W) float32 CUDA tensor (rows contiguous; a
        crop or other strided view is read in place) into `out` (a new dense
        tensor when None; any view with contiguous rows otherwise); returns it."""
        fj, out = self._prepare(Job(x, levels, sigma_r, m, K, R, T, out, m_map, sigma_map, sigma_max))
        self.run_jobs([fj], stream=stream, keep=(out, m_map, sigma_map))
        return out

    def run_fast(self, x, levels: int, sigma_r: float, m: float, n: int, R: float = 1.0, out=None, stream=None):
        """The fast LLF comparator (FLLF_FLAG_FAST_LLF): the detail remap sampled at
        n equally spaced intensities in [0, R] (n even), n + 1 pyramids."""
        fj, out = self._prepare(Job(x, levels, sigma_r, m, n, R, 0.0, out))
        fj.flags = FLLF_FLAG_FAST_LLF
        self.run_jobs([fj], stream=stream, keep=(out,))
        return out

    def run_static(self, x, levels: int, sigma_r: float, m: float, K: int, R: float = 1.0, T: float = 0.0,
                   out=None, m_map=None, stream=None, sigma_map=None, sigma_max: float = 0.0):
        """Like run, through fourier_llf_run_static: the workspace is the library's
        static device array (no workspace tensor is allocated).  `out` should be
        given by callers that must not allocate."""
        import torch
        fj, out = self._prepare(Job(x, levels, sigma_r, m, K, R, T, out, m_map, sigma_map, sigma_max))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().fourier_llf_run_static(self._ctx, ctypes.byref(fj), sptr), self._ctx)
        return out

    def boost_map(self, plane, radius: int, m_max: float, v_half: float, out=None, stream=None):
        """Variance-driven boost map of one (H, W) float32 CUDA plane (rows
        contiguous; a view of one channel is read in place); returns a dense
        (H, W) map for run(..., m_map=...)."""
        import torch
        if not (isinstance(plane, torch.Tensor) and plane.is_cuda and plane.dtype == torch.float32
                and plane.dim() == 2):
            raise TypeError("plane must be a 2-D CUDA float32 tensor")
        rp, _ = _pitches(plane)
        H, W = plane.shape
        out = out if out is not None else torch.empty((H, W), dtype=torch.float32, device=plane.device)
        if tuple(out.shape) != (H, W) or not out.is_contiguous() or out.dtype != torch.float32:
            raise ValueError("out must be a contiguous float32 (H, W) tensor")
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().fourier_llf_boost_map(self._ctx, plane.data_ptr(), W, H, rp, int(radius), float(m_max),
                                           float(v_half), out.data_ptr(), sptr), self._ctx)
        return out

    def run_batch(self, jobs: Sequence[Job], stream=None) -> List["object"]:
        """Filter several images (sizes and parameters may differ) in one call."""
        prepared = [self._prepare(j) for j in jobs]
        keep = [p[1] for p in prepared] + [j.m_map for j in jobs] + [j.sigma_map for j in jobs]
        self.run_jobs([p[0] for p in prepared], stream=stream, keep=keep)
        return [p[1] for p in prepared]


class Graph:
    """A captured schedule (``fllf_graph``); keeps its workspace alive."""

    def __init__(self, handle, workspace):
        self._g = handle
        self.workspace = workspace

    def launch(self, stream=None) -> None:
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.workspace.device)
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().fourier_llf_graph_launch(self._g, sptr))

    def close(self) -> None:
        if getattr(self, "_g", None):
            lib().fourier_llf_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (``fllf_server``) over a device arena of
    `arena_bytes` taken from torch.  Jobs are marshalled like FourierLLF.run;
    scheduling, admission and launches happen in the library."""

    def __init__(self, llf: FourierLLF, arena_bytes: int, max_active: int = 64):
        import torch
        self.llf = llf
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=llf.device)
        h = ctypes.c_void_p()
        _check(lib().fourier_llf_server_create(llf._ctx, self.arena.data_ptr(), self.arena.numel(),
                                               int(max_active), ctypes.byref(h)), llf._ctx)
        self._s = h
        self._keep = {}  # tag -> tensors that must outlive the job

    def submit(self, job: Job, tag: int, ready_event=None):
        """Queue a job; returns its output tensor (valid once `tag` is polled).
        `ready_event`: a torch.cuda.Event recorded after the input was written."""
        fj, out = self.llf._prepare(job)
        ev = ready_event.cuda_event if ready_event is not None else None
        _check(lib().fourier_llf_server_submit(self._s, ctypes.byref(fj), int(tag), ev), self.llf._ctx)
        self._keep[int(tag)] = (job, out, ready_event)
        return out

    def step(self, stream=None) -> int:
        """Admit and enqueue one pass of every admitted job; returns jobs not yet reported."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.llf.device)
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        pending = ctypes.c_int32()
        _check(lib().fourier_llf_server_step(self._s, sptr, ctypes.byref(pending)), self.llf._ctx)
        return int(pending.value)

    def poll(self, max_n: int = 256) -> List[int]:
        """Tags of jobs whose output is ready (non-blocking)."""
        buf = (ctypes.c_uint64 * max_n)()
        n = ctypes.c_int32()
        _check(lib().fourier_llf_server_poll(self._s, buf, max_n, ctypes.byref(n)), self.llf._ctx)
        tags = [int(buf[i]) for i in range(n.value)]
        for t in tags:
            self._keep.pop(t, None)
        return tags

    def stats(self) -> dict:
        st = FllfServerStats()
        _check(lib().fourier_llf_server_stats(self._s, ctypes.byref(st)), self.llf._ctx)
        return {name: getattr(st, name) for name, _ in FllfServerStats._fields_}

    def close(self) -> None:
        if getattr(self, "_s", None):
            lib().fourier_llf_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
