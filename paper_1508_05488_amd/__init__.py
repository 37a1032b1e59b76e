"""chainhull: the CudaChain convex hull hot path on MI355X (gfx950).

A thin ctypes binding over ``libchainhull.so`` (built in-tree by
``paper_1508_05488_amd.build``).  Each function marshals arguments to the C
ABI declared in ``include/chainhull.h`` and nothing more: every step of the
method runs in the library's HIP kernels and its host finish.  PyTorch only
provides device memory and the current HIP stream.  There is no fallback:
when the library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libchainhull.so")

CH_OK, CH_EINVAL, CH_EDOMAIN, CH_ENOMEM, CH_EHIP, CH_EADMIT, CH_ECAPACITY = 0, -1, -2, -3, -4, -5, -6
NOALLOC_MAX_POINTS = 1 << 20      # CH_NOALLOC_MAX_POINTS
NOALLOC_SCRATCH_BYTES = 96 << 20  # CH_NOALLOC_SCRATCH_BYTES
CH_BATCH_REDO = -(2 ** 31)

# C entry points declared in include/chainhull.h
EXPORTS = ("hull2d", "hull2d_async", "hull2d_noalloc", "hull2d_batched", "hull2d_batched_async", "chainhull_polygon", "chainhull_finish_host",
           "chainhull_last_stats", "chainhull_last_batch_stats", "chainhull_set_timing", "chainhull_strerror",
           "chainhull_release", "chainhull_release_stream", "chainhull_workspace_bytes", "chainhull_spa_chunked",
           "chainhull_server_create", "chainhull_server_submit", "chainhull_server_wait",
           "chainhull_server_stats", "chainhull_server_destroy", "chainhull_set_tuning", "chainhull_get_tuning")

STAGES = ("sample", "stream", "cand", "sort", "spa", "finish_dev", "gather", "finish")


class ChainHullError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        msg = f"{what}: " if what else ""
        super().__init__(f"{msg}{strerror(status)} (status {status})")


class ChStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("ext_idx", ctypes.c_int32 * 4),
        ("ext_xy", ctypes.c_int32 * 8),
        ("s1", ctypes.c_int64 * 4),
        ("open", ctypes.c_int64),
        ("candidates", ctypes.c_int64),
        ("s2", ctypes.c_int64 * 4),
        ("polygon", ctypes.c_int64),
        ("hull", ctypes.c_int64),
        ("ms", ctypes.c_float * 8),
        ("device_finish", ctypes.c_int32),
        ("fused", ctypes.c_int32),
        ("ms_pre", ctypes.c_float),
        ("ms_finish", ctypes.c_float),
    ]

    def as_dict(self) -> dict:
        return {
            "n": self.n,
            "ext_idx": list(self.ext_idx),
            "ext_xy": list(self.ext_xy),
            "s1": list(self.s1),
            "open": self.open,
            "candidates": self.candidates,
            "s2": list(self.s2),
            "polygon": self.polygon,
            "hull": self.hull,
            "ms": dict(zip(STAGES, list(self.ms))),
            "device_finish": bool(self.device_finish),
            "fused": bool(self.fused),
            "ms_pre": self.ms_pre,
            "ms_finish": self.ms_finish,
        }


class ChBatchStats(ctypes.Structure):
    _fields_ = [
        ("num_sets", ctypes.c_int32),
        ("device_sets", ctypes.c_int32),
        ("redo_sets", ctypes.c_int32),
        ("points", ctypes.c_int64),
        ("ms_kernel", ctypes.c_float),
        ("ms_total", ctypes.c_float),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ChServerStats(ctypes.Structure):
    _fields_ = [
        ("completed", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("batched_requests", ctypes.c_int64),
        ("single_requests", ctypes.c_int64),
        ("points", ctypes.c_int64),
        ("pending", ctypes.c_int64),
        ("max_inflight", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("reserved_bytes", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved0"}


class ChTuning(ctypes.Structure):
    """Launch shapes (include/chainhull.h, ch_tuning)."""
    _fields_ = [
        ("stream_grid", ctypes.c_int32),
        ("stream_unroll", ctypes.c_int32),
        ("cand_per_row", ctypes.c_int32),
        ("chain_grid", ctypes.c_int32),
        ("wide_grid", ctypes.c_int32),
        ("batch_unroll", ctypes.c_int32),
        ("batch_order", ctypes.c_int32),
        ("serve_batch_max", ctypes.c_int32),
        ("fused_max", ctypes.c_int32),
        ("list_max", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


TUNING_FIELDS = tuple(k for k, _ in ChTuning._fields_)
TUNING_DIR = os.path.join(_PKG, "tuning")

_lib = None
_tuning_loaded = None
_tuning_note = None


def lib():
    """Load libchainhull.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1508_05488_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.hull2d.argtypes = [vp, i64, vp, vp, vp]
    L.hull2d_async.argtypes = [vp, i64, vp, vp, vp]
    L.hull2d_async.restype = ctypes.c_int
    L.hull2d_noalloc.argtypes = [vp, i64, vp, vp, vp]
    L.hull2d_noalloc.restype = ctypes.c_int
    L.hull2d.restype = ctypes.c_int
    L.hull2d_batched.argtypes = [vp, vp, i32, vp, vp, vp]
    L.hull2d_batched.restype = ctypes.c_int
    L.hull2d_batched_async.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.hull2d_batched_async.restype = ctypes.c_int
    L.chainhull_polygon.argtypes = [vp, i64, vp, ctypes.POINTER(i64), ctypes.POINTER(ChStats), vp]
    L.chainhull_polygon.restype = ctypes.c_int
    L.chainhull_finish_host.argtypes = [vp, vp, i64, vp, ctypes.POINTER(i64)]
    L.chainhull_finish_host.restype = ctypes.c_int
    L.chainhull_last_stats.argtypes = [ctypes.POINTER(ChStats)]
    L.chainhull_last_stats.restype = ctypes.c_int
    L.chainhull_last_batch_stats.argtypes = [ctypes.POINTER(ChBatchStats)]
    L.chainhull_last_batch_stats.restype = ctypes.c_int
    L.chainhull_set_timing.argtypes = [ctypes.c_int]
    L.chainhull_set_timing.restype = None
    L.chainhull_strerror.argtypes = [ctypes.c_int]
    L.chainhull_strerror.restype = ctypes.c_char_p
    L.chainhull_release.argtypes = []
    L.chainhull_release.restype = None
    L.chainhull_spa_chunked.argtypes = [vp, i64, ctypes.c_uint32, i64, vp, vp]
    L.chainhull_spa_chunked.restype = ctypes.c_int
    L.chainhull_release_stream.argtypes = [vp]
    L.chainhull_release_stream.restype = ctypes.c_int
    L.chainhull_server_create.argtypes = [i32, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.chainhull_server_create.restype = ctypes.c_int
    L.chainhull_server_submit.argtypes = [vp, vp, i64, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    L.chainhull_server_submit.restype = ctypes.c_int
    L.chainhull_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.chainhull_server_wait.restype = ctypes.c_int
    L.chainhull_server_stats.argtypes = [vp, ctypes.POINTER(ChServerStats)]
    L.chainhull_server_stats.restype = ctypes.c_int
    L.chainhull_server_destroy.argtypes = [vp]
    L.chainhull_server_destroy.restype = ctypes.c_int
    L.chainhull_workspace_bytes.argtypes = [i64]
    L.chainhull_workspace_bytes.restype = ctypes.c_size_t
    L.chainhull_set_tuning.argtypes = [i64, ctypes.POINTER(ChTuning)]
    L.chainhull_set_tuning.restype = ctypes.c_int
    L.chainhull_get_tuning.argtypes = [i64, ctypes.POINTER(ChTuning)]
    L.chainhull_get_tuning.restype = ctypes.c_int
    _lib = L
    load_tuning()
    return L


def get_tuning(n: int = -1) -> dict:
    """The launch shapes a call with n points uses (n < 0: the defaults)."""
    t = ChTuning()
    _check(lib().chainhull_get_tuning(int(n), ctypes.byref(t)), "chainhull_get_tuning")
    return t.as_dict()


def set_tuning(n_max: int, tuning: dict) -> None:
    """Use these shapes for calls of at most n_max points."""
    t = ChTuning(**{k: int(tuning[k]) for k in TUNING_FIELDS})
    _check(lib().chainhull_set_tuning(int(n_max), ctypes.byref(t)), "chainhull_set_tuning")


def clear_tuning() -> None:
    """Back to the default shapes for every call."""
    lib().chainhull_set_tuning(-1, None)


def device_key() -> str:
    """The current GPU's name and architecture, the key of its tuning file."""
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "gpu").split(":")[0]
    name = "".join(c if c.isalnum() else "_" for c in p.name).strip("_")
    return f"{arch}_{name}"


def tuning_path(key: str | None = None) -> str:
    return os.path.join(TUNING_DIR, f"{key or device_key()}.json")


def load_tuning(path: str | None = None):
    """Apply the autotuner's saved shapes for the current GPU (a JSON file
    under tuning/, written by autotune.py), when one exists: the file of the
    device's key, else the one file of its architecture (the device's
    reported name can differ between processes, under a profiler for
    instance).  Returns the path applied, or None (defaults; the reason in
    tuning_note()).  Without a GPU nothing is read."""
    global _tuning_loaded, _tuning_note
    import glob
    import json
    if path is None:
        try:
            import torch
            if not torch.cuda.is_available():
                _tuning_note = "no GPU"
                return None
            key = device_key()
            path = tuning_path(key)
            if not os.path.exists(path):
                same_arch = sorted(glob.glob(os.path.join(TUNING_DIR, key.split("_")[0] + "_*.json")))
                if len(same_arch) == 1:
                    path = same_arch[0]
        except Exception as e:  # (no usable device: the defaults)
            _tuning_note = f"no device key: {e!r}"
            return None
    if not os.path.exists(path):
        _tuning_note = f"no tuning file {os.path.basename(path)}"
        _tuning_loaded = None
        return None
    with open(path) as f:
        doc = json.load(f)
    L = _lib
    L.chainhull_set_tuning(-1, None)
    for c in doc.get("classes", []):
        t = ChTuning(**{k: int(c["tuning"][k]) for k in TUNING_FIELDS})
        rc = L.chainhull_set_tuning(int(c["n_max"]), ctypes.byref(t))
        if rc != CH_OK:
            raise ChainHullError(rc, f"tuning file {path}")
    _tuning_loaded = path
    _tuning_note = None
    return path


def tuning_note():
    """Why no tuning file was applied (None when one was)."""
    lib()
    return _tuning_note


def tuning_source():
    """The tuning file applied when the library was loaded, or None."""
    lib()
    return _tuning_loaded


def strerror(status: int) -> str:
    return lib().chainhull_strerror(int(status)).decode()


def _check(rc: int, what: str) -> None:
    if rc != CH_OK:
        raise ChainHullError(rc, what)


def _stream_ptr(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _device_points(points):
    import torch
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch.Tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 2:
        raise TypeError("points must be float32 with shape [n, 2]")
    if not points.is_contiguous():
        raise TypeError("points must be contiguous")
    return points


def hull2d(points, stream=None):
    """Hull vertex indices (int32 tensor on the points' device)."""
    import torch
    pts = _device_points(points)
    n = pts.shape[0]
    with torch.cuda.device(pts.device):
        out = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
        cnt = torch.empty(1, dtype=torch.int32, device=pts.device)
        rc = lib().hull2d(pts.data_ptr(), n, out.data_ptr(), cnt.data_ptr(), _stream_ptr(stream))
        _check(rc, "hull2d")
        h = int(cnt.item())
    return out[:h]


def hull2d_into(points, out_idx, out_count, stream=None) -> int:
    """hull2d writing into caller-provided device tensors; returns the status."""
    return lib().hull2d(points.data_ptr(), points.shape[0], out_idx.data_ptr(), out_count.data_ptr(),
                        _stream_ptr(stream))


def hull2d_async(points, out_idx, out_count, stream=None) -> int:
    """hull2d with every step on the device, queued on the stream and not
    synchronised: out_count (CUDA int32 [1]) receives the hull size or a
    negative status (CH_EHIP if the device finish gave up: then call
    hull2d, which finishes on the host).  out_idx: CUDA
    int32 with room for the points.  Returns the status of the launch."""
    return lib().hull2d_async(points.data_ptr(), points.shape[0], out_idx.data_ptr(), out_count.data_ptr(),
                              _stream_ptr(stream))


def hull2d_noalloc(points, out_idx, out_count, stream=None) -> int:
    """hull2d_async on the library's fixed per-device buffer: allocates
    nothing (at most NOALLOC_MAX_POINTS points, else CH_ECAPACITY).  Calls
    that overlap on one device race.  Returns the status of the launch."""
    return lib().hull2d_noalloc(points.data_ptr(), points.shape[0], out_idx.data_ptr(), out_count.data_ptr(),
                                _stream_ptr(stream))


def hull2d_batched(points, offsets, stream=None):
    """Hulls of concatenated sets.  Returns (list of int32 tensors, counts tensor)."""
    import torch
    pts = _device_points(points)
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    num = offs.shape[0] - 1
    with torch.cuda.device(pts.device):
        out = torch.empty(max(int(offs[-1]) if num >= 0 else 0, 1), dtype=torch.int32, device=pts.device)
        cnt = torch.zeros(max(num, 1), dtype=torch.int32, device=pts.device)
        rc = lib().hull2d_batched(pts.data_ptr(), offs.ctypes.data, num, out.data_ptr(), cnt.data_ptr(),
                                  _stream_ptr(stream))
        _check(rc, "hull2d_batched")
        counts = cnt[:num].cpu().numpy()
    return [out[int(offs[s]): int(offs[s]) + int(counts[s])] for s in range(num)], cnt[:num]


def hull2d_batched_async(points, offsets, order, out_idx, out_counts, stream=None) -> int:
    """The batched kernel alone, queued on the stream (capturable in a
    graph).  offsets: CUDA int64 [num_sets + 1]; order: CUDA int32
    [num_sets] or None; out_idx, out_counts: CUDA int32.  Returns the
    status of the launch."""
    import torch
    pts = _device_points(points)
    for t, dt, name in ((offsets, torch.int64, "offsets"), (out_idx, torch.int32, "out_idx"),
                        (out_counts, torch.int32, "out_counts")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous CUDA {dt} tensor")
    if order is not None and (not order.is_cuda or order.dtype != torch.int32 or not order.is_contiguous()):
        raise TypeError("order must be a contiguous CUDA int32 tensor")
    num = offsets.numel() - 1
    with torch.cuda.device(pts.device):
        return lib().hull2d_batched_async(pts.data_ptr(), offsets.data_ptr(), 0 if order is None else order.data_ptr(),
                                          num, out_idx.data_ptr(), out_counts.data_ptr(), _stream_ptr(stream))


def polygon(points, stream=None):
    """Steps 1-6: the simple polygon (numpy int32 indices) and the call's counts."""
    import torch
    pts = _device_points(points)
    n = pts.shape[0]
    poly = np.empty(n + 4, dtype=np.int32)
    m = ctypes.c_int64(0)
    st = ChStats()
    with torch.cuda.device(pts.device):
        rc = lib().chainhull_polygon(pts.data_ptr(), n, poly.ctypes.data, ctypes.byref(m), ctypes.byref(st),
                                     _stream_ptr(stream))
    _check(rc, "chainhull_polygon")
    return poly[: m.value].copy(), st.as_dict()


def finish_host(poly_xy, poly_idx) -> np.ndarray:
    """Step 7 on the host: Melkman's hull of a simple polygon (no GPU needed)."""
    xy = np.ascontiguousarray(np.asarray(poly_xy, dtype=np.int32).reshape(-1, 2))
    idx = np.ascontiguousarray(np.asarray(poly_idx, dtype=np.int32).reshape(-1))
    if xy.shape[0] != idx.shape[0]:
        raise ValueError("poly_xy and poly_idx differ in length")
    m = idx.shape[0]
    out = np.empty(max(m, 1), dtype=np.int32)
    h = ctypes.c_int64(0)
    rc = lib().chainhull_finish_host(xy.ctypes.data, idx.ctypes.data, m, out.ctypes.data, ctypes.byref(h))
    _check(rc, "chainhull_finish_host")
    return out[: h.value].copy()


def last_stats() -> dict:
    st = ChStats()
    _check(lib().chainhull_last_stats(ctypes.byref(st)), "chainhull_last_stats")
    return st.as_dict()


def last_batch_stats() -> dict:
    st = ChBatchStats()
    _check(lib().chainhull_last_batch_stats(ctypes.byref(st)), "chainhull_last_batch_stats")
    return st.as_dict()


def set_timing(enable) -> None:
    """0/False: off; 1/True: every stage; 2: steps 1-6 and the finish as
    two spans only (ms_pre, ms_finish)."""
    lib().chainhull_set_timing(2 if enable == 2 else (1 if enable else 0))


def release() -> None:
    lib().chainhull_release()


def release_stream(stream) -> None:
    """Free the library workspace of one stream (no call on it may be running)."""
    _check(lib().chainhull_release_stream(_stream_ptr(stream)), "chainhull_release_stream")


def workspace_bytes(n: int) -> int:
    return int(lib().chainhull_workspace_bytes(int(n)))


def spa_chunked(k2_sorted, sigma: int, chunk: int, stream=None):
    """The paper's SPA in subsets of ``chunk`` points over one region's
    sorted k2 values (a CUDA int32 tensor holding values in [0, 2^23)).
    Returns a bool tensor of survivors."""
    import torch
    if not isinstance(k2_sorted, torch.Tensor) or not k2_sorted.is_cuda or k2_sorted.dtype != torch.int32:
        raise TypeError("k2_sorted must be a CUDA int32 tensor")
    k2 = k2_sorted.contiguous()
    m = k2.numel()
    keep = torch.empty(max(m, 1), dtype=torch.uint8, device=k2.device)
    with torch.cuda.device(k2.device):
        rc = lib().chainhull_spa_chunked(k2.data_ptr(), m, int(sigma), int(chunk), keep.data_ptr(),
                                         _stream_ptr(stream))
    _check(rc, "chainhull_spa_chunked")
    return keep[:m].bool()


class Server:
    """Continuous-batching hull server on one device (chainhull_server_*).

    ``submit(points)`` takes a CUDA float32 [n, 2] tensor and returns a
    ticket at once; ``wait(ticket)`` blocks and returns (hull int32 tensor,
    latency in ms).  The points and output tensors of a request are kept
    alive here until it is waited for."""

    def __init__(self, workers: int = 4, mem_budget: int = 288 << 30, device=None):
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().chainhull_server_create(int(workers), int(mem_budget), ctypes.byref(h)),
                   "chainhull_server_create")
        self._h = h
        self._live = {}

    def submit(self, points, out_idx=None, out_count=None) -> int:
        import torch
        pts = _device_points(points)
        n = pts.shape[0]
        if out_idx is None:
            out_idx = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
        if out_count is None:
            out_count = torch.zeros(1, dtype=torch.int32, device=pts.device)
        # the workers' streams are not ordered after the caller's: the points
        # (and the count's zero fill) must be complete before a worker reads
        # them
        torch.cuda.current_stream(pts.device).synchronize()
        t = ctypes.c_uint64(0)
        rc = lib().chainhull_server_submit(self._h, pts.data_ptr(), n, out_idx.data_ptr(), out_count.data_ptr(),
                                           ctypes.byref(t))
        _check(rc, "chainhull_server_submit")
        self._live[t.value] = (pts, out_idx, out_count)
        return t.value

    def wait(self, ticket: int):
        h = ctypes.c_int32(0)
        ms = ctypes.c_double(0.0)
        rc = lib().chainhull_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(h), ctypes.byref(ms))
        pts, out_idx, _ = self._live.pop(ticket)
        _check(rc, "chainhull_server_wait")
        return out_idx[: h.value], ms.value

    def stats(self) -> dict:
        st = ChServerStats()
        _check(lib().chainhull_server_stats(self._h, ctypes.byref(st)), "chainhull_server_stats")
        return st.as_dict()

    def close(self) -> None:
        if self._h:
            lib().chainhull_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
