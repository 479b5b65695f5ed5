"""Python binding of libglcm, the gfx950 gray-level co-occurrence matrix library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/glcm.h.  PyTorch supplies device
memory and streams.  The functions keep the C names:

    glcm_compute(img, N, lo=0, hi=None, offsets=((1, 0),), out=None, stream=None, plan=None)
        -> torch.Tensor [K, N, N] uint32 on the current device
    glcm_features(P, out=None, stream=None) -> torch.Tensor [K, 5] float32
    glcm_histogram(img, N, lo=0, hi=None, out=None, stream=None, plan=None) -> torch.Tensor [N] uint32
    glcm_symmetrize(P, out=None) / glcm_normalize(P) / glcm_average(P, m) / glcm_haralick(P)
        -> P + P^T [K, N, N] uint32 / P / sum P [K, N, N] float32 /
           mean of normalised groups of m [K/m, N, N] float32 / statistics f1..f13 [K, 13] float32
    glcm_haralick_mcc(P) -> maximal correlation coefficient (f14) [K] float32
    glcm_offset_polar(d, theta_deg) -> (dx, dy)
    glcm_plan_create(dtype, N, offsets, max_W, max_H, flags=0) -> Plan
    glcm_batch_compute(images_or_tileset, plan, ...) -> (counts [T, K, N, N], statistics [T, K, 5])
    Server(lanes, hbm_budget, result_pool_bytes): the request server
        (glcm_server_submit / wait / query / fetch / release / drain / stats)

Conventions (Eq. (1) of the paper, made precise): out[k][i][j] counts pixels
(x, y) with level i whose neighbour (x + dx_k, y + dy_k) lies inside the image
and has level j; levels are q(v) = floor((v - lo) * N / (hi - lo + 1)),
clamped to [0, N-1].

If the library is not built the functions raise; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

__all__ = [
    "GlcmError", "Plan", "Tuning", "glcm_abi_version", "glcm_strerror", "glcm_last_hip_error",
    "glcm_offset_polar", "glcm_plan_create", "glcm_plan_destroy", "glcm_plan_tuning", "glcm_plan_autotune",
    "glcm_compute",
    "glcm_compute_static",
    "glcm_features", "library_path", "U8", "U16", "FLAG_FORCE_GENERIC", "FLAG_FORCE_PARTITIONED",
    "FLAG_FORCE_GLOBAL", "FLAG_SERIAL_UPLOAD", "FLAG_TIMING", "FLAG_FORCE_SLABS", "FLAG_FORCE_L2", "FLAG_FORCE_BLOCKS", "glcm_batch_compute", "Tile", "TileSet", "prepare_tiles", "PATH_NAMES", "glcm_plan_kernel_time",
    "glcm_plan_rebind", "glcm_plan_workspace", "glcm_plan_cache_stats", "glcm_plan_cache_clear", "Server", "RequestInfo", "ServerStats", "PreparedBatch",
    "glcm_histogram", "glcm_symmetrize", "glcm_normalize", "glcm_average", "glcm_haralick", "HARALICK_NAMES",
    "glcm_haralick_mcc", "BatchTuning",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libglcm.so")

U8, U16 = 0, 1
FLAG_FORCE_GENERIC = 1 << 0
FLAG_FORCE_PARTITIONED = 1 << 1
FLAG_FORCE_GLOBAL = 1 << 2
FLAG_SERIAL_UPLOAD = 1 << 3
FLAG_TIMING = 1 << 4
FLAG_FORCE_SLABS = 1 << 5
FLAG_FORCE_L2 = 1 << 6
FLAG_FORCE_BLOCKS = 1 << 7
STATIC_MAX_WORDS = 1 << 18  # GLCM_STATIC_MAX_WORDS: largest K * N * N of glcm_compute_static
PATH_NAMES = {0: "generic", 1: "slabs", 2: "partitioned", 3: "global", 4: "strips", 5: "l2", 6: "blocks"}

STATUS = {0: "GLCM_OK", -1: "GLCM_EINVAL", -2: "GLCM_ENOMEM", -3: "GLCM_EUNSUPPORTED",
          -4: "GLCM_EHIP", -5: "GLCM_EBUSY"}


class GlcmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = f"{what}: {STATUS.get(status, status)} ({_lib().glcm_strerror(status).decode()})"
        if status == -4:
            msg += f", hipError {_lib().glcm_last_hip_error()}"
        super().__init__(msg)


class Offset(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_int32), ("dy", ctypes.c_int32)]


class Tile(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("stride", ctypes.c_int64), ("W", ctypes.c_int32), ("H", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("stride", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("N", ctypes.c_int32), ("lo", ctypes.c_uint32), ("hi", ctypes.c_uint32),
                ("offsets", ctypes.c_void_p), ("K", ctypes.c_int32), ("features", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("feat", ctypes.c_void_p)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("lane", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("done_us", ctypes.c_double), ("out", ctypes.c_void_p), ("feat", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("lanes", ctypes.c_int32), ("max_inflight", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_uint64), ("max_bytes_in_use", ctypes.c_uint64),
                ("fused_launches", ctypes.c_uint64), ("fused_requests", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("replicas", ctypes.c_int), ("wg_size", ctypes.c_int), ("rows_per_wave", ctypes.c_int),
                ("tile_rows", ctypes.c_int), ("counter_bits", ctypes.c_int), ("merge", ctypes.c_int),
                ("path", ctypes.c_int), ("partitions", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchTuning(ctypes.Structure):
    _fields_ = [("replicas", ctypes.c_int), ("min_rows", ctypes.c_int), ("wg_size", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_L = None


def library_path() -> str:
    return _LIB_PATH


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_1710_06189_amd/build.py "
                               "(or __graft_entry__.build())")
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i32, u32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_int64
        lib.glcm_abi_version.restype = i32
        lib.glcm_strerror.restype = ctypes.c_char_p
        lib.glcm_strerror.argtypes = [i32]
        lib.glcm_last_hip_error.restype = i32
        lib.glcm_offset_polar.restype = i32
        lib.glcm_offset_polar.argtypes = [i32, i32, ctypes.POINTER(Offset)]
        lib.glcm_plan_create.restype = i32
        lib.glcm_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, ctypes.POINTER(Offset), i32, i32, u32]
        lib.glcm_plan_tuning.restype = i32
        lib.glcm_plan_tuning.argtypes = [vp, ctypes.POINTER(Tuning), i32]
        lib.glcm_plan_autotune.restype = i32
        lib.glcm_plan_autotune.argtypes = [vp, vp, i32, i32, i64, u32, u32, i32, vp, ctypes.POINTER(Tuning)]
        lib.glcm_plan_kernel_time.restype = i32
        lib.glcm_plan_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        lib.glcm_plan_destroy.restype = i32
        lib.glcm_plan_destroy.argtypes = [vp]
        lib.glcm_compute.restype = i32
        lib.glcm_compute.argtypes = [vp, vp, i32, i32, i64, i32, i32, u32, u32, ctypes.POINTER(Offset), i32, vp, vp]
        lib.glcm_compute_static.restype = i32
        lib.glcm_compute_static.argtypes = [vp, i32, i32, i64, i32, i32, u32, u32, ctypes.POINTER(Offset), i32, vp,
                                            vp]
        lib.glcm_features.restype = i32
        lib.glcm_features.argtypes = [vp, i32, i32, vp, vp]
        lib.glcm_histogram.restype = i32
        lib.glcm_histogram.argtypes = [vp, vp, i32, i32, i64, i32, i32, u32, u32, vp, vp]
        for name in ("glcm_symmetrize", "glcm_normalize", "glcm_haralick", "glcm_haralick_mcc"):
            getattr(lib, name).restype = i32
            getattr(lib, name).argtypes = [vp, i32, i32, vp, vp]
        lib.glcm_batch_tuning.restype = i32
        lib.glcm_batch_tuning.argtypes = [vp, ctypes.POINTER(BatchTuning), i32]
        lib.glcm_batch_autotune.restype = i32
        lib.glcm_batch_autotune.argtypes = [vp, ctypes.POINTER(Tile), i32, u32, u32, i32, ctypes.POINTER(BatchTuning)]
        lib.glcm_average.restype = i32
        lib.glcm_average.argtypes = [vp, i32, i32, i32, vp, vp]
        lib.glcm_batch_compute.restype = i32
        lib.glcm_batch_compute.argtypes = [vp, ctypes.POINTER(Tile), i32, u32, u32, vp, vp, vp]
        lib.glcm_batch_prepare.restype = i32
        lib.glcm_batch_prepare.argtypes = [vp, ctypes.POINTER(Tile), i32, ctypes.POINTER(vp)]
        lib.glcm_batch_run.restype = i32
        lib.glcm_batch_run.argtypes = [vp, u32, u32, vp, vp, vp]
        lib.glcm_batch_destroy.restype = i32
        lib.glcm_batch_destroy.argtypes = [vp]
        lib.glcm_plan_rebind.restype = i32
        lib.glcm_plan_rebind.argtypes = [vp, ctypes.POINTER(Offset), i32]
        lib.glcm_plan_workspace.restype = i32
        lib.glcm_plan_workspace.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        lib.glcm_plan_cache_stats.restype = i32
        lib.glcm_plan_cache_stats.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]
        lib.glcm_plan_cache_clear.restype = i32
        lib.glcm_plan_cache_clear.argtypes = []
        u64 = ctypes.c_uint64
        lib.glcm_server_create.restype = i32
        lib.glcm_server_create.argtypes = [ctypes.POINTER(vp), i32, u64, u64, u32]
        lib.glcm_server_submit.restype = i32
        lib.glcm_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]
        lib.glcm_server_query.restype = i32
        lib.glcm_server_query.argtypes = [vp, u64, ctypes.POINTER(RequestInfo)]
        lib.glcm_server_wait.restype = i32
        lib.glcm_server_wait.argtypes = [vp, u64, ctypes.POINTER(RequestInfo)]
        lib.glcm_server_fetch.restype = i32
        lib.glcm_server_fetch.argtypes = [vp, u64, vp, vp, vp]
        lib.glcm_server_release.restype = i32
        lib.glcm_server_release.argtypes = [vp, u64]
        lib.glcm_server_drain.restype = i32
        lib.glcm_server_drain.argtypes = [vp]
        lib.glcm_server_stats.restype = i32
        lib.glcm_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        lib.glcm_server_destroy.restype = i32
        lib.glcm_server_destroy.argtypes = [vp]
        _L = lib
    return _L


def _check(status: int, what: str):
    if status != 0:
        raise GlcmError(status, what)


def _offsets(offsets):
    offs = [(int(dx), int(dy)) for dx, dy in offsets]
    arr = (Offset * max(1, len(offs)))(*[Offset(dx, dy) for dx, dy in offs])
    return arr, len(offs)


def _stream_handle(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def glcm_abi_version() -> int:
    return int(_lib().glcm_abi_version())


def glcm_strerror(status: int) -> str:
    return _lib().glcm_strerror(status).decode()


def glcm_last_hip_error() -> int:
    return int(_lib().glcm_last_hip_error())


def glcm_offset_polar(d: int, theta_deg: int):
    o = Offset()
    _check(_lib().glcm_offset_polar(d, theta_deg, ctypes.byref(o)), "glcm_offset_polar")
    return (o.dx, o.dy)


class Plan:
    """Owner of a glcm_plan_t (workspace, upload stream and pinned staging)."""

    def __init__(self, handle, dtype, N, offsets):
        self.handle = handle
        self.dtype, self.N, self.offsets = dtype, N, [tuple(o) for o in offsets]

    @property
    def tuning(self) -> Tuning:
        t = Tuning()
        _check(_lib().glcm_plan_tuning(self.handle, ctypes.byref(t), 0), "glcm_plan_tuning")
        return t

    def set_tuning(self, **kw) -> Tuning:
        t = self.tuning
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(_lib().glcm_plan_tuning(self.handle, ctypes.byref(t), 1), "glcm_plan_tuning")
        return t

    def autotune(self, img, lo=0, hi=None, repeats=5, stream=None) -> Tuning:
        """Times the candidate layouts on `img` (a device tensor) and keeps the fastest."""
        ptr, W, H, stride, dt, keep = _image_args(img)
        if dt != self.dtype:
            raise ValueError("image dtype differs from the plan's")
        if hi is None:
            hi = 255 if dt == U8 else 65535
        t = Tuning()
        _check(_lib().glcm_plan_autotune(self.handle, ctypes.c_void_p(ptr), W, H, stride, int(lo), int(hi),
                                         int(repeats), _stream_handle(stream), ctypes.byref(t)),
               "glcm_plan_autotune")
        del keep
        return t

    @property
    def batch_tuning(self) -> BatchTuning:
        t = BatchTuning()
        _check(_lib().glcm_batch_tuning(self.handle, ctypes.byref(t), 0), "glcm_batch_tuning")
        return t

    def set_batch_tuning(self, replicas=0, min_rows=0, wg_size=0) -> BatchTuning:
        """Batch-kernel layout (0 = default): LDS copies per bin 4/8/16, shortest row run 1..256,
        threads per workgroup 256/512."""
        t = BatchTuning(int(replicas), int(min_rows), int(wg_size))
        _check(_lib().glcm_batch_tuning(self.handle, ctypes.byref(t), 1), "glcm_batch_tuning")
        return t

    def batch_autotune(self, images, lo=0, hi=None, repeats=3) -> BatchTuning:
        """Times the batch layouts on `images` (device tensors or a TileSet) and keeps the fastest."""
        ts = images if isinstance(images, TileSet) else TileSet(images, self.dtype)
        if hi is None:
            hi = 255 if self.dtype == U8 else 65535
        t = BatchTuning()
        _check(_lib().glcm_batch_autotune(self.handle, ts.tiles, ts.T, int(lo), int(hi), int(repeats),
                                          ctypes.byref(t)), "glcm_batch_autotune")
        return t

    def kernel_time(self):
        """(total ms, launches) of the counting kernel since the last read (plans made with FLAG_TIMING)."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        _check(_lib().glcm_plan_kernel_time(self.handle, ctypes.byref(ms), ctypes.byref(n)), "glcm_plan_kernel_time")
        return ms.value, n.value

    def close(self):
        if self.handle:
            _lib().glcm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def glcm_plan_create(dtype, N, offsets, max_W, max_H, flags=0) -> Plan:
    dt = _dtype_code(dtype)
    arr, K = _offsets(offsets)
    h = ctypes.c_void_p()
    _check(_lib().glcm_plan_create(ctypes.byref(h), dt, int(N), K, arr, int(max_W), int(max_H), int(flags)),
           "glcm_plan_create")
    return Plan(h, dt, N, offsets)


def glcm_plan_tuning(plan: Plan) -> Tuning:
    return plan.tuning


def glcm_plan_cache_stats():
    """(plans, device bytes) held by the internal cache behind plan=None calls."""
    n, b = ctypes.c_int32(), ctypes.c_uint64()
    _check(_lib().glcm_plan_cache_stats(ctypes.byref(n), ctypes.byref(b)), "glcm_plan_cache_stats")
    return n.value, b.value


def glcm_plan_cache_clear():
    """Destroys every idle plan of the internal cache."""
    _check(_lib().glcm_plan_cache_clear(), "glcm_plan_cache_clear")


def glcm_plan_autotune(plan: Plan, img, lo=0, hi=None, repeats=5, stream=None) -> Tuning:
    return plan.autotune(img, lo, hi, repeats, stream)


def glcm_plan_kernel_time(plan: Plan):
    return plan.kernel_time()


def glcm_plan_destroy(plan: Plan):
    plan.close()


def glcm_plan_rebind(plan: Plan, offsets):
    """Re-targets `plan` at another offset list of at most its creation K."""
    arr, K = _offsets(offsets)
    _check(_lib().glcm_plan_rebind(plan.handle, arr, K), "glcm_plan_rebind")
    plan.offsets = [tuple(o) for o in offsets]


def glcm_plan_workspace(plan: Plan) -> int:
    """Device bytes the plan holds now."""
    b = ctypes.c_size_t()
    _check(_lib().glcm_plan_workspace(plan.handle, ctypes.byref(b)), "glcm_plan_workspace")
    return int(b.value)


def _dtype_code(dtype) -> int:
    if dtype in (U8, U16):
        return dtype
    if dtype in (torch.uint8, np.uint8):
        return U8
    if dtype in (torch.uint16, np.uint16):
        return U16
    raise ValueError(f"unsupported pixel dtype {dtype}")


def _image_args(img):
    """(pointer, W, H, stride_elements, dtype_code, keepalive) of a 2-D image."""
    if isinstance(img, np.ndarray):
        if img.ndim != 2 or img.dtype not in (np.uint8, np.uint16):
            raise ValueError("img must be a 2-D uint8 or uint16 array")
        if img.strides[1] != img.itemsize or img.strides[0] % img.itemsize:
            img = np.ascontiguousarray(img)
        H, W = img.shape
        return img.ctypes.data, W, H, img.strides[0] // img.itemsize, _dtype_code(img.dtype), img
    if isinstance(img, torch.Tensor):
        if img.dim() != 2 or img.dtype not in (torch.uint8, torch.uint16):
            raise ValueError("img must be a 2-D torch.uint8 or torch.uint16 tensor")
        if img.stride(1) != 1:
            img = img.contiguous()
        H, W = img.shape
        return img.data_ptr(), W, H, img.stride(0), _dtype_code(img.dtype), img
    raise TypeError("img must be a numpy array or a torch tensor")


def glcm_compute(img, N, lo=0, hi=None, offsets=((1, 0),), out=None, stream=None, plan=None):
    """Co-occurrence counts of `img` for each offset, as a [K, N, N] uint32 tensor.

    `img` may live on the GPU (torch tensor) or on the host (numpy array or CPU
    tensor, pinned or pageable); host images are streamed to the GPU in row
    tiles.  `out`, if given, must be a contiguous device tensor of K*N*N 32-bit
    elements; it is overwritten."""
    ptr, W, H, stride, dt, keep = _image_args(img)
    if hi is None:
        hi = 255 if dt == U8 else 65535
    arr, K = _offsets(offsets)
    dev = img.device if isinstance(img, torch.Tensor) and img.is_cuda else torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty((K, N, N), dtype=torch.uint32, device=dev)
    elif not (out.is_cuda and out.is_contiguous() and out.numel() == K * N * N and out.element_size() == 4):
        raise ValueError("out must be a contiguous CUDA tensor of K*N*N 32-bit elements")
    s = _stream_handle(stream)
    _check(_lib().glcm_compute(plan.handle if plan is not None else None, ctypes.c_void_p(ptr), W, H, stride, dt,
                               int(N), int(lo), int(hi), arr, K, ctypes.c_void_p(out.data_ptr()), s),
           "glcm_compute")
    del keep
    return out


def glcm_compute_static(img, N, lo=0, hi=None, offsets=((1, 0),), out=None, stream=None):
    """glcm_compute for a device image without a plan and without device
    allocation inside the call (its merge uses the library's static per-GPU
    array; calls that overlap on one GPU race).  `out` should be given by
    callers that may not allocate; K * N * N <= STATIC_MAX_WORDS."""
    if not (isinstance(img, torch.Tensor) and img.is_cuda):
        raise ValueError("img must be a CUDA tensor")
    ptr, W, H, stride, dt, keep = _image_args(img)
    if hi is None:
        hi = 255 if dt == U8 else 65535
    arr, K = _offsets(offsets)
    if out is None:
        out = torch.empty((K, N, N), dtype=torch.uint32, device=img.device)
    elif not (out.is_cuda and out.is_contiguous() and out.numel() == K * N * N and out.element_size() == 4):
        raise ValueError("out must be a contiguous CUDA tensor of K*N*N 32-bit elements")
    _check(_lib().glcm_compute_static(ctypes.c_void_p(ptr), W, H, stride, dt, int(N), int(lo), int(hi), arr, K,
                                      ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
           "glcm_compute_static")
    del keep
    return out


def glcm_features(P, out=None, stream=None):
    """Contrast, energy, entropy, homogeneity and correlation of each GLCM in
    `P` ([K, N, N] or [N, N], 32-bit, on the GPU), as a [K, 5] float32 tensor."""
    if not (isinstance(P, torch.Tensor) and P.is_cuda and P.element_size() == 4 and P.is_contiguous()):
        raise ValueError("P must be a contiguous CUDA tensor of 32-bit counts")
    if P.dim() == 2:
        P = P.unsqueeze(0)
    K, N, N2 = P.shape
    if N != N2:
        raise ValueError("P must be [K, N, N]")
    if out is None:
        out = torch.empty((K, 5), dtype=torch.float32, device=P.device)
    s = _stream_handle(stream)
    _check(_lib().glcm_features(ctypes.c_void_p(P.data_ptr()), K, N, ctypes.c_void_p(out.data_ptr()), s),
           "glcm_features")
    return out


def glcm_histogram(img, N, lo=0, hi=None, out=None, stream=None, plan=None):
    """Histogram of the quantized levels of a device image, as an [N] uint32 tensor."""
    if not (isinstance(img, torch.Tensor) and img.is_cuda):
        raise ValueError("img must be a CUDA tensor")
    ptr, W, H, stride, dt, keep = _image_args(img)
    if hi is None:
        hi = 255 if dt == U8 else 65535
    if out is None:
        out = torch.empty(N, dtype=torch.uint32, device=img.device)
    elif not (out.is_cuda and out.is_contiguous() and out.numel() == N and out.element_size() == 4):
        raise ValueError("out must be a contiguous CUDA tensor of N 32-bit elements")
    _check(_lib().glcm_histogram(plan.handle if plan is not None else None, ctypes.c_void_p(ptr), W, H, stride, dt,
                                 int(N), int(lo), int(hi), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
           "glcm_histogram")
    del keep
    return out


def _matrices(P):
    if not (isinstance(P, torch.Tensor) and P.is_cuda and P.element_size() == 4 and P.is_contiguous()):
        raise ValueError("P must be a contiguous CUDA tensor of 32-bit counts")
    if P.dim() == 2:
        P = P.unsqueeze(0)
    if P.dim() != 3 or P.shape[1] != P.shape[2]:
        raise ValueError("P must be [K, N, N]")
    return P, P.shape[0], P.shape[1]


def _output(out, shape, dtype, device):
    if out is None:
        return torch.empty(shape, dtype=dtype, device=device)
    n = int(np.prod(shape))
    if not (out.is_cuda and out.is_contiguous() and out.numel() == n and out.element_size() == 4):
        raise ValueError(f"out must be a contiguous CUDA tensor of {n} 32-bit elements")
    return out


def glcm_symmetrize(P, out=None, stream=None):
    """P + P^T per matrix (uint32, modulo 2^32); out may be P itself."""
    P, K, N = _matrices(P)
    out = _output(out, (K, N, N), torch.uint32, P.device)
    _check(_lib().glcm_symmetrize(ctypes.c_void_p(P.data_ptr()), K, N, ctypes.c_void_p(out.data_ptr()),
                                  _stream_handle(stream)), "glcm_symmetrize")
    return out


def glcm_normalize(P, out=None, stream=None):
    """P / sum(P) per matrix, float32 (zeros for an empty matrix)."""
    P, K, N = _matrices(P)
    out = _output(out, (K, N, N), torch.float32, P.device)
    _check(_lib().glcm_normalize(ctypes.c_void_p(P.data_ptr()), K, N, ctypes.c_void_p(out.data_ptr()),
                                 _stream_handle(stream)), "glcm_normalize")
    return out


def glcm_average(P, m, out=None, stream=None):
    """Mean of the normalised matrices over consecutive groups of m, float32 [K/m, N, N]."""
    P, K, N = _matrices(P)
    if m < 1 or K % m:
        raise ValueError("K must be a positive multiple of m")
    out = _output(out, (K // m, N, N), torch.float32, P.device)
    _check(_lib().glcm_average(ctypes.c_void_p(P.data_ptr()), K, N, int(m), ctypes.c_void_p(out.data_ptr()),
                               _stream_handle(stream)), "glcm_average")
    return out


HARALICK_NAMES = ("asm", "contrast", "correlation", "variance", "idm", "sum_average", "sum_variance",
                  "sum_entropy", "entropy", "difference_variance", "difference_entropy", "imc1", "imc2")


def glcm_haralick(P, out=None, stream=None):
    """Haralick's statistics f1..f13 of each matrix (names in HARALICK_NAMES), float32 [K, 13]."""
    P, K, N = _matrices(P)
    out = _output(out, (K, 13), torch.float32, P.device)
    _check(_lib().glcm_haralick(ctypes.c_void_p(P.data_ptr()), K, N, ctypes.c_void_p(out.data_ptr()),
                                _stream_handle(stream)), "glcm_haralick")
    return out


def glcm_haralick_mcc(P, out=None, stream=None):
    """Haralick's maximal correlation coefficient (f14) of each matrix, float32 [K]."""
    P, K, N = _matrices(P)
    out = _output(out, (K,), torch.float32, P.device)
    _check(_lib().glcm_haralick_mcc(ctypes.c_void_p(P.data_ptr()), K, N, ctypes.c_void_p(out.data_ptr()),
                                    _stream_handle(stream)), "glcm_haralick_mcc")
    return out


class TileSet:
    """Descriptors of a batch of device images, built once and reusable."""

    def __init__(self, images, dtype):
        T = len(images)
        if T < 1:
            raise ValueError("images must not be empty")
        self.tiles = (Tile * T)()
        self.keep = []
        for i, img in enumerate(images):
            if not (isinstance(img, torch.Tensor) and img.is_cuda):
                raise ValueError("batch images must be CUDA tensors")
            ptr, W, H, stride, dt, k = _image_args(img)
            if dt != dtype:
                raise ValueError("image dtype differs from the plan's")
            self.tiles[i] = Tile(ptr, stride, W, H)
            self.keep.append(k)
        self.T = T
        self.device = images[0].device


def prepare_tiles(images, plan) -> TileSet:
    return TileSet(images, plan.dtype)


def glcm_batch_compute(images, plan, lo=0, hi=None, out=None, features=True, stream=None):
    """Counts (and statistics) of many device images in one launch.

    `images`: sequence of 2-D CUDA tensors (uint8 or uint16, the plan's dtype),
    any sizes up to the plan's max_W x max_H, or a TileSet from
    prepare_tiles().  Returns (out [T, K, N, N] uint32, feats [T, K, 5]
    float32 or None)."""
    ts = images if isinstance(images, TileSet) else TileSet(images, plan.dtype)
    T, tiles, dev = ts.T, ts.tiles, ts.device
    if hi is None:
        hi = 255 if plan.dtype == U8 else 65535
    K, N = len(plan.offsets), plan.N
    if out is None:
        out = torch.empty((T, K, N, N), dtype=torch.uint32, device=dev)
    elif not (out.is_cuda and out.is_contiguous() and out.numel() == T * K * N * N and out.element_size() == 4):
        raise ValueError("out must be a contiguous CUDA tensor of T*K*N*N 32-bit elements")
    feats = None
    if features is True:
        feats = torch.empty((T, K, 5), dtype=torch.float32, device=dev)
    elif isinstance(features, torch.Tensor):
        feats = features
    s = _stream_handle(stream)
    _check(_lib().glcm_batch_compute(plan.handle, tiles, T, int(lo), int(hi), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(feats.data_ptr()) if feats is not None else None, s),
           "glcm_batch_compute")
    return out, feats


class PreparedBatch:
    """A batch whose descriptors live on the device (glcm_batch_prepare):
    run() only queues kernels, so it can be captured in a graph.  The images
    (and the plan's dtype, N and offsets at preparation) are fixed; their
    pixels may change between runs."""

    def __init__(self, images, plan):
        ts = images if isinstance(images, TileSet) else TileSet(images, plan.dtype)
        h = ctypes.c_void_p()
        _check(_lib().glcm_batch_prepare(plan.handle, ts.tiles, ts.T, ctypes.byref(h)), "glcm_batch_prepare")
        self.handle, self.tileset = h, ts
        self.T, self.K, self.N, self.dtype = ts.T, len(plan.offsets), plan.N, plan.dtype

    def run(self, lo=0, hi=None, out=None, features=None, stream=None):
        """Queues the batch; returns (out [T, K, N, N], features or None)."""
        if hi is None:
            hi = 255 if self.dtype == U8 else 65535
        dev = self.tileset.device
        if out is None:
            out = torch.empty((self.T, self.K, self.N, self.N), dtype=torch.uint32, device=dev)
        elif not (out.is_cuda and out.is_contiguous() and out.numel() == self.T * self.K * self.N * self.N
                  and out.element_size() == 4):
            raise ValueError("out must be a contiguous CUDA tensor of T*K*N*N 32-bit elements")
        if features is True:
            features = torch.empty((self.T, self.K, 5), dtype=torch.float32, device=dev)
        _check(_lib().glcm_batch_run(self.handle, int(lo), int(hi), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(features.data_ptr()) if isinstance(features, torch.Tensor)
                                     else None, _stream_handle(stream)), "glcm_batch_run")
        return out, (features if isinstance(features, torch.Tensor) else None)

    def close(self):
        if self.handle:
            _lib().glcm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Owner of a glcm_server_t: requests of mixed size, N and offsets admitted
    onto `lanes` HIP streams as lanes and the HBM budget allow.

    submit() takes a 2-D image (a device tensor of any row stride, or a host
    numpy array or CPU tensor, pinned or pageable, which the lane streams to
    the GPU) and returns a ticket; results go to the given `out` / `feat`
    tensors or, if omitted, to the server's device pool (then read them with
    fetch() and free them with release()).  A host image must stay unchanged
    until its request is done (the server keeps a reference)."""

    def __init__(self, lanes=4, hbm_budget=32 << 30, result_pool_bytes=256 << 20):
        h = ctypes.c_void_p()
        _check(_lib().glcm_server_create(ctypes.byref(h), int(lanes), int(hbm_budget), int(result_pool_bytes), 0),
               "glcm_server_create")
        self.handle = h
        self._keep = {}  # ticket -> tensors the request reads or writes

    def submit(self, img, N, lo=0, hi=None, offsets=((1, 0),), features=False, out=None, feat=None) -> int:
        ptr, W, H, stride, dt, keep = _image_args(img)
        if hi is None:
            hi = 255 if dt == U8 else 65535
        arr, K = _offsets(offsets)
        for t, n in ((out, K * N * N), (feat, K * 5)):
            if t is not None and not (t.is_cuda and t.is_contiguous() and t.numel() == n and t.element_size() == 4):
                raise ValueError("out / feat must be contiguous CUDA tensors of K*N*N / K*5 32-bit elements")
        r = Request(ctypes.c_void_p(ptr), W, H, stride, dt, int(N), int(lo), int(hi),
                    ctypes.cast(arr, ctypes.c_void_p), K, 1 if features else 0,
                    ctypes.c_void_p(out.data_ptr() if out is not None else 0),
                    ctypes.c_void_p(feat.data_ptr() if feat is not None else 0))
        ticket = ctypes.c_uint64()
        _check(_lib().glcm_server_submit(self.handle, ctypes.byref(r), ctypes.byref(ticket)), "glcm_server_submit")
        self._keep[ticket.value] = (keep, out, feat, K, int(N), bool(features))
        return ticket.value

    def query(self, ticket) -> RequestInfo:
        info = RequestInfo()
        _check(_lib().glcm_server_query(self.handle, int(ticket), ctypes.byref(info)), "glcm_server_query")
        return info

    def wait(self, ticket) -> RequestInfo:
        info = RequestInfo()
        _check(_lib().glcm_server_wait(self.handle, int(ticket), ctypes.byref(info)), "glcm_server_wait")
        return info

    def fetch(self, ticket, stream=None):
        """Copies a done request's results into new tensors: (counts [K, N, N] uint32, statistics [K, 5] or None)."""
        _, _, _, K, N, feats = self._keep[int(ticket)]
        dev = torch.device("cuda", torch.cuda.current_device())
        out = torch.empty((K, N, N), dtype=torch.uint32, device=dev)
        feat = torch.empty((K, 5), dtype=torch.float32, device=dev) if feats else None
        _check(_lib().glcm_server_fetch(self.handle, int(ticket), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(feat.data_ptr() if feat is not None else 0),
                                        _stream_handle(stream)), "glcm_server_fetch")
        return out, feat

    def release(self, ticket):
        _check(_lib().glcm_server_release(self.handle, int(ticket)), "glcm_server_release")
        self._keep.pop(int(ticket), None)

    def drain(self):
        _check(_lib().glcm_server_drain(self.handle), "glcm_server_drain")

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(_lib().glcm_server_stats(self.handle, ctypes.byref(st)), "glcm_server_stats")
        return st

    def close(self):
        if self.handle:
            _lib().glcm_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
