"""CPU oracle for GLCM counts and Haralick statistics (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The library and its Python binding never do: the oracle shares
no code with the HIP path.  The arithmetic lives in ``glcm_oracle.c`` (plain C,
built with gcc); this module only builds it and marshals numpy arrays.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glcm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_quantize.restype = ctypes.c_uint32
        lib.oracle_quantize.argtypes = [ctypes.c_uint32] * 4
        lib.oracle_glcm_rows.restype = ctypes.c_int
        lib.oracle_glcm_rows.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
            ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_features.restype = None
        lib.oracle_features.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_histogram.restype = ctypes.c_int
        lib.oracle_histogram.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        for name in ("oracle_symmetric", "oracle_normalize"):
            getattr(lib, name).restype = None
            getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_average.restype = None
        lib.oracle_average.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_haralick.restype = ctypes.c_int
        lib.oracle_haralick.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        _lib = lib
    return _lib


def quantize(v: int, N: int, lo: int, hi: int) -> int:
    return int(_load().oracle_quantize(v, N, lo, hi))


def quantize_array(values, N: int, lo: int, hi: int) -> np.ndarray:
    q = _load().oracle_quantize
    return np.array([q(int(v), N, lo, hi) for v in np.asarray(values).ravel()],
                    dtype=np.int64).reshape(np.shape(values))


def glcm(img: np.ndarray, N: int, lo: int, hi: int, offsets, rows=None) -> np.ndarray:
    """Counts P[k][i][j] (uint32) of a 2-D uint8/uint16 image for offsets (dx, dy).

    ``img`` may be a strided view (row stride in elements, unit column stride).
    ``rows=(y0, y1)`` restricts the FIRST pixel to rows y0..y1-1."""
    img = np.asarray(img)
    if img.ndim != 2 or img.dtype not in (np.uint8, np.uint16):
        raise ValueError("img must be a 2-D uint8 or uint16 array")
    if img.strides[1] != img.itemsize:
        img = np.ascontiguousarray(img)
    H, W = img.shape
    stride = img.strides[0] // img.itemsize
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 2))
    K = offs.shape[0]
    out = np.zeros((K, N, N), dtype=np.uint32)
    y0, y1 = (0, H) if rows is None else rows
    rc = _load().oracle_glcm_rows(img.ctypes.data, W, H, stride, img.itemsize, N, lo, hi,
                                  offs.ctypes.data, K, y0, y1, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_glcm_rows rejected its arguments or a count overflowed")
    return out


def features(P: np.ndarray) -> np.ndarray:
    """Five statistics per GLCM in float64: contrast, energy, entropy,
    homogeneity, correlation.  ``P`` has shape [K, N, N] (or [N, N])."""
    P = np.ascontiguousarray(P, dtype=np.uint32)
    squeeze = P.ndim == 2
    if squeeze:
        P = P[None]
    K, N, _ = P.shape
    out = np.zeros((K, 5), dtype=np.float64)
    _load().oracle_features(P.ctypes.data, K, N, out.ctypes.data)
    return out[0] if squeeze else out


def histogram(img: np.ndarray, N: int, lo: int, hi: int) -> np.ndarray:
    """h[i] (uint32, N entries) = number of pixels of a 2-D uint8/uint16 image
    (strided views allowed) whose quantized level is i."""
    img = np.asarray(img)
    if img.ndim != 2 or img.dtype not in (np.uint8, np.uint16):
        raise ValueError("img must be a 2-D uint8 or uint16 array")
    if img.strides[1] != img.itemsize:
        img = np.ascontiguousarray(img)
    H, W = img.shape
    out = np.zeros(N, dtype=np.uint32)
    rc = _load().oracle_histogram(img.ctypes.data, W, H, img.strides[0] // img.itemsize, img.itemsize,
                                  N, lo, hi, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_histogram rejected its arguments")
    return out


def _stack(P: np.ndarray):
    P = np.ascontiguousarray(P, dtype=np.uint32)
    squeeze = P.ndim == 2
    return (P[None] if squeeze else P), squeeze


def symmetric(P: np.ndarray) -> np.ndarray:
    """P + P^T per matrix (uint32, modulo 2^32); shape [K, N, N] or [N, N]."""
    P, squeeze = _stack(P)
    K, N, _ = P.shape
    out = np.empty_like(P)
    _load().oracle_symmetric(P.ctypes.data, K, N, out.ctypes.data)
    return out[0] if squeeze else out


def normalize(P: np.ndarray) -> np.ndarray:
    """P / sum(P) per matrix in float64 (all zeros for an empty matrix)."""
    P, squeeze = _stack(P)
    K, N, _ = P.shape
    out = np.empty(P.shape, dtype=np.float64)
    _load().oracle_normalize(P.ctypes.data, K, N, out.ctypes.data)
    return out[0] if squeeze else out


def average(P: np.ndarray, m: int) -> np.ndarray:
    """Mean of the normalised matrices over consecutive groups of m, float64
    [K/m, N, N]."""
    P, _ = _stack(P)
    K, N, _ = P.shape
    if m < 1 or K % m:
        raise ValueError("K must be a positive multiple of m")
    out = np.empty((K // m, N, N), dtype=np.float64)
    _load().oracle_average(P.ctypes.data, K, N, m, out.ctypes.data)
    return out


HARALICK_NAMES = ("asm", "contrast", "correlation", "variance", "idm", "sum_average", "sum_variance",
                  "sum_entropy", "entropy", "difference_variance", "difference_entropy", "imc1", "imc2")


def haralick(P: np.ndarray) -> np.ndarray:
    """Haralick's f1..f13 per matrix in float64, shape [K, 13] (or [13])."""
    P, squeeze = _stack(P)
    K, N, _ = P.shape
    out = np.zeros((K, 13), dtype=np.float64)
    if _load().oracle_haralick(P.ctypes.data, K, N, out.ctypes.data) != 0:
        raise MemoryError("oracle_haralick could not allocate")
    return out[0] if squeeze else out


def haralick_mcc(P: np.ndarray) -> np.ndarray:
    """Haralick's fourteenth statistic, the maximal correlation coefficient,
    per matrix in float64: the square root of the second largest eigenvalue of
    Q(i, j) = sum_k p(i, k) p(j, k) / (px(i) py(k)), p = P / T (cited in the
    introduction with the other thirteen).  Terms with px(i) = 0 or py(k) = 0
    are 0; an empty matrix or a single eigenvalue gives 0.  The eigenvalues
    come from numpy's general (non-symmetric) eigenvalue routine."""
    P, squeeze = _stack(P)
    out = np.zeros(P.shape[0], dtype=np.float64)
    for k, M in enumerate(P):
        T = int(M.astype(np.uint64).sum())
        if T == 0:
            continue
        p = M.astype(np.float64) / T
        px, py = p.sum(axis=1), p.sum(axis=0)
        N = p.shape[0]
        # Q(i, j) = sum_c [p(i, c) / px(i)] [p(j, c) / py(c)], as one matrix product
        A = np.divide(p, px[:, None], out=np.zeros_like(p), where=px[:, None] > 0)
        C = np.divide(p, py[None, :], out=np.zeros_like(p), where=py[None, :] > 0)
        Q = A @ C.T
        ev = np.sort(np.linalg.eigvals(Q).real)[::-1]
        out[k] = np.sqrt(max(0.0, ev[1])) if N > 1 else 0.0
    return out[0] if squeeze else out
