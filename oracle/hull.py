"""TEST INFRASTRUCTURE ONLY: ctypes front end of the plain C hull oracle.

``andrew_hull.c`` holds the arithmetic (Andrew's monotone chain with exact
int64 orientation tests, the paper's reference [4]); this file only builds it
with gcc, loads it and marshals numpy arrays.  Nothing in the product package
imports this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "andrew_hull.c")
_LIB = os.path.join(_HERE, "liboracle_hull.so")
_lib = None


class OracleDomainError(ValueError):
    """The input holds a value outside integer [0, 2**23)."""


def build() -> str:
    """Compile the C oracle with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_hull.restype = ctypes.c_int
    lib.oracle_hull.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_first_invalid.restype = ctypes.c_int64
    lib.oracle_first_invalid.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    _lib = lib
    return lib


def _as_points(points) -> np.ndarray:
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32))
    if pts.ndim != 2 or pts.shape[1] != 2:
        raise ValueError("points must have shape [n, 2]")
    return pts


def first_invalid(points) -> int:
    pts = _as_points(points)
    return int(_load().oracle_first_invalid(pts.ctypes.data, pts.shape[0]))


def hull(points) -> np.ndarray:
    """Hull vertex indices (int32), CCW from the lowest-then-leftmost vertex."""
    pts = _as_points(points)
    n = pts.shape[0]
    out = np.empty(max(n, 1), dtype=np.int32)
    h = ctypes.c_int64(0)
    rc = _load().oracle_hull(pts.ctypes.data, n, out.ctypes.data, ctypes.byref(h))
    if rc == -2:
        raise OracleDomainError("point coordinates must be integers in [0, 2**23)")
    if rc != 0:
        raise RuntimeError(f"oracle_hull failed with status {rc}")
    return out[: h.value].copy()
