"""ctypes wrapper of the FP64 C oracle (test infrastructure only)."""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gee_oracle.c")
_LIB = os.path.join(_HERE, "libgee_oracle.so")

# The oracle's own option bits (the C file defines the same meaning independently).
OR_DIAG = 1
OR_LAPLACIAN = 2
OR_CORRELATION = 4
OR_SYMMETRIZE = 8
OR_DIRECTED_DEGREES = 16

_ERRORS = {-1: "bad argument", -2: "label out of range", -3: "node index out of range",
           -4: "non-finite weight", -6: "out of host memory"}

_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return _LIB


def build_oracle(src: str = _SRC, out: str = _LIB, extra_flags=()) -> str:
    """Compile the C oracle with gcc into a shared library."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", *extra_flags, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def load(path: str | None = None):
    """Load (building first if absent) the oracle library; `path` loads another build."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build_oracle()
            _lib = _bind(ctypes.CDLL(_LIB))
        return _lib


def _bind(lib):
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.gee_oracle_class_counts.argtypes = [i32p, ctypes.c_int64, ctypes.c_int32, i64p]
    lib.gee_oracle_class_counts.restype = ctypes.c_int
    lib.gee_oracle_degrees.argtypes = [i32p, i32p, f64p, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_uint32, f64p]
    lib.gee_oracle_degrees.restype = ctypes.c_int
    lib.gee_oracle_in_degrees.argtypes = [i32p, i32p, f64p, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_uint32, f64p]
    lib.gee_oracle_in_degrees.restype = ctypes.c_int
    lib.gee_oracle_embed.argtypes = [i32p, i32p, f64p, ctypes.c_int64, ctypes.c_int64, i32p,
                                     ctypes.c_int32, ctypes.c_uint32, f64p]
    lib.gee_oracle_embed.restype = ctypes.c_int
    return lib


def _ptr(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _flags(diag, lap, cor, sym, deg_io=False):
    return ((OR_DIAG if diag else 0) | (OR_LAPLACIAN if lap else 0)
            | (OR_CORRELATION if cor else 0) | (OR_SYMMETRIZE if sym else 0)
            | (OR_DIRECTED_DEGREES if deg_io else 0))


class OracleError(ValueError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}: {_ERRORS.get(code, 'unknown')}")
        self.code = code


def _prep(src, dst, w):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    w64 = None if w is None else np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    return src, dst, w64


def class_counts(labels, K: int, lib=None) -> np.ndarray:
    lib = lib or load()
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.zeros(K, dtype=np.int64)
    rc = lib.gee_oracle_class_counts(_ptr(labels, ctypes.c_int32), labels.shape[0], K,
                                     _ptr(out, ctypes.c_int64))
    if rc:
        raise OracleError(rc)
    return out


def degrees(src, dst, w, N: int, diag=False, sym=True, lib=None) -> np.ndarray:
    lib = lib or load()
    src, dst, w64 = _prep(src, dst, w)
    out = np.zeros(max(N, 1), dtype=np.float64)
    rc = lib.gee_oracle_degrees(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                                _ptr(w64, ctypes.c_double), src.shape[0], N,
                                _flags(diag, False, False, sym), _ptr(out, ctypes.c_double))
    if rc:
        raise OracleError(rc)
    return out[:N]


def in_degrees(src, dst, w, N: int, diag=False, sym=True, lib=None) -> np.ndarray:
    """Column sums of A (+ I): the in-degrees of the directed-degree Laplacian."""
    lib = lib or load()
    src, dst, w64 = _prep(src, dst, w)
    out = np.zeros(max(N, 1), dtype=np.float64)
    rc = lib.gee_oracle_in_degrees(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                                   _ptr(w64, ctypes.c_double), src.shape[0], N,
                                   _flags(diag, False, False, sym), _ptr(out, ctypes.c_double))
    if rc:
        raise OracleError(rc)
    return out[:N]


def embed(src, dst, w, N: int, labels, K: int, diag=False, lap=False, cor=False, sym=True,
          lib=None, deg_io=False) -> np.ndarray:
    """Z (float64, N x K) for one edge list; `w` None means every weight is 1. `deg_io`:
    under the Laplacian, out-degrees on the left and in-degrees on the right."""
    lib = lib or load()
    src, dst, w64 = _prep(src, dst, w)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    Z = np.zeros((max(N, 0), K), dtype=np.float64)
    rc = lib.gee_oracle_embed(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                              _ptr(w64, ctypes.c_double), src.shape[0], N,
                              _ptr(labels, ctypes.c_int32), K, _flags(diag, lap, cor, sym, deg_io),
                              _ptr(Z, ctypes.c_double))
    if rc:
        raise OracleError(rc)
    return Z


def embed_graph(g, lib=None) -> np.ndarray:
    """`embed` for a gee_workloads.Graph."""
    return embed(g.src, g.dst, g.w, g.N, g.labels, g.K, diag=g.diag, lap=g.lap, cor=g.cor,
                 sym=g.sym, lib=lib, deg_io=getattr(g, "deg_io", False))
