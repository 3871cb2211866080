"""ctypes declarations of libgee.so (the C ABI of include/gee.h)."""

from __future__ import annotations

import ctypes
import os
import threading

import torch  # noqa: F401  (loads torch's HIP runtime first, so libgee shares it)

from .build import LIB

_lock = threading.Lock()
_lib = None

c_i32p = ctypes.c_void_p  # device pointers are passed as plain addresses
c_f32p = ctypes.c_void_p


class GeeSchedule(ctypes.Structure):
    _fields_ = [("wave_entries", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("tile_entries", ctypes.c_int32), ("bucket_rows_log2", ctypes.c_int32)]


class GeeGraph(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("E", ctypes.c_int64), ("N", ctypes.c_int32), ("labels", ctypes.c_void_p),
                ("K", ctypes.c_int32), ("flags", ctypes.c_uint32), ("Z", ctypes.c_void_p),
                ("sched", GeeSchedule)]


SYMBOLS = {
    # name: (restype, argtypes)
    "gee_abi_version": (ctypes.c_int, []),
    "gee_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gee_last_hip_error": (ctypes.c_char_p, []),
    "gee_init": (ctypes.c_int, []),
    "gee_profile_kernel": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gee_get_data_errors": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "gee_take_data_errors_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gee_default_schedule": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_uint32, ctypes.POINTER(GeeSchedule)]),
    "gee_class_counts": (ctypes.c_int, [c_i32p, ctypes.c_int32, ctypes.c_int32, c_i32p,
                                        ctypes.c_void_p]),
    "gee_csr_capacity": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_uint32]),
    "gee_build_csr_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                                         ctypes.POINTER(GeeSchedule)]),
    "gee_build_csr": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_uint32, c_i32p, c_i32p, c_f32p, ctypes.c_void_p]),
    "gee_build_csr_ws": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_uint32, c_i32p, c_i32p, c_f32p,
                                        ctypes.POINTER(GeeSchedule), ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "gee_embed_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                     ctypes.c_uint32, ctypes.c_int,
                                                     ctypes.POINTER(GeeSchedule)]),
    "gee_embed": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                 ctypes.c_int32, ctypes.c_uint32, c_f32p, ctypes.c_void_p]),
    "gee_embed_ws": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                    ctypes.c_int32, ctypes.c_uint32, c_f32p, ctypes.POINTER(GeeSchedule),
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gee_scratch_bytes": (ctypes.c_size_t, []),
    "gee_embed_noalloc": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                         ctypes.c_int32, ctypes.c_uint32, c_f32p, ctypes.c_void_p]),
    "gee_embed_csr_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                         ctypes.c_uint32, ctypes.POINTER(GeeSchedule)]),
    "gee_embed_csr": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                     ctypes.c_int32, ctypes.c_uint32, c_f32p, ctypes.c_void_p]),
    "gee_embed_csr_ws": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                        ctypes.c_int32, ctypes.c_uint32, c_f32p,
                                        ctypes.POINTER(GeeSchedule), ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "gee_embed_sparse_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                            ctypes.c_uint32, ctypes.c_int,
                                                            ctypes.POINTER(GeeSchedule)]),
    "gee_embed_sparse": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                        ctypes.c_int32, ctypes.c_uint32, c_i32p, c_i32p, c_f32p,
                                        ctypes.c_int64, ctypes.c_void_p]),
    "gee_embed_sparse_ws": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                           ctypes.c_int32, ctypes.c_uint32, c_i32p, c_i32p, c_f32p,
                                           ctypes.c_int64, ctypes.POINTER(GeeSchedule), ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_void_p]),
    "gee_embed_atomic_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]),
    "gee_embed_atomic": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                        ctypes.c_int32, ctypes.c_uint32, c_f32p, ctypes.c_void_p]),
    "gee_embed_atomic_ws": (ctypes.c_int, [c_i32p, c_i32p, c_f32p, ctypes.c_int64, ctypes.c_int32, c_i32p,
                                           ctypes.c_int32, ctypes.c_uint32, c_f32p, ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_void_p]),
    "gee_embed_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(GeeGraph), ctypes.c_int32]),
    "gee_embed_batch_ws": (ctypes.c_int, [ctypes.POINTER(GeeGraph), ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "gee_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(GeeGraph), ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "gee_batch_plan_create_ws": (ctypes.c_int, [ctypes.POINTER(GeeGraph), ctypes.c_int32, ctypes.c_size_t,
                                                ctypes.POINTER(ctypes.c_void_p)]),
    "gee_batch_plan_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "gee_batch_plan_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GeeGraph), ctypes.c_int32]),
    "gee_batch_plan_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gee_batch_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}


def lib_path() -> str:
    """libgee.so in the package, or the build GEE_LIBRARY names (e.g. the GEE_DEBUG build
    libgee_debug.so beside it)."""
    return os.environ.get("GEE_LIBRARY") or LIB


def load():
    """Load libgee.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    with _lock:
        if _lib is None:
            path = lib_path()
            if not os.path.exists(path):
                raise RuntimeError(
                    f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                    "(or python -m paper_2406_03726_amd.build). The GEE path has no CPU fallback.")
            lib = ctypes.CDLL(path)
            for name, (res, args) in SYMBOLS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
        return _lib
