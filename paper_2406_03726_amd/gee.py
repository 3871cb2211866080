"""Python binding of libgee: the C ABI's entry points under the same names.

Argument marshalling only: tensors are checked for device, dtype and layout and their
device addresses and the current HIP stream are handed to the library. Every step of
the embedding runs in the library's HIP kernels; there is no CPU path.
"""

from __future__ import annotations

import contextlib
import ctypes
from typing import Optional

import torch

from . import _lib

GEE_DIAG = 1 << 0
GEE_LAPLACIAN = 1 << 1
GEE_CORRELATION = 1 << 2
GEE_SYMMETRIZE = 1 << 3
GEE_DIRECTED_DEGREES = 1 << 4
GEE_NO_VALIDATE = 1 << 8

GEE_DATA_INTERNAL = 1 << 30  # GEE_DEBUG builds only
GEE_DATA_LABEL = 1 << 0
GEE_DATA_INDEX = 1 << 1
GEE_DATA_WEIGHT = 1 << 2
GEE_DATA_CSR = 1 << 3

GEE_OK = 0
GEE_ERR_ARG = -1
GEE_ERR_TOO_LARGE = -5
GEE_ERR_OOM = -6
GEE_ERR_HIP = -7
GEE_ERR_UNSUPPORTED = -8
GEE_ERR_WORKSPACE = -9
GEE_ERR_SCRATCH = -10


class GeeError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib.load()
        msg = lib.gee_status_string(code).decode()
        hip = lib.gee_last_hip_error().decode() if code in (GEE_ERR_HIP, GEE_ERR_OOM) else ""
        super().__init__(f"{where}: {msg} ({code})" + (f": {hip}" if hip else ""))
        self.code = code


def flags_of(diag=False, lap=False, cor=False, sym=True, deg_io=False) -> int:
    return ((GEE_DIAG if diag else 0) | (GEE_LAPLACIAN if lap else 0)
            | (GEE_CORRELATION if cor else 0) | (GEE_SYMMETRIZE if sym else 0)
            | (GEE_DIRECTED_DEGREES if deg_io else 0))


def _check(rc: int, where: str):
    if rc != GEE_OK:
        raise GeeError(rc, where)


def _dev(t: Optional[torch.Tensor], dtype, name: str, device=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _on(stream):
    """Allocations made by a call belong to the stream its kernels run on: torch's caching
    allocator then hands their memory to another stream only after that stream's work on
    it is done (a workspace freed when the call returns is not reused under the kernels)."""
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


def schedule(wave_entries=0, waves_per_block=0, tile_entries=0, bucket_rows_log2=0) -> _lib.GeeSchedule:
    return _lib.GeeSchedule(wave_entries, waves_per_block, tile_entries, bucket_rows_log2)


def _sched_ptr(s):
    if s is None:
        return None
    if isinstance(s, dict):
        s = schedule(**s)
    return ctypes.byref(s)


def gee_abi_version() -> int:
    return _lib.load().gee_abi_version()


def gee_init() -> None:
    _check(_lib.load().gee_init(), "gee_init")


def gee_get_data_errors(stream=None) -> int:
    bits = ctypes.c_uint32(0)
    _check(_lib.load().gee_get_data_errors(_stream(stream), ctypes.byref(bits)), "gee_get_data_errors")
    return int(bits.value)


def gee_take_data_errors_async(dst: torch.Tensor, stream=None) -> None:
    """Enqueue the take of the stream's data-error bits into dst[0] (an int32 tensor in
    device memory or pinned host memory); read dst once the stream has passed this point."""
    if dst.dtype != torch.int32 or dst.numel() < 1:
        raise ValueError("dst must hold an int32")
    if not dst.is_cuda and not dst.is_pinned():
        raise ValueError("dst must be device memory or pinned host memory")
    _check(_lib.load().gee_take_data_errors_async(_stream(stream), ctypes.c_void_p(dst.data_ptr())),
           "gee_take_data_errors_async")


def gee_default_schedule(E: int, N: int, K: int, flags: int) -> dict:
    s = _lib.GeeSchedule()
    _check(_lib.load().gee_default_schedule(E, N, K, flags, ctypes.byref(s)), "gee_default_schedule")
    return {f: getattr(s, f) for f, _ in _lib.GeeSchedule._fields_}


def gee_class_counts(labels: torch.Tensor, K: int, counts: Optional[torch.Tensor] = None,
                     stream=None) -> torch.Tensor:
    labels = _dev(labels, torch.int32, "labels")
    with _on(stream):
        if counts is None:
            counts = torch.empty(K, dtype=torch.int32, device=labels.device)
        _dev(counts, torch.int32, "counts", labels.device)
        _check(_lib.load().gee_class_counts(_ptr(labels), labels.numel(), K, _ptr(counts), _stream(stream)),
               "gee_class_counts")
    return counts


def gee_csr_capacity(E: int, flags: int) -> int:
    return int(_lib.load().gee_csr_capacity(E, flags))


def gee_build_csr(src: torch.Tensor, dst: torch.Tensor, w: Optional[torch.Tensor], N: int, flags: int,
                  row_ptr: Optional[torch.Tensor] = None, col: Optional[torch.Tensor] = None,
                  val: Optional[torch.Tensor] = None, sched=None, stream=None,
                  workspace: Optional[torch.Tensor] = None):
    """Returns (row_ptr, col, val) with col/val at full capacity; the entry count is
    row_ptr[N] (read it with row_ptr[-1].item() when needed)."""
    src = _dev(src, torch.int32, "src")
    dst = _dev(dst, torch.int32, "dst", src.device)
    w = _dev(w, torch.float32, "w", src.device)
    E = src.numel()
    if dst.numel() != E or (w is not None and w.numel() != E):
        raise ValueError("src, dst and w must have the same length")
    cap = gee_csr_capacity(E, flags)
    dev = src.device
    lib = _lib.load()
    sp = _sched_ptr(sched)
    nbytes = lib.gee_build_csr_workspace_bytes(E, N, flags, sp)
    if nbytes == 0:
        raise GeeError(GEE_ERR_ARG, "gee_build_csr_workspace_bytes")
    with _on(stream):
        if row_ptr is None:
            row_ptr = torch.empty(N + 1, dtype=torch.int32, device=dev)
        if col is None:
            col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        if val is None and w is not None:
            val = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        ws = workspace if workspace is not None and workspace.numel() >= nbytes else \
            torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _check(lib.gee_build_csr_ws(_ptr(src), _ptr(dst), _ptr(w), E, N, flags, _ptr(row_ptr), _ptr(col),
                                    _ptr(val), sp, _ptr(ws), ws.numel(), _stream(stream)), "gee_build_csr")
    return row_ptr, col, val


def gee_build_csr_workspace_bytes(E: int, N: int, flags: int, sched=None) -> int:
    return int(_lib.load().gee_build_csr_workspace_bytes(E, N, flags, _sched_ptr(sched)))


def gee_embed(src: torch.Tensor, dst: torch.Tensor, w: Optional[torch.Tensor], labels: torch.Tensor,
              K: int, flags: int, Z: Optional[torch.Tensor] = None, sched=None,
              workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Z (float32, N x K) of the edge list; N is labels.numel()."""
    labels = _dev(labels, torch.int32, "labels")
    dev = labels.device
    src = _dev(src, torch.int32, "src", dev)
    dst = _dev(dst, torch.int32, "dst", dev)
    w = _dev(w, torch.float32, "w", dev)
    E = src.numel()
    N = labels.numel()
    if dst.numel() != E or (w is not None and w.numel() != E):
        raise ValueError("src, dst and w must have the same length")
    lib = _lib.load()
    sp = _sched_ptr(sched)
    nbytes = lib.gee_embed_workspace_bytes(E, N, K, flags, int(w is not None), sp)
    if nbytes == 0 and N > 0:
        raise GeeError(GEE_ERR_ARG if E >= 0 else GEE_ERR_TOO_LARGE, "gee_embed_workspace_bytes")
    with _on(stream):
        if Z is None:
            Z = torch.empty((N, K), dtype=torch.float32, device=dev)
        _dev(Z, torch.float32, "Z", dev)
        if Z.numel() != N * K:
            raise ValueError("Z must hold N * K floats")
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        _check(lib.gee_embed_ws(_ptr(src), _ptr(dst), _ptr(w), E, N, _ptr(labels), K, flags, _ptr(Z), sp,
                                _ptr(workspace), workspace.numel(), _stream(stream)), "gee_embed")
    return Z


def gee_scratch_bytes() -> int:
    """Size of the library's fixed scratch (the most workspace gee_embed_noalloc can use)."""
    return int(_lib.load().gee_scratch_bytes())


def gee_embed_noalloc(src: torch.Tensor, dst: torch.Tensor, w: Optional[torch.Tensor], labels: torch.Tensor,
                      K: int, flags: int, Z: torch.Tensor, stream=None) -> torch.Tensor:
    """gee_embed into a caller's Z with the library's fixed scratch as workspace: nothing is
    allocated (neither by the library nor here). Calls overlapping on one device race."""
    labels = _dev(labels, torch.int32, "labels")
    dev = labels.device
    src = _dev(src, torch.int32, "src", dev)
    dst = _dev(dst, torch.int32, "dst", dev)
    w = _dev(w, torch.float32, "w", dev)
    _dev(Z, torch.float32, "Z", dev)
    E = src.numel()
    N = labels.numel()
    if dst.numel() != E or (w is not None and w.numel() != E):
        raise ValueError("src, dst and w must have the same length")
    if Z.numel() != N * K:
        raise ValueError("Z must hold N * K floats")
    _check(_lib.load().gee_embed_noalloc(_ptr(src), _ptr(dst), _ptr(w), E, N, _ptr(labels), K, flags, _ptr(Z),
                                         _stream(stream)), "gee_embed_noalloc")
    return Z


def gee_embed_workspace_bytes(E: int, N: int, K: int, flags: int, weighted: bool, sched=None) -> int:
    return int(_lib.load().gee_embed_workspace_bytes(E, N, K, flags, int(weighted), _sched_ptr(sched)))


def gee_embed_csr(row_ptr: torch.Tensor, col: torch.Tensor, val: Optional[torch.Tensor], M: int,
                  labels: torch.Tensor, K: int, flags: int, Z: Optional[torch.Tensor] = None,
                  sched=None, workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Z from a resident CSR with M entries (row_ptr[N] must equal M)."""
    labels = _dev(labels, torch.int32, "labels")
    dev = labels.device
    row_ptr = _dev(row_ptr, torch.int32, "row_ptr", dev)
    col = _dev(col, torch.int32, "col", dev)
    val = _dev(val, torch.float32, "val", dev)
    N = labels.numel()
    if row_ptr.numel() != N + 1 or col.numel() < M or (val is not None and val.numel() < M):
        raise ValueError("row_ptr must have N + 1 entries and col/val at least M")
    lib = _lib.load()
    sp = _sched_ptr(sched)
    nbytes = lib.gee_embed_csr_workspace_bytes(M, N, K, flags, sp)
    with _on(stream):
        if Z is None:
            Z = torch.empty((N, K), dtype=torch.float32, device=dev)
        _dev(Z, torch.float32, "Z", dev)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        _check(lib.gee_embed_csr_ws(_ptr(row_ptr), _ptr(col), _ptr(val), M, N, _ptr(labels), K, flags,
                                    _ptr(Z), sp, _ptr(workspace), workspace.numel(), _stream(stream)),
               "gee_embed_csr")
    return Z


def gee_embed_csr_workspace_bytes(M: int, N: int, K: int, flags: int, sched=None) -> int:
    return int(_lib.load().gee_embed_csr_workspace_bytes(M, N, K, flags, _sched_ptr(sched)))


def gee_embed_sparse_workspace_bytes(E: int, N: int, K: int, flags: int, weighted: bool, sched=None) -> int:
    return int(_lib.load().gee_embed_sparse_workspace_bytes(E, N, K, flags, int(weighted), _sched_ptr(sched)))


def gee_embed_sparse(src: torch.Tensor, dst: torch.Tensor, w: Optional[torch.Tensor], labels: torch.Tensor,
                     K: int, flags: int, capacity: Optional[int] = None, row_ptr: Optional[torch.Tensor] = None,
                     col: Optional[torch.Tensor] = None, val: Optional[torch.Tensor] = None, sched=None,
                     workspace: Optional[torch.Tensor] = None, stream=None):
    """Z in sparse storage: (row_ptr int32[N + 1], col int32[capacity], val float32[capacity]).
    The number of stored entries is row_ptr[N]; capacity defaults to N * K (always enough)."""
    labels = _dev(labels, torch.int32, "labels")
    dev = labels.device
    src = _dev(src, torch.int32, "src", dev)
    dst = _dev(dst, torch.int32, "dst", dev)
    w = _dev(w, torch.float32, "w", dev)
    E = src.numel()
    N = labels.numel()
    if dst.numel() != E or (w is not None and w.numel() != E):
        raise ValueError("src, dst and w must have the same length")
    if capacity is None:
        capacity = N * K if col is None else col.numel()
    lib = _lib.load()
    sp = _sched_ptr(sched)
    nbytes = lib.gee_embed_sparse_workspace_bytes(E, N, K, flags, int(w is not None), sp)
    if nbytes == 0:
        raise GeeError(GEE_ERR_ARG if E >= 0 else GEE_ERR_TOO_LARGE, "gee_embed_sparse_workspace_bytes")
    with _on(stream):
        if row_ptr is None:
            row_ptr = torch.empty(N + 1, dtype=torch.int32, device=dev)
        if col is None and capacity > 0:
            col = torch.empty(capacity, dtype=torch.int32, device=dev)
        if val is None and capacity > 0:
            val = torch.empty(capacity, dtype=torch.float32, device=dev)
        _dev(row_ptr, torch.int32, "row_ptr", dev)
        _dev(col, torch.int32, "col", dev)
        _dev(val, torch.float32, "val", dev)
        if row_ptr.numel() != N + 1 or (capacity > 0 and (col.numel() < capacity or val.numel() < capacity)):
            raise ValueError("row_ptr must have N + 1 entries and col/val at least capacity")
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _check(lib.gee_embed_sparse_ws(_ptr(src), _ptr(dst), _ptr(w), E, N, _ptr(labels), K, flags,
                                       _ptr(row_ptr), _ptr(col), _ptr(val), capacity, sp, _ptr(workspace),
                                       workspace.numel(), _stream(stream)), "gee_embed_sparse")
    return row_ptr, col, val


def gee_embed_atomic_workspace_bytes(N: int, K: int, flags: int) -> int:
    return int(_lib.load().gee_embed_atomic_workspace_bytes(N, K, flags))


def gee_embed_atomic(src: torch.Tensor, dst: torch.Tensor, w: Optional[torch.Tensor], labels: torch.Tensor,
                     K: int, flags: int, Z: Optional[torch.Tensor] = None,
                     workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Z (float32, N x K) of the edge list by the original, edge-list form of GEE (float
    atomics: the last bits of Z may differ between calls); N is labels.numel()."""
    labels = _dev(labels, torch.int32, "labels")
    dev = labels.device
    src = _dev(src, torch.int32, "src", dev)
    dst = _dev(dst, torch.int32, "dst", dev)
    w = _dev(w, torch.float32, "w", dev)
    E = src.numel()
    N = labels.numel()
    if dst.numel() != E or (w is not None and w.numel() != E):
        raise ValueError("src, dst and w must have the same length")
    lib = _lib.load()
    nbytes = lib.gee_embed_atomic_workspace_bytes(N, K, flags)
    if nbytes == 0 and N > 0:
        raise GeeError(GEE_ERR_ARG, "gee_embed_atomic_workspace_bytes")
    with _on(stream):
        if Z is None:
            Z = torch.empty((N, K), dtype=torch.float32, device=dev)
        _dev(Z, torch.float32, "Z", dev)
        if Z.numel() != N * K:
            raise ValueError("Z must hold N * K floats")
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        _check(lib.gee_embed_atomic_ws(_ptr(src), _ptr(dst), _ptr(w), E, N, _ptr(labels), K, flags, _ptr(Z),
                                       _ptr(workspace), workspace.numel(), _stream(stream)), "gee_embed_atomic")
    return Z


# ----------------------------------------------------------------------------- batches

def _graph_struct(g: dict, dev, sizing: bool = False) -> _lib.GeeGraph:
    """One gee_graph from a dict with src, dst, w (or None), labels, K, flags, Z and an
    optional sched; N is labels.numel(). For workspace sizing Z may be None."""
    labels = _dev(g["labels"], torch.int32, "labels", dev)
    src = _dev(g["src"], torch.int32, "src", dev)
    dst = _dev(g["dst"], torch.int32, "dst", dev)
    w = _dev(g.get("w"), torch.float32, "w", dev)
    Z = g.get("Z")
    E, N, K = src.numel(), labels.numel(), int(g["K"])
    if dst.numel() != E or (w is not None and w.numel() != E):
        raise ValueError("src, dst and w must have the same length")
    if Z is None and not sizing:
        raise ValueError("Z is required")
    if Z is not None:
        _dev(Z, torch.float32, "Z", dev)
        if Z.numel() != N * K:
            raise ValueError("Z must hold N * K floats")
    sc = g.get("sched")
    if sc is None:
        sc = schedule()
    elif isinstance(sc, dict):
        sc = schedule(**sc)
    return _lib.GeeGraph(src.data_ptr(), dst.data_ptr(), None if w is None else w.data_ptr(), E, N,
                         labels.data_ptr(), K, int(g["flags"]), None if Z is None else Z.data_ptr(), sc)


def _graph_array(graphs, dev, sizing: bool = False):
    arr = (_lib.GeeGraph * len(graphs))()
    for i, g in enumerate(graphs):
        arr[i] = _graph_struct(g, dev, sizing)
    return arr


def batch_workspace_bytes_of_sizes(sizes) -> int:
    """Workspace of gee_embed_batch for graphs given by sizes alone: tuples (E, N, K, flags,
    weighted[, sched]). Host-only (no device, no tensors): the library's size query reads only
    sizes, flags, weights-or-not and schedules."""
    arr = (_lib.GeeGraph * len(sizes))()
    for i, t in enumerate(sizes):
        E, N, K, fl, weighted = t[:5]
        sc = t[5] if len(t) > 5 else None
        if sc is None:
            sc = schedule()
        elif isinstance(sc, dict):
            sc = schedule(**sc)
        # a non-NULL weight pointer marks a weighted graph; the size query never reads it
        arr[i] = _lib.GeeGraph(None, None, 16 if weighted else None, int(E), int(N), None, int(K), int(fl),
                               None, sc)
    n = int(_lib.load().gee_embed_batch_workspace_bytes(arr, len(sizes)))
    if n == 0:
        raise GeeError(GEE_ERR_ARG, "gee_embed_batch_workspace_bytes")
    return n


def gee_embed_batch_workspace_bytes(graphs) -> int:
    """Workspace of gee_embed_batch for these graphs (their Z may be None here)."""
    dev = graphs[0]["labels"].device
    arr = _graph_array(graphs, dev, sizing=True)
    n = int(_lib.load().gee_embed_batch_workspace_bytes(arr, len(graphs)))
    if n == 0:
        raise GeeError(GEE_ERR_ARG, "gee_embed_batch_workspace_bytes")
    return n


def gee_embed_batch(graphs, workspace: Optional[torch.Tensor] = None, stream=None):
    """gee_embed of every graph (dicts: src, dst, w, labels, K, flags, Z[, sched]) in one
    launch sequence; each Z is written in place."""
    if not graphs:
        return
    dev = graphs[0]["labels"].device
    arr = _graph_array(graphs, dev)
    lib = _lib.load()
    nbytes = lib.gee_embed_batch_workspace_bytes(arr, len(graphs))
    if nbytes == 0:
        raise GeeError(GEE_ERR_ARG, "gee_embed_batch_workspace_bytes")
    with _on(stream):
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _check(lib.gee_embed_batch_ws(arr, len(graphs), _ptr(workspace), workspace.numel(), _stream(stream)),
               "gee_embed_batch_ws")


class BatchPlan:
    """gee_batch_plan: the graphs' launch sequence captured once in a hipGraph; launch()
    replays it, update() gives the plan another set of graphs (no allocation; the plan's
    workspace must hold them: workspace_bytes reserves room for larger sets). The graphs'
    tensors are kept referenced while the plan holds them."""

    def __init__(self, graphs, workspace_bytes: int = 0):
        if not graphs:
            raise ValueError("a batch plan needs at least one graph")
        self._graphs = list(graphs)
        dev = self._graphs[0]["labels"].device
        arr = _graph_array(self._graphs, dev)
        h = ctypes.c_void_p()
        _check(_lib.load().gee_batch_plan_create_ws(arr, len(self._graphs), int(workspace_bytes), ctypes.byref(h)),
               "gee_batch_plan_create")
        self._h = h

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.load().gee_batch_plan_workspace_bytes(self._h)) if self._h else 0

    def update(self, graphs):
        """Replace the plan's graphs (the caller has synchronized the plan's last launch)."""
        if not self._h:
            raise RuntimeError("batch plan destroyed")
        graphs = list(graphs)
        if not graphs:
            raise ValueError("a batch plan needs at least one graph")
        arr = _graph_array(graphs, graphs[0]["labels"].device)
        _check(_lib.load().gee_batch_plan_update(self._h, arr, len(graphs)), "gee_batch_plan_update")
        self._graphs = graphs

    def launch(self, stream=None):
        if not self._h:
            raise RuntimeError("batch plan destroyed")
        _check(_lib.load().gee_batch_plan_launch(self._h, _stream(stream)), "gee_batch_plan_launch")

    def destroy(self):
        if self._h:
            _check(_lib.load().gee_batch_plan_destroy(self._h), "gee_batch_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
