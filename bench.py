#!/usr/bin/env python
"""Benchmark of the sparse GEE hot path on one MI355X.

A step is one whole pass of the path over the workload: gee_embed on the edge list
(class counts, CSR build, degrees, Laplacian rescale, per-row class scatter, diagonal
term, correlation), inputs resident in HBM. Default workload: Chung-Lu power-law graph,
N=600,000, E=10,000,000 undirected weighted edges, K=50 (10% unknown labels), all
options on.

Prints one JSON line. `value` is edges embedded per second over the timed steps.
`batched` adds the 512-graph batched form (one captured batch plan against 512 plain
calls) and `serving` the served form (Poisson requests, budget admission and continuous
batching against the plain per-request loop, p50/p99 latency).
`original` adds the original, edge-list form of GEE (gee_embed_atomic: one pass of float
atomics over the edge list, no CSR) on the same workload and, as in the paper's GEE
against sparse GEE comparison, both forms on the 2,000- and 10,000-node SBM graphs with the
options off and all on.
`sparse` adds Z in sparse storage (gee_embed_sparse) on the same workload.
`roofline` is for the kernel with the largest share of the step, timed live with HIP
events recorded around each of its launches on the launch stream (library hook), and
priced with its algorithmic bytes against the 8 TB/s HBM peak. `cpu_baseline` is the
FP64 oracle timed on this host.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges embedded/sec + % HBM peak; served p50/p99 latency vs plain per-graph loop"
HBM_PEAK_GBS = 8000.0

KERNELS = ["class_count_partial", "class_count_final", "a_hist", "digit_scan", "a_scatter",
           "b_hist", "b_scan", "b_scatter", "c_tiles", "c_hist", "c_scan", "c_scatter", "bucket_sort", "graph_meta", "zero_steps", "node_rows", "degree_rows",
           "degree_fixup", "node_coef", "fill_empty", "embed_rows", "embed_fixup", "bucket_part_count", "bucket_part_fill", "bucket_degree",
           "bucket_degree_fix", "bucket_embed", "bucket_embed_fix", "csr_prep"]


def algorithmic_bytes(name, E, N, K, M, weighted, n_empty):
    """Bytes a kernel must move at minimum for one launch (inputs read once, outputs
    written once), from the sizes of its own inputs and outputs."""
    wv = 4 if weighted else 0
    if name == "class_count_partial":
        return 4 * N
    if name == "a_hist":  # edge list; on the edge-list paths also the labels (class counts)
        return 8 * E + 4 * N
    if name == "a_scatter":  # edge list in, (low row bits u16, col[, w]) per entry out
        return (8 + wv) * E + (2 + 4 + wv) * M
    if name == "b_hist":
        return 2 * M
    if name == "b_scatter":  # (low row bits u16, col[, w]) in; on the bucket path (column word
        # with the row in bucket packed in[, w]) out
        return (2 + 4 + wv) * M + (4 + wv) * M
    if name == "bucket_sort":  # all buckets counted as if sorted here (an upper bound when
        # the largest buckets go to the pass-C tiles): key, col, val in; CSR out
        return (2 + 4 + wv) * M + (4 + wv) * M + 4 * (N + 1)
    if name == "node_rows":
        return 4 * (N + 1) + 4 * N + 8 * N + 4 * N
    if name == "degree_rows":
        return 4 * (N + 1) + 4 * M + 4 * N + 8 * N + 4 * N
    if name == "fill_empty":
        return 4 * (N + 1) + 4 * K * n_empty
    if name == "embed_rows":
        return 4 * (N + 1) + (4 + wv) * M + 8 * N + 4 * N + 4 * N * K
    if name == "bucket_degree":  # bucketed (packed column word[, w]) in; labels in, s_i and the 5-byte
        # {c_i, y_i} records out
        return (4 + wv) * M + 4 * N + 4 * N + 5 * N
    if name == "bucket_embed":  # bucketed (column word with the row in bucket packed above it[, w]) in,
        # the 5-byte {c_j, y_j} records and s_i once, Z out (after a pass B, as on every workload
        # measured here)
        return (4 + wv) * M + 5 * N + 4 * N + 4 * N * K
    if name == "edge_scatter":  # edge list in, {c_j, y_j} once, Z written once
        return (8 + wv) * E + 8 * N + 4 * N * K
    if name == "edge_prep":  # labels; under the Laplacian the edge list and the degrees
        return 4 * N + (8 + wv) * E + 4 * N
    if name == "edge_init":
        return 4 * N * K + 4 * N
    if name == "edge_coef":
        return 4 * N + 4 * N + 4 * N + 8 * N
    if name == "edge_finish":
        return 2 * 4 * N * K + 4 * N + 8 * N
    return 0


# Bytes each step of the path must move at minimum, from its definition (inputs read once,
# outputs written once), independent of this library's layouts: the edge list, the CSR of
# Section 3 (row_ptr, col, val), labels, the per-node coefficients and Z.
STEPS = ("a1", "a2", "a3", "a4_a6", "embed", "e2e")


def step_bytes(step, E, N, K, M, weighted):
    """a1 class counts; a2 edge list -> CSR; a3 degrees from the CSR; a4_a6 rescale, class
    scatter and correlation from the CSR (row_ptr, col, val, labels, gathered c, Z); embed =
    a3 + a4_a6; e2e = the whole call's minimum (edge list and labels in, Z out)."""
    wv = 4 if weighted else 0
    if step == "a1":
        return 4 * N + 8 * K
    if step == "a2":
        return (8 + wv) * E + 4 * (N + 1) + (4 + wv) * M
    if step == "a3":
        return 4 * (N + 1) + wv * M + 4 * N
    if step == "a4_a6":
        return 4 * (N + 1) + (4 + wv) * M + 4 * N + 4 * N + 4 * N * K
    if step == "embed":
        return step_bytes("a3", E, N, K, M, weighted) + step_bytes("a4_a6", E, N, K, M, weighted)
    if step == "e2e":
        return (8 + wv) * E + 4 * N + 4 * N * K
    raise ValueError(step)


# Which step each kernel of the edge-list paths belongs to.
KERNEL_STEP = {
    "class_count_partial": "a1", "class_count_final": "a1",
    "a_hist": "a2", "digit_scan": "a2", "a_scatter": "a2", "b_hist": "a2", "b_scan": "a2", "b_scatter": "a2",
    "c_tiles": "a2", "c_hist": "a2", "c_scan": "a2", "c_scatter": "a2", "bucket_sort": "a2",
    "bucket_part_count": "a2", "bucket_part_fill": "a2", "graph_meta": "a2", "zero_steps": "a2", "csr_prep": "a2",
    "node_rows": "a3", "degree_rows": "a3", "degree_fixup": "a3", "node_coef": "a3",
    "bucket_degree": "a3", "bucket_degree_fix": "a3",
    "fill_empty": "a4_a6", "embed_rows": "a4_a6", "embed_fixup": "a4_a6",
    "bucket_embed": "a4_a6", "bucket_embed_fix": "a4_a6",
}


def call_times(torch, fn, reps=30, warmup=5, cold=None):
    """hipEvent time of fn() on the current stream: median, p10 and p90 over `reps` calls
    after `warmup`. With cold (a device tensor of at least 512 MiB), the tensor is
    overwritten before every call, outside the timed events, which evicts the inputs from
    the 256 MB last-level cache (MALL)."""
    import numpy as np

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for i in range(reps):
        if cold is not None:
            cold.fill_(float(i))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return {"median_ms": round(float(np.median(ts)), 5), "p10_ms": round(float(np.percentile(ts, 10)), 5),
            "p90_ms": round(float(np.percentile(ts, 90)), 5), "reps": reps}


def graph_times(torch, fn, reps=30, cold=None, out=None):
    """The same call captured once in a hipGraph (torch.cuda.CUDAGraph) and replayed: what a
    launch-bound caller pays per call once the host's launch work is gone. fn must launch on
    the current stream. With `out` (a float tensor fn writes), one replay first checks that
    the graph does write it. An error entry when the call cannot be captured."""
    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()  # warm the call on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            fn()
        torch.cuda.synchronize()
        if out is not None:
            out.fill_(float("nan"))
            gr.replay()
            torch.cuda.synchronize()
            if bool(torch.isnan(out).any()):
                return {"error": "the captured graph did not write the output"}
        res = call_times(torch, gr.replay, reps=reps, warmup=3, cold=cold)
        del gr
        return res
    except Exception as e:  # noqa: BLE001 - a missing variant must not cost the benchmark line
        torch.cuda.synchronize()
        return {"error": repr(e)[:200]}


def sparse_leg(torch, np, gee, lib, dev, g, tens, Z_dense, steps, ev):
    """Z in sparse storage (gee_embed_sparse) on the benchmark workload: time per call against
    the dense call, stored entries and bytes, and the compaction kernels' own times."""
    src, dst, w, lab = tens
    flags = gee.flags_of(g.diag, g.lap, g.cor, g.sym)
    E, N, K = g.E, g.N, g.K
    rp = torch.empty(N + 1, dtype=torch.int32, device=dev)
    col = torch.empty(N * K, dtype=torch.int32, device=dev)
    val = torch.empty(N * K, dtype=torch.float32, device=dev)
    ws = torch.empty(gee.gee_embed_sparse_workspace_bytes(E, N, K, flags, w is not None), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream()

    def call():
        gee.gee_embed_sparse(src, dst, w, lab, K, flags, row_ptr=rp, col=col, val=val, workspace=ws, stream=stream)

    ms = _time_calls(torch, call, steps)
    nnz = int(rp[-1].item())
    kernels = {}
    for name in ("zs_count", "zs_tile_sum", "zs_write"):
        a, b = ev.create(), ev.create()
        lib.gee_profile_kernel(name.encode(), a, b)
        call()
        torch.cuda.synchronize()
        lib.gee_profile_kernel(name.encode(), None, None)
        try:
            kms = ev.elapsed_ms(a, b)
        except RuntimeError:  # not launched: the class-scatter kernels counted the rows (or did not)
            ev.hip.hipGetLastError()
            ev.destroy(a)
            ev.destroy(b)
            continue
        # zs_count reads Z; zs_tile_sum the row counts the class-scatter kernels wrote; zs_write
        # (on the bucket path, as on this workload) the row counts and the non-zero pairs the
        # class-scatter kernels staged in, row_ptr and the pairs' classes and values out
        nb = {"zs_count": 4 * N * K, "zs_tile_sum": 4 * N,
              "zs_write": 4 * N + 8 * nnz + 4 * (N + 1) + 8 * nnz}[name]
        kernels[name] = {"ms": round(kms, 5), "algorithmic_bytes": int(nb), "GB_per_s": round(nb / (kms * 1e-3) / 1e9, 1)}
        ev.destroy(a)
        ev.destroy(b)
    same = bool(torch.equal(Z_dense.reshape(-1)[(torch.repeat_interleave(
        torch.arange(N, device=dev), (rp[1:] - rp[:-1]).long()) * K + col[:nnz].long())], val[:nnz]))
    out = {"ms_per_call": round(ms, 5), "edges_per_s": round(E / (ms * 1e-3), 1), "nnz": nnz,
           "density": round(nnz / (N * K), 4), "sparse_bytes": 4 * (N + 1) + 8 * nnz, "dense_bytes": 4 * N * K,
           "values_equal_dense_call": same, "kernels": kernels}
    del rp, col, val, ws
    return out


EDGE_KERNELS = ["edge_init", "edge_prep", "edge_coef", "edge_scatter", "edge_finish"]


def _time_calls(torch, fn, reps, warmup=3):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def original_leg(torch, np, gee, lib, dev, g, tens, Z_sparse, steps, ev):
    """The original GEE form against the sparse path: the benchmark workload, then the
    2,000-node SBM graph (launch-bound sizes) and the 10,000-node SBM graph, each with the
    options off and all on."""
    src, dst, w, lab = tens
    flags = gee.flags_of(g.diag, g.lap, g.cor, g.sym)
    E, N, K = g.E, g.N, g.K
    Z = torch.empty((N, K), dtype=torch.float32, device=dev)
    ws = torch.empty(max(1, gee.gee_embed_atomic_workspace_bytes(N, K, flags)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def call():
        gee.gee_embed_atomic(src, dst, w, lab, K, flags, Z=Z, workspace=ws, stream=stream)

    ms = _time_calls(torch, call, steps)
    if gee.gee_get_data_errors() != 0:
        raise RuntimeError("device reported a data error in the original form")
    kernels = {}
    for name in EDGE_KERNELS:
        a, b = ev.create(), ev.create()
        lib.gee_profile_kernel(name.encode(), a, b)
        call()
        torch.cuda.synchronize()
        lib.gee_profile_kernel(name.encode(), None, None)
        try:
            kms = ev.elapsed_ms(a, b)
            nb = algorithmic_bytes(name, E, N, K, 0, w is not None, 0)
            kernels[name] = {"ms": round(kms, 5), "algorithmic_bytes": int(nb),
                             "GB_per_s": round(nb / (kms * 1e-3) / 1e9, 1) if kms > 0 else None}
        except RuntimeError:  # not launched for this workload
            pass
        ev.destroy(a)
        ev.destroy(b)
    nz = Z_sparse != 0
    rel = float(((Z - Z_sparse).abs()[nz] / Z_sparse.abs()[nz]).max().item()) if bool(nz.any()) else 0.0
    out = {"ms_per_call": round(ms, 5), "edges_per_s": round(E / (ms * 1e-3), 1),
           "max_rel_diff_to_sparse_path": rel, "same_zero_entries_as_sparse_path": bool(torch.equal(Z != 0, nz)),
           "kernels": kernels}
    del Z, ws
    def compare(gs, opt, reps):
        t = lambda a, dt: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa
        s2, d2, w2, l2 = t(gs.src, torch.int32), t(gs.dst, torch.int32), t(gs.w, torch.float32), t(gs.labels, torch.int32)
        f2 = gee.flags_of(gs.diag, gs.lap, gs.cor, gs.sym)
        Zs = torch.empty((gs.N, gs.K), dtype=torch.float32, device=dev)
        Za = torch.empty_like(Zs)
        wss = torch.empty(max(1, gee.gee_embed_workspace_bytes(gs.E, gs.N, gs.K, f2, w2 is not None)),
                          dtype=torch.uint8, device=dev)
        wsa = torch.empty(max(1, gee.gee_embed_atomic_workspace_bytes(gs.N, gs.K, f2)), dtype=torch.uint8,
                          device=dev)
        sp_ms = _time_calls(torch, lambda: gee.gee_embed(s2, d2, w2, l2, gs.K, f2, Z=Zs, workspace=wss,
                                                          stream=stream), reps)
        at_ms = _time_calls(torch, lambda: gee.gee_embed_atomic(s2, d2, w2, l2, gs.K, f2, Z=Za, workspace=wsa,
                                                                 stream=stream), reps)
        nz2 = Zs != 0
        return {"workload": gs.name, "E": gs.E, "options": opt, "sparse_ms_per_call": round(sp_ms, 5),
                "original_ms_per_call": round(at_ms, 5),
                "max_rel_diff": float(((Za - Zs).abs()[nz2] / Zs.abs()[nz2]).max().item())}

    out["sbm_n2000"] = [compare(make_workload(f"sbm_small_{opt}"), opt, 200) for opt in ("off", "all")]
    gd = make_workload("sbm_dense")  # all options; the paper's 10,000-node SBM graph
    out["sbm_n10000"] = [compare(gd.with_options(False, False, False, name=gd.name + "_off"), "off", 20),
                         compare(gd, "all", 20)]
    return out


def copy_ceiling(torch, dev, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of `nbytes`, the
    practical HBM ceiling on this GPU beside the spec peak; None if it cannot be measured."""
    try:
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            b.copy_(a)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        del a, b
        torch.cuda.empty_cache()
        return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    except Exception:  # noqa: BLE001 - a missing ceiling must not cost the benchmark line
        return None


def _progress(msg):
    """One line on stderr when a phase of the run has finished (the JSON line stays alone
    on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    from gee_workloads import powerlaw_10m, sbm_dense, sbm_small

    if name == "powerlaw_10m":
        return powerlaw_10m()
    if name == "sbm_dense":
        return sbm_dense()
    if name == "sbm_small_all":
        return sbm_small("all")
    if name == "sbm_small_off":
        return sbm_small("off")
    raise ValueError(name)


class HipEvents:
    """hipEvent create/elapsed through the HIP runtime torch already loaded."""

    def __init__(self):
        import ctypes

        import torch

        path = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
        self.ct = ctypes
        self.hip = ctypes.CDLL(path)
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        h = self.ct.c_void_p()
        rc = self.hip.hipEventCreate(self.ct.byref(h))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed ({rc})")
        return h

    def elapsed_ms(self, a, b):
        out = self.ct.c_float()
        rc = self.hip.hipEventElapsedTime(self.ct.byref(out), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(out.value)

    def destroy(self, h):
        self.hip.hipEventDestroy(h)


def cpu_baseline(g, budget_s=12.0, max_reps=30):
    """The FP64 oracle (single-threaded C edge-list loop) on one host core: the process is
    pinned to the first core it may run on while the oracle (and then the scipy route) is
    timed, and unpinned afterwards."""
    from oracle import oracle as orc

    orc.load()
    allowed = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    core = min(allowed) if allowed else None
    if core is not None:
        os.sched_setaffinity(0, {core})
    try:
        reps, total = 0, 0.0
        while reps < max_reps and (total < budget_s or reps < 1):
            t0 = time.perf_counter()
            orc.embed_graph(g)
            total += time.perf_counter() - t0
            reps += 1
        out = {"value": g.E * reps / total, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload edge list, {reps} repetition(s), {total:.1f} s of CPU time",
               "pinned_core": core, "host_cpu": _cpu_model(), "host_threads": os.cpu_count(),
               "host_threads_allowed": len(allowed) if allowed else None}
        out["scipy_route"] = scipy_baseline(g)
    finally:
        if allowed:
            os.sched_setaffinity(0, allowed)
    return out


def scipy_baseline(g, budget_s=10.0, max_reps=10):
    """The paper's design on this host: scipy.sparse CSR products in FP64 (one thread for
    the sparse products; numpy may use more for the dense steps). None if it fails."""
    try:
        from oracle.scipy_route import scipy_route

        reps, total = 0, 0.0
        while reps < max_reps and (total < budget_s or reps < 1):
            t0 = time.perf_counter()
            scipy_route(g.src, g.dst, g.w, g.N, g.labels, g.K, g.diag, g.lap, g.cor, g.sym)
            total += time.perf_counter() - t0
            reps += 1
        return {"value": g.E * reps / total, "unit": "edges/s", "kind": "scipy.sparse route (the paper's design)",
                "sample": f"the full workload edge list, {reps} repetition(s), {total:.1f} s"}
    except Exception as e:  # noqa: BLE001 - a missing context figure must not cost the benchmark line
        return {"error": repr(e)[:200]}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ----------------------------------------------------------------------------- systems legs

def _gen_batched(g):
    from gee_workloads.configs import batched_one

    x = batched_one(g)
    return x.src, x.dst, x.w, x.labels, x.K, (x.diag, x.lap, x.cor, x.sym)


def _gen_serving(g, e_max):
    from gee_workloads.configs import serving_one

    x = serving_one(g, e_max=e_max)
    return x.src, x.dst, x.w, x.labels, x.K, (x.diag, x.lap, x.cor, x.sym)


def gen_parallel(fn, args_list, procs):
    """Seeded graphs drawn in worker processes (CPU only; they never touch the GPU)."""
    import multiprocessing as mp

    with mp.get_context("spawn").Pool(procs) as pool:
        return pool.starmap(fn, args_list, chunksize=1)


def _to_items(raw, torch, np, gee, dev, table):
    items = []
    for src, dst, w, lab, K, opts in raw:
        t = lambda a, dt: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa
        it = dict(src=t(src, torch.int32), dst=t(dst, torch.int32), w=t(w, torch.float32),
                  labels=t(lab, torch.int32), K=int(K), flags=gee.flags_of(*opts))
        sc = table.lookup(it["src"].numel(), it["labels"].numel(), it["K"], it["flags"]) if table else {}
        it["sched"] = sc or None
        items.append(it)
    return items


def batched_leg(torch, np, gee, dev, table, procs, reps=5, G=512):
    """512 graphs of the batched recipe: one captured batch plan (hipGraph replay) against
    512 back-to-back plain gee_embed_ws calls on one stream, same per-graph schedules."""
    t0 = time.perf_counter()
    raw = gen_parallel(_gen_batched, [(i,) for i in range(G)], procs)
    gen_s = time.perf_counter() - t0
    items = _to_items(raw, torch, np, gee, dev, table)
    del raw
    for it in items:
        it["Z"] = torch.empty((it["labels"].numel(), it["K"]), dtype=torch.float32, device=dev)
    E_tot = sum(it["src"].numel() for it in items)
    ws_max = max(gee.gee_embed_workspace_bytes(it["src"].numel(), it["labels"].numel(), it["K"], it["flags"],
                                               it["w"] is not None, it["sched"]) for it in items)
    ws = torch.empty(ws_max, dtype=torch.uint8, device=dev)
    Zp = [torch.empty_like(it["Z"]) for it in items]

    def plain_loop():
        for it, z in zip(items, Zp):
            gee.gee_embed(it["src"], it["dst"], it["w"], it["labels"], it["K"], it["flags"], Z=z,
                          sched=it["sched"], workspace=ws)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    plain_ms = timed(plain_loop)
    # the same 512 plain calls captured in one hipGraph: the plain loop without its host
    # launch work, which separates the gain of batching from the host's per-call cost
    plain_graph = graph_times(torch, plain_loop, reps=reps, out=Zp[-1])
    plan = gee.BatchPlan(items)
    batch_ms = timed(lambda: plan.launch())
    torch.cuda.synchronize()
    same = all(torch.equal(it["Z"], z) for it, z in zip(items, Zp))
    plan.destroy()
    # the same batch with the library's default schedules (what the tuned table gains)
    dflt = [dict(it, sched=None, Z=torch.empty_like(it["Z"])) for it in items]
    plan_d = gee.BatchPlan(dflt)
    default_ms = timed(lambda: plan_d.launch())
    plan_d.destroy()
    del dflt
    e2e = sum(step_bytes("e2e", it["src"].numel(), it["labels"].numel(), it["K"], 0, it["w"] is not None)
              for it in items)
    return {"graphs": G, "edges": int(E_tot), "generation_s": round(gen_s, 1),
            "plain_loop_ms": round(plain_ms, 3), "batch_plan_ms": round(batch_ms, 3),
            "plain_loop_graph_captured": plain_graph,
            "plain_edges_per_s": round(E_tot / (plain_ms * 1e-3), 1),
            "batch_edges_per_s": round(E_tot / (batch_ms * 1e-3), 1),
            "batch_plan_default_schedules_ms": round(default_ms, 3),
            "tuned_gain_vs_default": round(default_ms / batch_ms, 3),
            "speedup": round(plain_ms / batch_ms, 3),
            "speedup_vs_captured_plain": round(plain_graph["median_ms"] / batch_ms, 3)
            if "median_ms" in plain_graph else None,
            "e2e_min_bytes": int(e2e), "batch_e2e_hbm_frac": round(e2e / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bitwise_equal_to_plain": same,
            "schedules": "autotuned table" if table and table.entries else "library defaults"}


def serving_leg(torch, np, gee, dev, table, procs, pool_n=64, e_max=20_000_000, n_req=10_000,
                loads=(0.3, 0.5, 0.7, 0.9, 1.1, 1.5), slots=4, budget_gb=32.0, max_batch=16,
                max_batch_edges=2_000_000, max_inflight_edges=None, big_edges=8_000_000, n_check=1_000):
    """Poisson requests from a pool of serving-recipe graphs: the server (budget admission,
    continuous batching over `slots` streams) against the plain per-request loop, n_req
    requests per load; requests of at least big_edges edges run one at a time, smaller ones
    passing a large one that waits. Success criterion: with L* the plain loop's p99 at 0.5 x its
    saturation rate, the server keeps p99 <= L* up to a higher load than the plain loop.
    Every result of a separate untimed burst of n_check requests (all arriving at once, so
    batches are as full and overlapped as they get) is compared bitwise with the plain
    result of its graph."""
    from paper_2406_03726_amd.serve import GeeServer, GpuBackend, Request, run_plain, summarize

    t0 = time.perf_counter()
    raw = gen_parallel(_gen_serving, [(i, e_max) for i in range(pool_n)], procs)
    gen_s = time.perf_counter() - t0
    pool = _to_items(raw, torch, np, gee, dev, table)
    del raw
    ws_max = max(gee.gee_embed_workspace_bytes(it["src"].numel(), it["labels"].numel(), it["K"], it["flags"],
                                               it["w"] is not None, it["sched"]) for it in pool)
    ws = torch.empty(ws_max, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def embed_one(r):
        g = r.graph
        r.result = gee.gee_embed(g["src"], g["dst"], g["w"], g["labels"], g["K"], g["flags"],
                                 sched=g["sched"], workspace=ws, stream=stream)
        stream.synchronize()

    def service_ms(it, reps=3):
        """Median of `reps` plain calls after one warm call; the last result is kept."""
        r = Request(0, it, 0.0)
        embed_one(r)
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            embed_one(r)
            ts.append(time.perf_counter() - t1)
        return float(np.median(ts)), r.result

    # plain service time per pool graph -> saturation rate of the plain loop (its result is
    # the graph's reference result), and beside it the same graph with the library's default
    # schedules, measured the same way right after it
    svc, svc_d, refs = [], [], []
    for it in pool:
        t, z = service_ms(it)
        svc.append(t)
        refs.append(z)
        svc_d.append(service_ms(dict(it, sched=None))[0])
    mu = 1.0 / float(np.mean(svc))
    rng = np.random.default_rng(20240603)
    out = {"pool_graphs": pool_n, "pool_edges_mean": int(np.mean([it["src"].numel() for it in pool])),
           "generation_s": round(gen_s, 1), "requests_per_load": n_req, "slots": slots,
           "budget_bytes": int(budget_gb * 2 ** 30), "max_batch": max_batch, "max_batch_edges": max_batch_edges,
           "max_inflight_edges": max_inflight_edges, "big_edges": big_edges, "max_big_inflight": 1,
           "plain_saturation_req_per_s": round(mu, 1),
           "pool_plain_ms_tuned": round(float(np.sum(svc)) * 1e3, 3),
           "pool_plain_ms_default_schedules": round(float(np.sum(svc_d)) * 1e3, 3),
           "schedules": "autotuned table" if table and table.entries else "library defaults", "loads": []}

    # one backend for every run (its streams, per-slot workspaces and the graphs' cached sizing
    # outlive each server); the pool is staged and complete, so batches need not wait for the
    # submitting stream
    torch.cuda.synchronize()
    backend = GpuBackend(slots=slots, table=table, sync_inputs=False)

    def server(on_done=None):
        return GeeServer(backend, int(budget_gb * 2 ** 30), max_batch=max_batch,
                         max_batch_edges=max_batch_edges, max_inflight_edges=max_inflight_edges,
                         on_done=on_done or drop, big_edges=big_edges, max_big_inflight=1)

    def drop(r):
        r.result = None  # results are not kept through the timed runs

    # warm-up of the served path (the plain loop's was the service-time pass): every pool
    # graph once through the server, so its streams' allocator caches hold their sizes
    server().run_trace([Request(i, it, 0.0, E=int(it["src"].numel())) for i, it in enumerate(pool)], busy_poll=True)
    torch.cuda.synchronize()

    # equality pass: every served result against its graph's plain result
    picks = rng.integers(0, pool_n, size=n_check)
    bad = []
    multi = []

    def check(r):
        if r.error is None and not torch.equal(r.result, refs[r.graph["_pool"]]):
            bad.append(r.rid)
        r.result = None

    for i, it in enumerate(pool):
        it["_pool"] = i
    chk = server(on_done=check)
    chk.run_trace([Request(i, pool[int(p)], 0.0, E=int(pool[int(p)]["src"].numel())) for i, p in enumerate(picks)],
                  busy_poll=True)
    torch.cuda.synchronize()
    multi = [len(b) for b in chk.launch_log]
    out["equality_check"] = {"requests": n_check, "mismatches": len(bad), "batches": len(multi),
                             "largest_batch": max(multi) if multi else 0,
                             "batches_of_several": sum(1 for m in multi if m > 1),
                             "peak_batches_in_flight": chk.peak_flights}
    _progress(f"serving equality pass: {len(bad)} mismatches over {n_check} requests")

    picks = rng.integers(0, pool_n, size=n_req)
    for frac in loads:
        lam = frac * mu
        arr = np.cumsum(rng.exponential(1.0 / lam, size=n_req))

        def mk():
            return [Request(i, pool[int(p)], float(a), E=int(pool[int(p)]["src"].numel()))
                    for i, (p, a) in enumerate(zip(picks, arr))]

        plain = run_plain(mk(), embed_one, on_done=drop, busy_poll=True)
        srv = server()
        served = srv.run_trace(mk(), busy_poll=True)
        torch.cuda.synchronize()
        sp, ss = summarize(plain), summarize(served)
        out["loads"].append({"load_vs_plain_saturation": frac, "rate_req_per_s": round(lam, 1),
                             "plain": {k: round(v, 3) for k, v in sp.items()},
                             "served": {k: round(v, 3) for k, v in ss.items()},
                             "served_peak_bytes": srv.peak_in_use, "served_peak_batches": srv.peak_flights,
                             "served_batches": len(srv.launch_log)})
        _progress(f"serving load {frac}: plain p99 {sp['p99_ms']:.2f} ms, served p99 {ss['p99_ms']:.2f} ms")
        del plain, served
    # L*: the plain loop's p99 at half its saturation rate
    lstar = next((x["plain"]["p99_ms"] for x in out["loads"] if x["load_vs_plain_saturation"] == 0.5), None)
    if lstar is not None:
        def max_load(side):
            ok = [x["load_vs_plain_saturation"] for x in out["loads"] if x[side]["p99_ms"] <= lstar]
            return max(ok) if ok else None

        pm, sm = max_load("plain"), max_load("served")
        out["Lstar_ms"] = lstar
        out["plain_max_load_within_Lstar"] = pm
        out["served_max_load_within_Lstar"] = sm
        out["served_p99_at_or_below_plain_every_load"] = all(x["served"]["p99_ms"] <= x["plain"]["p99_ms"]
                                                             for x in out["loads"])
        out["success"] = bool(sm is not None and (pm is None or sm > pm))
    del refs, ws
    return out


# ----------------------------------------------------------------------------- HBM traffic

PROFILES = os.path.join(ROOT, "profiles")
CALIB_BYTES = 1 << 30  # device-to-device copy that calibrates the byte counters


def _code_only(text: str) -> str:
    """C/C++ source without its comments and with whitespace runs collapsed (string and
    character literals kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash() -> str:
    """Hash of the HIP sources' code (comments and layout left out): traffic figures taken
    from a build of other code do not count."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2406_03726_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                h.update(name.encode() + b"\0" + _code_only(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_path(workload: str) -> str:
    return os.path.join(PROFILES, f"hbm_traffic_gee_embed_{workload}.md")


# Counters of the two rocprofv3 --pmc passes (at most 4 TCC counters a pass). Bytes come
# from request counts by size, so no calibration factor is needed: reads are the 32-, 64-
# and 128-byte read requests the L2 sends to the fabric, writes the 32- and 64-byte write
# requests; the DRAM-bound counts (in 32-byte units) are reported beside them.
PMC_PASSES = (("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum"),
              ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_RDREQ_DRAM_32B_sum",
               "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"))


def kernel_key(name: str) -> str:
    """Hook name of a kernel from the name rocprofv3 prints (the partition passes' shared
    segment kernels are pass B on the bucket path, pass C when they write the CSR)."""
    base = name.split("(")[0].replace("void ", "").strip()
    tmpl = base[base.index("<"):] if "<" in base else ""
    base = base.split("<")[0].split("::")[-1]
    if "copyBuffer" in base:
        return "copy"
    if base == "seg_hist":
        return "b_hist"
    if base == "seg_scan":
        return "b_scan"
    if base == "seg_scatter":
        return "c_scatter" if "true" in tmpl else "b_scatter"
    return base


def _counter_means(csv_path: str):
    """{kernel: {counter: mean value per dispatch}, ...} and {kernel: dispatches}."""
    import csv

    vals, disp = {}, {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            k = kernel_key(r["Kernel_Name"])
            vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            disp.setdefault(k, set()).add(r.get("Dispatch_Id", r.get("Correlation_Id")))
    means = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in vals.items()}
    return means, {k: len(v) for k, v in disp.items()}


def write_traffic(csv_a: str, csv_b: str, workload: str, commands: str) -> str:
    """Turns the two counter passes over `bench.py --pmc-target` (a 1 GiB copy, then two
    gee_embed calls) into the per-launch HBM bytes of every kernel of the call."""
    ma, na = _counter_means(csv_a)
    mb, _ = _counter_means(csv_b)
    kernels = {}
    for k in sorted(set(ma) & set(mb)):
        a, b = ma[k], mb[k]
        rd = 32 * a["TCC_EA0_RDREQ_32B_sum"] + 64 * a["TCC_EA0_RDREQ_64B_sum"] + 128 * a["TCC_EA0_RDREQ_128B_sum"]
        wr = 32 * (b["TCC_EA0_WRREQ_sum"] - b["TCC_EA0_WRREQ_64B_sum"]) + 64 * b["TCC_EA0_WRREQ_64B_sum"]
        kernels[k] = {"launches": na[k], "read_bytes": int(rd), "write_bytes": int(wr),
                      "bytes": int(rd + wr), "dram_read_bytes": int(32 * b["TCC_EA0_RDREQ_DRAM_32B_sum"]),
                      "dram_write_bytes": int(32 * b["TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"]),
                      "read_requests": int(a["TCC_EA0_RDREQ_sum"]),
                      "read_requests_by_size": [int(a["TCC_EA0_RDREQ_32B_sum"]), int(a["TCC_EA0_RDREQ_64B_sum"]),
                                                int(a["TCC_EA0_RDREQ_128B_sum"])]}
    copy = kernels.pop("copy", None)
    known = set(KERNELS) | set(EDGE_KERNELS) | {"zs_count", "zs_tile_sum", "zs_write"}
    kernels = {k: v for k, v in kernels.items() if k in known}  # the library's kernels only
    out = {"workload": workload, "source_hash": source_hash(), "calib_bytes": CALIB_BYTES,
           "copy_check": copy, "kernels": kernels}
    path = traffic_path(workload)
    os.makedirs(PROFILES, exist_ok=True)
    with open(path, "w") as f:
        f.write(f"# HBM traffic of every kernel of one `gee_embed` call on `{workload}`\n\n")
        f.write("Two rocprofv3 counter passes over the same command (a 1 GiB device-to-device copy, then two\n"
                "calls). Bytes per launch from the L2's fabric requests by size: reads = 32/64/128-byte read\n"
                "requests, writes = 32/64-byte write requests; the DRAM-bound counts (32-byte units) beside\n"
                "them. The copy row checks the method: it should read and write about 1 GiB each.\n"
                "Commands (from /tmp, TMPDIR=/tmp, on the MI355X box):\n\n")
        f.write("```\n" + commands.strip() + "\n```\n\n")
        f.write("| kernel | launches | read MB | write MB | DRAM read MB | DRAM write MB |\n|---|---|---|---|---|---|\n")
        rows = ([("copy (check)", copy)] if copy else []) + sorted(kernels.items(), key=lambda kv: -kv[1]["bytes"])
        for k, d in rows:
            f.write(f"| `{k}` | {d['launches']} | {d['read_bytes'] / 1e6:.1f} | {d['write_bytes'] / 1e6:.1f} | "
                    f"{d['dram_read_bytes'] / 1e6:.1f} | {d['dram_write_bytes'] / 1e6:.1f} |\n")
        f.write("\n```json\n" + json.dumps(out, indent=1) + "\n```\n")
    return path


def write_trace(trace_csv: str, workload: str, commands: str) -> str:
    """Turns a rocprofv3 --kernel-trace CSV of `bench.py --legs none` into the per-kernel
    durations of one gee_embed call on the benchmark workload: the calls are the runs from
    a_hist to bucket_embed_fix, each kernel's median over them, and the calls' median span
    (first start to last end)."""
    import csv
    import statistics

    seq = []
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            seq.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), kernel_key(r["Kernel_Name"])))
    seq.sort()
    calls, cur = [], None
    for st, en, k in seq:
        if k == "a_hist":
            cur = [(st, en, k)]
        elif cur is not None:
            cur.append((st, en, k))
            if k == "bucket_embed_fix":
                calls.append(cur)
                cur = None
    if not calls:
        raise SystemExit(f"no gee_embed call in {trace_csv}")
    names = [k for _, _, k in calls[0]]
    per = {k: statistics.median([(c[i][1] - c[i][0]) / 1e3 for c in calls if len(c) == len(names)])
           for i, k in enumerate(names)}
    span = statistics.median([(c[-1][1] - c[0][0]) / 1e3 for c in calls])
    out = {"workload": workload, "source_hash": source_hash(), "calls": len(calls), "span_us": round(span, 1),
           "kernels_us": {k: round(v, 1) for k, v in per.items()}}
    path = os.path.join(PROFILES, f"kernel_trace_gee_embed_{workload}.md")
    os.makedirs(PROFILES, exist_ok=True)
    with open(path, "w") as f:
        f.write(f"# Kernel trace of `gee_embed` on `{workload}`\n\n")
        f.write("rocprofv3 kernel trace of the benchmark without its extra legs; every call of the path\n"
                "(a_hist through bucket_embed_fix) is taken, and each kernel's median duration over them.\n"
                "Command (from /tmp, TMPDIR=/tmp, on the MI355X box):\n\n")
        f.write("```\n" + commands.strip() + "\n```\n\n")
        f.write(f"{len(calls)} calls; median span of one call (first start to last end): {span:.1f} us.\n\n")
        f.write("| kernel | median us | share |\n|---|---|---|\n")
        tot = sum(per.values())
        for k, v in per.items():
            f.write(f"| `{k}` | {v:.1f} | {v / tot * 100:.1f} % |\n")
        f.write("\n```json\n" + json.dumps(out, indent=1) + "\n```\n")
    return path


def read_traffic(workload: str):
    """Per-kernel bytes per launch from the committed counter summary, or None when absent
    or taken from other sources than the current ones."""
    path = traffic_path(workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    i = text.find("```json")
    if i < 0:
        return None
    d = json.loads(text[i + 7:text.index("```", i + 7)])
    if d.get("source_hash") != source_hash():
        return None
    return d


def pmc_target(gee, torch, np):
    """What the counter runs profile: one calibration copy, then one warmup and one step
    of the default workload."""
    dev = torch.device("cuda:0")
    a = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a).fill_(2.0)  # also evicts `a` from the caches before the copy
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    g = make_workload("powerlaw_10m")
    t = lambda x, dt: None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(dev, dt)  # noqa
    src, dst, w, lab = t(g.src, torch.int32), t(g.dst, torch.int32), t(g.w, torch.float32), t(g.labels, torch.int32)
    flags = gee.flags_of(g.diag, g.lap, g.cor, g.sym)
    for _ in range(2):
        gee.gee_embed(src, dst, w, lab, g.K, flags)
    torch.cuda.synchronize()


def config_leg(torch, np, gee, dev, name, cold, reps=30):
    """One of the plain single-graph configurations (the 2,000-node SBM graph with the options
    off and all on, the 10,000-node SBM graph): hipEvent times warm and cold, the call
    captured in a hipGraph, edges/s and the HBM fractions of the whole call."""
    g = make_workload(name)
    t = lambda a, dt: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa
    src, dst, w, lab = t(g.src, torch.int32), t(g.dst, torch.int32), t(g.w, torch.float32), t(g.labels, torch.int32)
    flags = gee.flags_of(g.diag, g.lap, g.cor, g.sym)
    E, N, K = g.E, g.N, g.K
    Z = torch.empty((N, K), dtype=torch.float32, device=dev)
    ws = torch.empty(gee.gee_embed_workspace_bytes(E, N, K, flags, w is not None), dtype=torch.uint8, device=dev)

    def fn():
        gee.gee_embed(src, dst, w, lab, K, flags, Z=Z, workspace=ws, stream=torch.cuda.current_stream())

    warm = call_times(torch, fn, reps=reps)
    coldt = call_times(torch, fn, reps=reps, cold=cold)
    graph = graph_times(torch, fn, reps=reps, out=Z)
    rp, _, _ = gee.gee_build_csr(src, dst, w, N, flags)
    torch.cuda.synchronize()
    M = int(rp[-1].item())
    e2e, emb = step_bytes("e2e", E, N, K, M, w is not None), step_bytes("embed", E, N, K, M, w is not None)
    out = {"workload": g.name, "N": N, "E": E, "K": K, "M_csr_entries": M, "weighted": w is not None,
           "options": "+".join(o for o, on in (("diag", g.diag), ("laplacian", g.lap), ("correlation", g.cor)) if on)
           or "none", "warm": warm, "cold": coldt, "graph_captured": graph,
           "edges_per_s": round(E / (warm["median_ms"] * 1e-3), 1),
           "e2e_min_bytes": int(e2e), "embed_bytes": int(emb),
           "e2e_hbm_frac_warm": round(e2e / (warm["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "e2e_hbm_frac_cold": round(e2e / (coldt["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del Z, ws, rp
    return out


def csr_build_leg(torch, np, gee, g, tens, M, cold, reps=30):
    """gee_build_csr (the CSR of Section 3, bit-exact) on the benchmark workload."""
    src, dst, w, lab = tens
    flags = gee.flags_of(g.diag, g.lap, g.cor, g.sym)
    dev = src.device
    N = g.N
    rp = torch.empty(N + 1, dtype=torch.int32, device=dev)
    col = torch.empty(M, dtype=torch.int32, device=dev)
    val = torch.empty(M, dtype=torch.float32, device=dev) if w is not None else None
    ws = torch.empty(gee.gee_build_csr_workspace_bytes(g.E, N, flags), dtype=torch.uint8, device=dev)

    def fn():
        gee.gee_build_csr(src, dst, w, N, flags, row_ptr=rp, col=col, val=val, workspace=ws)

    warm = call_times(torch, fn, reps=reps)
    coldt = call_times(torch, fn, reps=reps, cold=cold)
    b = step_bytes("a2", g.E, N, g.K, M, w is not None)
    out = {"warm": warm, "cold": coldt, "edges_per_s": round(g.E / (warm["median_ms"] * 1e-3), 1),
           "algorithmic_bytes": int(b), "hbm_frac_warm": round(b / (warm["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del rp, col, val, ws
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="powerlaw_10m",
                    choices=["powerlaw_10m", "sbm_dense", "sbm_small_all", "sbm_small_off"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--report", default=None, help="also write a detailed JSON report here")
    ap.add_argument("--legs", default="configs,csr,original,sparse,batched,serving",
                    help="legs to add to the line: configs, csr, original, sparse, batched, serving "
                         "(comma list, or none)")
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1),
                    help="worker processes that draw the systems legs' graphs")
    ap.add_argument("--pmc-target", action="store_true",
                    help="run only what the rocprofv3 counter runs measure (a calibration copy and two steps)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("PASS1_CSV", "PASS2_CSV"),
                    help="host only: turn the two counter passes into the committed traffic summary")
    ap.add_argument("--traffic-commands", default="")
    ap.add_argument("--write-trace", metavar="KERNEL_TRACE_CSV",
                    help="host only: turn a rocprofv3 kernel trace into the committed per-kernel summary")
    args = ap.parse_args()

    if args.write_trace:
        print(write_trace(args.write_trace, "chunglu_n600k_e10m_k50", args.traffic_commands))
        return

    if args.write_traffic:
        print(write_traffic(args.write_traffic[0], args.write_traffic[1], "chunglu_n600k_e10m_k50",
                            args.traffic_commands))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the library has no "
                                   "multi-GPU (sharded) form",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2406_03726_amd as gee
    from paper_2406_03726_amd import _lib

    if not os.path.exists(_lib.LIB):
        import __graft_entry__

        __graft_entry__.build()
    lib = _lib.load()
    if args.pmc_target:
        pmc_target(gee, torch, np)
        return

    t_gen = time.perf_counter()
    g = make_workload(args.workload)
    t_gen = time.perf_counter() - t_gen
    _progress(f"workload {g.name} generated in {t_gen:.1f} s")
    dev = torch.device("cuda:0")
    t = lambda a, dt: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa
    src, dst, w, lab = t(g.src, torch.int32), t(g.dst, torch.int32), t(g.w, torch.float32), t(g.labels, torch.int32)
    flags = gee.flags_of(g.diag, g.lap, g.cor, g.sym)
    E, N, K = g.E, g.N, g.K
    weighted = w is not None
    Z = torch.empty((N, K), dtype=torch.float32, device=dev)
    ws_bytes = gee.gee_embed_workspace_bytes(E, N, K, flags, weighted)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        # (on the stream current at the call, so that the captured variant records it)
        gee.gee_embed(src, dst, w, lab, K, flags, Z=Z, workspace=ws, stream=torch.cuda.current_stream())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if gee.gee_get_data_errors() != 0:
        raise RuntimeError("device reported a data error on the benchmark input")

    # CSR entry count and empty rows (for the byte counts)
    rp, col, val = gee.gee_build_csr(src, dst, w, N, flags)
    torch.cuda.synchronize()
    M = int(rp[-1].item())
    n_empty = int((rp[1:] == rp[:-1]).sum().item())

    ev = HipEvents()

    # Untimed pass: each kernel's duration, to find the dominant one.
    per_kernel = {}
    for name in KERNELS:
        a, b = ev.create(), ev.create()
        lib.gee_profile_kernel(name.encode(), a, b)
        step()
        torch.cuda.synchronize()
        lib.gee_profile_kernel(name.encode(), None, None)
        try:
            per_kernel[name] = ev.elapsed_ms(a, b)
        except RuntimeError:  # not launched for this workload
            ev.hip.hipGetLastError()  # (the failed query leaves its error for the next HIP call)
        ev.destroy(a)
        ev.destroy(b)
    dominant = max(per_kernel, key=per_kernel.get)
    _progress(f"per-kernel pass done; dominant kernel {dominant}")

    # Timed region: K steps; HIP events around every launch of the dominant kernel.
    pairs = [(ev.create(), ev.create()) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lib.gee_profile_kernel(dominant.encode(), pairs[i][0], pairs[i][1])
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.gee_profile_kernel(dominant.encode(), None, None)
    dom_ms = [ev.elapsed_ms(a, b) for a, b in pairs]
    for a, b in pairs:
        ev.destroy(a)
        ev.destroy(b)

    elapsed = t1 - t0
    _progress(f"timed {args.steps} steps: {elapsed / args.steps * 1e3:.4f} ms per step")
    ms_per_step = elapsed / args.steps * 1e3
    value = E * args.steps / elapsed
    dom_avg_ms = float(np.mean(dom_ms))
    # The dominant kernel is priced with the bytes of the step it carries out, from the
    # step's definition (for the class-scatter kernels: row_ptr, col, val, labels, the
    # gathered coefficients and Z), not with this library's own layout.
    dstep = KERNEL_STEP.get(dominant)
    alg = step_bytes(dstep, E, N, K, M, weighted) if dstep else algorithmic_bytes(dominant, E, N, K, M, weighted,
                                                                                   n_empty)
    layout = algorithmic_bytes(dominant, E, N, K, M, weighted, n_empty)
    achieved = alg / (dom_avg_ms * 1e-3) / 1e9
    trf = read_traffic(g.name)
    tk = trf["kernels"].get(dominant) if trf else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tk["bytes"] if tk else None,
                "kernel": dominant, "step": dstep, "algorithmic_bytes_per_launch": int(alg),
                "layout_bytes_per_launch": int(layout),
                "layout_frac": round(layout / (dom_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "avg_launch_ms": round(dom_avg_ms, 5)}
    roofline["copy_ceiling_GBps"] = copy_ceiling(torch, dev)
    if tk:
        roofline["traffic_unit"] = "bytes per launch (L2 fabric read + write requests by size)"
        roofline["traffic_read"] = tk["read_bytes"]
        roofline["traffic_write"] = tk["write_bytes"]
        roofline["traffic_over_algorithmic"] = round(tk["bytes"] / alg, 3)

    # The whole call: hipEvent times warm and cold (a 512 MiB overwrite before each call
    # evicts the last-level cache), the call captured in a hipGraph, the HBM fractions of
    # its minimum bytes, and the counter bytes of its kernels over their summed durations.
    cold = torch.empty((512 << 20) // 4, dtype=torch.float32, device=dev)
    warm_t = call_times(torch, step)
    cold_t = call_times(torch, step, cold=cold)
    graph_t = graph_times(torch, step, out=Z)
    e2e_min_bytes = step_bytes("e2e", E, N, K, M, weighted)
    embed_bytes = step_bytes("embed", E, N, K, M, weighted)
    embed_ms = sum(ms for k, ms in per_kernel.items() if KERNEL_STEP.get(k) in ("a3", "a4_a6"))
    call = {"warm": warm_t, "cold": cold_t, "graph_captured": graph_t,
            "e2e_min_bytes": int(e2e_min_bytes),
            "e2e_hbm_frac_warm": round(e2e_min_bytes / (warm_t["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "e2e_hbm_frac_cold": round(e2e_min_bytes / (cold_t["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "embed_bytes": int(embed_bytes), "embed_kernels_ms": round(embed_ms, 5),
            "embed_hbm_frac": round(embed_bytes / (embed_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if embed_ms else None}
    if trf:
        ks = [k for k in per_kernel if k in trf["kernels"]]
        cb = sum(trf["kernels"][k]["bytes"] for k in ks)
        cms = sum(per_kernel[k] for k in ks)
        call.update({"counter_bytes": int(cb), "counter_kernels_ms": round(cms, 5),
                     "call_counter_GBps": round(cb / (cms * 1e-3) / 1e9, 1),
                     "call_counter_frac": round(cb / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "counter_kernels": len(ks), "kernels_without_counters": sorted(set(per_kernel) - set(ks))})
    else:
        call.update({"counter_bytes": None, "call_counter_GBps": None,
                     "counter_note": "no counter summary for the current HIP sources"})
    _progress("call timings done")

    # Steady state on a resident CSR (re-embedding, the serving/iterative form).
    Zr = torch.empty_like(Z)
    ws2 = torch.empty(max(1, gee.gee_embed_csr_workspace_bytes(M, N, K, flags)), dtype=torch.uint8, device=dev)
    for _ in range(3):
        gee.gee_embed_csr(rp, col, val, M, lab, K, flags, Z=Zr, workspace=ws2, stream=stream)
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    for _ in range(args.steps):
        gee.gee_embed_csr(rp, col, val, M, lab, K, flags, Z=Zr, workspace=ws2, stream=stream)
    torch.cuda.synchronize()
    resident_ms = (time.perf_counter() - tr0) / args.steps * 1e3
    nzm = Z != 0
    rel_diff = float(((Z - Zr).abs()[nzm] / Z.abs()[nzm]).max().item()) if bool(nzm.any()) else 0.0
    zeros_same = bool(torch.equal(Z == 0, Zr == 0))
    del Zr, ws2

    kernels = {}
    for name, ms in per_kernel.items():
        b = algorithmic_bytes(name, E, N, K, M, weighted, n_empty)
        kernels[name] = {"ms": round(ms, 5), "step": KERNEL_STEP.get(name), "layout_bytes": int(b),
                         "layout_GB_per_s": round(b / (ms * 1e-3) / 1e9, 1) if (b and ms > 0) else None}
        if trf and name in trf["kernels"]:
            cb = trf["kernels"][name]["bytes"]
            kernels[name]["counter_bytes"] = cb
            kernels[name]["counter_GB_per_s"] = round(cb / (ms * 1e-3) / 1e9, 1) if ms > 0 else None

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": g.name, "N": N, "E": E, "M_csr_entries": M, "K": K,
                   "options": "+".join(o for o, on in (("diag", g.diag), ("laplacian", g.lap),
                                                       ("correlation", g.cor)) if on) or "none",
                   "weighted": weighted, "symmetrize": g.sym, "schedule": gee.gee_default_schedule(E, N, K, flags)},
        "roofline": roofline,
        "call": call,
        "e2e_hbm_frac_min_bytes": round(e2e_min_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": kernels,
        "resident_csr_embed": {"ms_per_call": round(resident_ms, 5),
                               "edges_per_s": round(E / (resident_ms * 1e-3), 1),
                               "max_rel_diff_to_edge_list_path": rel_diff,
                               "same_zero_entries_as_edge_list_path": zeros_same},
    }
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    if "csr" in legs:
        out["csr_build"] = csr_build_leg(torch, np, gee, g, (src, dst, w, lab), M, cold)
        _progress("CSR-build leg done")
    del rp, col, val
    if "configs" in legs:
        out["configs"] = {nm: config_leg(torch, np, gee, dev, nm, cold)
                          for nm in ("sbm_small_off", "sbm_small_all", "sbm_dense")}
        torch.cuda.empty_cache()
        _progress("configs leg done")
    if "original" in legs:
        out["original_gee_form"] = original_leg(torch, np, gee, lib, dev, g, (src, dst, w, lab), Z, args.steps, ev)
        _progress("original-form leg done")
        torch.cuda.empty_cache()
    if "sparse" in legs:
        out["sparse_z"] = sparse_leg(torch, np, gee, lib, dev, g, (src, dst, w, lab), Z, args.steps, ev)
        torch.cuda.empty_cache()
        _progress("sparse-Z leg done")
    del cold
    legs = [x for x in legs if x in ("batched", "serving")]
    if legs:
        from paper_2406_03726_amd.autotune import ScheduleTable

        table = ScheduleTable.load()
        if "batched" in legs:
            out["batched"] = batched_leg(torch, np, gee, dev, table, args.procs)
            _progress("batched leg done")
            torch.cuda.empty_cache()
        if "serving" in legs:
            out["serving"] = serving_leg(torch, np, gee, dev, table, args.procs)
            _progress("serving leg done")
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g)
    else:
        out["cpu_baseline"] = None
    line = json.dumps(out)
    if args.report:
        with open(args.report, "w") as f:
            json.dump({**out, "generation_s": t_gen, "dominant_ms_all": dom_ms}, f, indent=1)
    print(line, flush=True)


if __name__ == "__main__":
    main()
