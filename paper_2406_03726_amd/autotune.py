"""Schedule autotuner: per graph-statistics bucket, the schedules that measured fastest on
this device, kept as a JSON table, for the two paths a graph takes:

* edge lists (gee_embed, batches, serving): the bucket path's part size (entries per
  wavefront, `wave_entries`) crossed with its bucket size (32 or 64 rows,
  `bucket_rows_log2` 5 or 6);
* a resident CSR (gee_embed_csr, re-embedding with new labels): the embed kernel's
  entries per wavefront crossed with its wavefronts per workgroup (`waves_per_block`).

A graph is bucketed by (log2 of its CSR entry count, average-degree class, class-count
class). For every bucket the tuner embeds seeded synthetic graphs of that shape with each
candidate, times the calls with HIP events, and keeps the fastest. Candidates that give a
graph the same launch as another (a part size at least the graph's entry count) are not
timed twice. Lookups of a bucket the table lacks take the nearest tuned bucket of the same
degree and class-count classes, else the library's own default (zero fields).

The schedule changes only speed and floating-point summation order; a graph gets the
same schedule whether it is embedded alone or inside a batch (the lookup depends on the
graph's own sizes), so batched and plain results stay bitwise identical.

Usage on the GPU:  python -m paper_2406_03726_amd.autotune --out <table.json>
"""

from __future__ import annotations

import argparse
import json
import math
import os
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, Iterable, List, Optional, Tuple

GEE_SYMMETRIZE = 1 << 3
TABLE_VERSION = 2
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules_gfx950.json")

# entries per bucket part of gee_embed's bucket path (the library raises anything below
# 2048 to 2048 there), and its bucket sizes (log2 rows)
WAVE_ENTRIES = (2048, 4096, 8192, 16384)
BUCKET_SB = (5, 6)
# resident-CSR embed: entries per wavefront and wavefronts per workgroup
CSR_WAVE_ENTRIES = (256, 512, 1024, 2048, 4096)
CSR_WAVES_PER_BLOCK = (1, 2, 4)
PATHS = ("edge", "csr")
DEG_EDGES = (8.0, 32.0, 128.0)   # average degree classes: <8, <32, <128, >=128
K_EDGES = (16, 64)               # class-count classes: <=16, <=64, >64

Key = Tuple[int, int, int]


def entries_of(E: int, flags: int) -> int:
    """CSR entries bound of an edge list: 2E under symmetrization, else E."""
    return 2 * E if flags & GEE_SYMMETRIZE else E


def bucket_of(E: int, N: int, K: int, flags: int) -> Key:
    """(log2 of CSR entries rounded down, average-degree class, class-count class)."""
    M = max(entries_of(E, flags), 1)
    lm = int(math.floor(math.log2(M)))
    deg = M / max(N, 1)
    dc = sum(deg >= t for t in DEG_EDGES)
    kc = sum(K > t for t in K_EDGES)
    return (lm, dc, kc)


@dataclass
class ScheduleTable:
    """Bucket -> schedule fields, per path ("edge": edge lists, "csr": a resident CSR);
    missing fields and buckets mean the library default."""
    entries: Dict[Key, Dict[str, int]] = field(default_factory=dict)
    csr_entries: Dict[Key, Dict[str, int]] = field(default_factory=dict)
    device: str = "gfx950"
    meta: Dict[str, object] = field(default_factory=dict)

    def _of(self, path: str) -> Dict[Key, Dict[str, int]]:
        if path not in PATHS:
            raise ValueError(f"unknown path {path!r}")
        return self.entries if path == "edge" else self.csr_entries

    def lookup(self, E: int, N: int, K: int, flags: int, path: str = "edge") -> Dict[str, int]:
        """The bucket's schedule; else the tuned bucket of the same degree and class-count
        classes nearest in size (the smaller one on a tie); else {} (library default). For
        path "csr", E is the CSR's entry count and flags carry no symmetrization."""
        tab = self._of(path)
        key = bucket_of(E, N, K, flags)
        e = tab.get(key)
        if e is None:
            near = [k for k in tab if k[1:] == key[1:]]
            if near:
                e = tab[min(near, key=lambda k: (abs(k[0] - key[0]), k[0]))]
        return dict(e) if e else {}

    def to_json(self) -> str:
        def rows(tab):
            return [{"log2_entries": k[0], "degree_class": k[1], "class_count_class": k[2], **v}
                    for k, v in sorted(tab.items())]

        return json.dumps({"version": TABLE_VERSION, "device": self.device, "meta": self.meta,
                           "degree_class_edges": list(DEG_EDGES), "class_count_class_edges": list(K_EDGES),
                           "entries": rows(self.entries), "csr_entries": rows(self.csr_entries)}, indent=1)

    @classmethod
    def from_json(cls, text: str) -> "ScheduleTable":
        d = json.loads(text)
        if d.get("version") != TABLE_VERSION:
            raise ValueError(f"schedule table version {d.get('version')} is not {TABLE_VERSION}")
        if tuple(d.get("degree_class_edges", DEG_EDGES)) != DEG_EDGES or \
                tuple(d.get("class_count_class_edges", K_EDGES)) != K_EDGES:
            raise ValueError("schedule table uses other bucket edges")
        t = cls(device=d.get("device", "gfx950"), meta=d.get("meta", {}))
        for name, tab in (("entries", t.entries), ("csr_entries", t.csr_entries)):
            for r in d.get(name, []):
                key = (int(r["log2_entries"]), int(r["degree_class"]), int(r["class_count_class"]))
                sched = {f: int(r[f]) for f in ("wave_entries", "waves_per_block", "bucket_rows_log2") if f in r}
                _validate(sched)
                tab[key] = sched
        return t

    def save(self, path: str) -> None:
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            f.write(self.to_json())
        os.replace(tmp, path)

    @classmethod
    def load(cls, path: Optional[str] = None) -> "ScheduleTable":
        path = path or os.environ.get("GEE_SCHEDULE_TABLE") or DEFAULT_TABLE
        if not os.path.exists(path):
            return cls()
        with open(path) as f:
            return cls.from_json(f.read())


def _validate(s: Dict[str, int]) -> None:
    we = s.get("wave_entries", 0)
    if we and (we & (we - 1) or not 256 <= we <= 16384):
        raise ValueError(f"wave_entries {we} outside the library's range")
    wpb = s.get("waves_per_block", 0)
    if wpb and not 1 <= wpb <= 4:
        raise ValueError(f"waves_per_block {wpb} outside 1..4")
    sb = s.get("bucket_rows_log2", 0)
    if sb and not 1 <= sb <= 12:
        raise ValueError(f"bucket_rows_log2 {sb} outside 1..12")


def choose(timings: Dict[Tuple[Tuple[str, int], ...], float]) -> Dict[str, int]:
    """Fastest candidate; a tie goes to the candidate with fewer non-default fields, then
    to the smaller one in sorted order, so the choice is deterministic."""
    best = min(timings.items(), key=lambda kv: (kv[1], len(kv[0]), kv[0]))
    return dict(best[0])


def candidates(path: str = "edge", entries: Optional[int] = None) -> List[Dict[str, int]]:
    """The schedules timed for a shape. Edge lists: part sizes x 32/64-row buckets; part
    sizes at or above the shape's entry count all give one part per bucket, so only the
    smallest of them is kept. Resident CSR: the bucket kernels (part sizes x 32/64-row
    buckets, as for edge lists) and the CSR path's kernels (wavefront sizes x wavefronts per
    workgroup, wavefronts larger than the graph's entries dropped the same way)."""
    if path == "edge":
        we = list(WAVE_ENTRIES)
        if entries is not None:
            we = [w for w in we if w < entries] + [w for w in we if w >= entries][:1]
        return [{"wave_entries": w, "bucket_rows_log2": sb} for w in we for sb in BUCKET_SB]
    if path == "csr":
        we = list(CSR_WAVE_ENTRIES)
        if entries is not None:
            we = [w for w in we if w < entries] + [w for w in we if w >= entries][:1]
        return candidates("edge", entries) + [{"wave_entries": w, "waves_per_block": b} for w in we
                                               for b in CSR_WAVES_PER_BLOCK]
    raise ValueError(path)


def tune(shapes: Iterable[Tuple[int, int, int, int]], time_fn: Callable[[Tuple[int, int, int, int], Dict[str, int]], float],
         cands: Optional[List[Dict[str, int]]] = None, table: Optional[ScheduleTable] = None,
         path: str = "edge") -> ScheduleTable:
    """For each (E, N, K, flags) shape, time every candidate with `time_fn(shape, sched)`
    (seconds, lower is better) and store the fastest for the shape's bucket. Several shapes
    of one bucket add their times over the candidates they all timed. Without `cands`, each
    shape takes candidates(path, its entry count)."""
    table = table or ScheduleTable()
    tab = table._of(path)
    per_bucket: Dict[Key, Dict[Tuple[Tuple[str, int], ...], List[float]]] = {}
    for shape in shapes:
        key = bucket_of(*shape)
        acc = per_bucket.setdefault(key, {})
        cs = cands or candidates(path, entries_of(shape[0], shape[3]))
        for c in cs:
            t = float(time_fn(shape, c))
            ck = tuple(sorted((k, v) for k, v in c.items() if v))
            acc.setdefault(ck, []).append(t)
    for key, timings in per_bucket.items():
        n = max(len(v) for v in timings.values())
        full = {k: sum(v) for k, v in timings.items() if len(v) == n}
        tab[key] = choose(full)
    return table


# ----------------------------------------------------------------------------- GPU search

def default_shapes() -> List[Tuple[int, int, int, int]]:
    """Representative (E, N, K, flags) shapes covering the batched and serving workloads:
    entry counts from 2^11 to 2^25, average degree 5..200, K 2..128."""
    shapes = []
    for lm in (11, 14, 17, 20, 23):
        M = 1 << lm
        E = M // 2
        for deg in (6.0, 20.0, 60.0, 180.0):
            N = max(64, int(M / deg))
            for K in (8, 50, 128):
                shapes.append((E, N, K, 15))
    return shapes


def recipe_graphs(n_batched: int = 48, n_serving: int = 24, procs: int = 8):
    """Graphs drawn from the batched and the serving recipes (seeds of their own, not the
    benchmark's), as {(E, N, K, flags): Graph}: the tuner times these graphs themselves, so
    the buckets the two systems forms fall into are tuned on graphs of their kind (SBM and
    power-law, their degrees and class counts)."""
    import multiprocessing as mp

    with mp.get_context("spawn").Pool(procs) as pool:
        gs = pool.starmap(_recipe_graph, [("batched", 1000 + i) for i in range(n_batched)] +
                          [("serving", 1000 + i) for i in range(n_serving)], chunksize=1)
    out = {}
    for g in gs:
        f = (1 if g.diag else 0) | (2 if g.lap else 0) | (4 if g.cor else 0) | (GEE_SYMMETRIZE if g.sym else 0)
        out[(g.E, g.N, g.K, f)] = g
    return out


def _recipe_graph(kind: str, i: int):
    from gee_workloads.configs import batched_one, serving_one

    return batched_one(i) if kind == "batched" else serving_one(i)


def gpu_time_fn(reps: int = 5, path: str = "edge", given=None):
    """time_fn for tune(): seeded Chung-Lu graph of the shape (or the graph `given` holds
    for it) on cuda:0, median of `reps` calls measured with HIP events (after one warmup):
    gee_embed_ws for the edge-list path, gee_embed_csr_ws on the graph's CSR (built once)
    for the resident path."""
    import numpy as np
    import torch

    from . import gee
    from gee_workloads.generators import chung_lu_edges, rng_for, shuffle_and_orient, uniform_weights

    cache: Dict[Tuple[int, int, int, int], tuple] = {}
    dev = torch.device("cuda:0")

    def graph(shape):
        if shape not in cache:
            E, N, K, flags = shape
            if given is not None and shape in given:
                x = given[shape]
                s, d, lab = x.src, x.dst, x.labels
                w = x.w if x.w is not None else np.ones(x.E, np.float32)
            else:
                rng = rng_for(90, hash(shape) % (2 ** 31))
                E = min(E, N * (N - 1) // 4)
                dmax = min(N - 1.0, max(math.sqrt(N * 2.0 * E / N) * 4.0, 8.0))
                try:
                    s, d = chung_lu_edges(N, E, 2.1, dmax, rng)
                except ValueError:  # degree too close to N for a power law: uniform endpoints
                    s = rng.integers(0, N, size=E).astype(np.int32)
                    d = rng.integers(0, N, size=E).astype(np.int32)
                w = uniform_weights(s.shape[0], rng)
                s, d, w = shuffle_and_orient(s, d, w, rng)
                lab = rng.integers(0, K, size=N).astype(np.int32)
            t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
            g = (t(s, torch.int32), t(d, torch.int32), t(w, torch.float32), t(lab, torch.int32),
                 torch.empty((N, K), dtype=torch.float32, device=dev))
            if path == "csr":
                rp, col, val = gee.gee_build_csr(g[0], g[1], g[2], N, flags)
                torch.cuda.synchronize()
                g = g + (rp, col, val, int(rp[-1].item()))
            cache.clear()  # one graph at a time (the shapes come in order)
            cache[shape] = g
        return cache[shape]

    def time_fn(shape, sched):
        g = graph(shape)
        src, dst, w, lab, Z = g[:5]
        K, flags = shape[2], shape[3]
        if path == "csr":
            rp, col, val, M = g[5:]
            f2 = flags & ~GEE_SYMMETRIZE
            ws = torch.empty(max(1, gee.gee_embed_csr_workspace_bytes(M, lab.numel(), K, f2, sched)),
                             dtype=torch.uint8, device=dev)

            def call():
                gee.gee_embed_csr(rp, col, val, M, lab, K, f2, Z=Z, sched=sched, workspace=ws)
        else:
            nbytes = gee.gee_embed_workspace_bytes(src.numel(), lab.numel(), K, flags, True, sched)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)

            def call():
                gee.gee_embed(src, dst, w, lab, K, flags, Z=Z, sched=sched, workspace=ws)
        call()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            call()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return float(np.median(ts))

    return time_fn


def csr_shape(shape: Tuple[int, int, int, int]) -> Tuple[int, int, int, int]:
    """The resident-CSR lookup key of an edge-list shape: (CSR entries, N, K, flags
    without symmetrization)."""
    E, N, K, flags = shape
    return (entries_of(E, flags), N, K, flags & ~GEE_SYMMETRIZE)


def main(argv=None):
    ap = argparse.ArgumentParser(description="Tune embed schedules on this GPU and write the table.")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--paths", default="edge,csr")
    ap.add_argument("--no-recipes", action="store_true", help="synthetic shapes only")
    args = ap.parse_args(argv)
    t0 = time.time()
    given = {} if args.no_recipes else recipe_graphs()
    shapes = default_shapes() + list(given)
    print(f"{len(shapes)} shapes ({len(given)} drawn from the batched and serving recipes) in "
          f"{time.time() - t0:.1f} s", flush=True)
    table = ScheduleTable()
    for path in args.paths.split(","):
        tp = time.time()
        if path == "edge":
            tune(shapes, gpu_time_fn(args.reps, "edge", given), table=table, path="edge")
        else:
            # timed on the edge-list shape's graph, filed under its CSR's key
            fn = gpu_time_fn(args.reps, "csr", given)
            by_csr = {csr_shape(s): s for s in shapes}
            tune(list(by_csr), lambda cs, sched: fn(by_csr[cs], sched), table=table, path="csr")
        print(f"tuned the {path} path in {time.time() - tp:.1f} s", flush=True)
    table.meta = {"shapes": len(shapes), "recipe_graphs": len(given),
                  "wave_entries": list(WAVE_ENTRIES), "bucket_rows_log2": list(BUCKET_SB),
                  "csr_wave_entries": list(CSR_WAVE_ENTRIES), "csr_waves_per_block": list(CSR_WAVES_PER_BLOCK),
                  "seconds": round(time.time() - t0, 1)}
    table.save(args.out)
    print(f"wrote {len(table.entries)} + {len(table.csr_entries)} buckets to {args.out} in "
          f"{time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
