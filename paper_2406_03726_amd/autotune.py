"""Schedule autotuner: per graph-statistics bucket, the embed schedule (the part size of
gee_embed's bucket path) that measured fastest on this device, kept as a JSON table.

A graph is bucketed by (log2 of its CSR entry count, average-degree class, class-count
class). For every bucket the tuner embeds a few seeded synthetic graphs of that shape with
each candidate schedule, times the calls with HIP events, and keeps the fastest. Lookups of
a bucket the table lacks fall back to the library's own default (zero fields).

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
TABLE_VERSION = 1
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules_gfx950.json")

# entries per bucket part of gee_embed's bucket path (the library raises anything below
# 2048 to 2048 there)
WAVE_ENTRIES = (2048, 4096, 8192, 16384)
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
    """Bucket -> schedule fields (wave_entries, bucket_rows_log2); missing fields and
    buckets mean the library default."""
    entries: Dict[Key, Dict[str, int]] = field(default_factory=dict)
    device: str = "gfx950"
    meta: Dict[str, object] = field(default_factory=dict)

    def lookup(self, E: int, N: int, K: int, flags: int) -> Dict[str, int]:
        """The bucket's schedule; else the tuned bucket of the same degree and class-count
        classes nearest in size (the smaller one on a tie); else {} (library default)."""
        key = bucket_of(E, N, K, flags)
        e = self.entries.get(key)
        if e is None:
            near = [k for k in self.entries if k[1:] == key[1:]]
            if near:
                e = self.entries[min(near, key=lambda k: (abs(k[0] - key[0]), k[0]))]
        return dict(e) if e else {}

    def to_json(self) -> str:
        rows = [{"log2_entries": k[0], "degree_class": k[1], "class_count_class": k[2], **v}
                for k, v in sorted(self.entries.items())]
        return json.dumps({"version": TABLE_VERSION, "device": self.device, "meta": self.meta,
                           "degree_class_edges": list(DEG_EDGES), "class_count_class_edges": list(K_EDGES),
                           "entries": rows}, indent=1)

    @classmethod
    def from_json(cls, text: str) -> "ScheduleTable":
        d = json.loads(text)
        if d.get("version") != TABLE_VERSION:
            raise ValueError(f"schedule table version {d.get('version')} is not {TABLE_VERSION}")
        if tuple(d.get("degree_class_edges", DEG_EDGES)) != DEG_EDGES or \
                tuple(d.get("class_count_class_edges", K_EDGES)) != K_EDGES:
            raise ValueError("schedule table uses other bucket edges")
        t = cls(device=d.get("device", "gfx950"), meta=d.get("meta", {}))
        for r in d["entries"]:
            key = (int(r["log2_entries"]), int(r["degree_class"]), int(r["class_count_class"]))
            sched = {f: int(r[f]) for f in ("wave_entries", "waves_per_block", "bucket_rows_log2") if f in r}
            _validate(sched)
            t.entries[key] = sched
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


BUCKET_ROWS = (0, 8)  # CSR sort only: 0 the library's rule, 8 256-row buckets (pass-C partition)


def candidates(with_bucket_rows: bool = False) -> List[Dict[str, int]]:
    """Part sizes; with_bucket_rows also crosses them with CSR-sort bucket sizes (which
    gee_embed's bucket path does not read: it fixes its own bucket size)."""
    out = [{"wave_entries": we} for we in WAVE_ENTRIES]
    if with_bucket_rows:
        out = [dict(c, bucket_rows_log2=sb) for c in out for sb in BUCKET_ROWS]
    return out


def tune(shapes: Iterable[Tuple[int, int, int, int]], time_fn: Callable[[Tuple[int, int, int, int], Dict[str, int]], float],
         cands: Optional[List[Dict[str, int]]] = None, table: Optional[ScheduleTable] = None) -> ScheduleTable:
    """For each (E, N, K, flags) shape, time every candidate with `time_fn(shape, sched)`
    (seconds, lower is better) and store the fastest for the shape's bucket. Several shapes
    of one bucket add their times."""
    table = table or ScheduleTable()
    cands = cands or candidates()
    per_bucket: Dict[Key, Dict[Tuple[Tuple[str, int], ...], float]] = {}
    for shape in shapes:
        key = bucket_of(*shape)
        acc = per_bucket.setdefault(key, {})
        for c in cands:
            t = float(time_fn(shape, c))
            ck = tuple(sorted((k, v) for k, v in c.items() if v))
            acc[ck] = acc.get(ck, 0.0) + t
    for key, timings in per_bucket.items():
        table.entries[key] = choose(timings)
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


def gpu_time_fn(reps: int = 5):
    """time_fn for tune(): seeded Chung-Lu graph of the shape on cuda:0, median of `reps`
    gee_embed_ws calls measured with HIP events (after one warmup)."""
    import numpy as np
    import torch

    from . import gee
    from gee_workloads.generators import chung_lu_edges, rng_for, shuffle_and_orient, uniform_weights

    cache: Dict[Tuple[int, int, int, int], tuple] = {}
    dev = torch.device("cuda:0")

    def graph(shape):
        if shape not in cache:
            E, N, K, flags = shape
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
            cache[shape] = (t(s, torch.int32), t(d, torch.int32), t(w, torch.float32), t(lab, torch.int32),
                            torch.empty((N, K), dtype=torch.float32, device=dev))
        return cache[shape]

    def time_fn(shape, sched):
        src, dst, w, lab, Z = graph(shape)
        K, flags = shape[2], shape[3]
        nbytes = gee.gee_embed_workspace_bytes(src.numel(), lab.numel(), K, flags, True, sched)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        gee.gee_embed(src, dst, w, lab, K, flags, Z=Z, sched=sched, workspace=ws)
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            gee.gee_embed(src, dst, w, lab, K, flags, Z=Z, sched=sched, workspace=ws)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return float(np.median(ts))

    return time_fn


def main(argv=None):
    ap = argparse.ArgumentParser(description="Tune embed schedules on this GPU and write the table.")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    t0 = time.time()
    shapes = default_shapes()
    table = tune(shapes, gpu_time_fn(args.reps))
    table.meta = {"shapes": len(shapes), "wave_entries": list(WAVE_ENTRIES), "seconds": round(time.time() - t0, 1)}
    table.save(args.out)
    print(f"wrote {len(table.entries)} buckets to {args.out} in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
