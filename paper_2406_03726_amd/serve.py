"""Serving loop: graph-embedding requests admitted by a device-memory budget and run with
continuous batching over several HIP streams.

A request is one graph whose inputs are already on the device (edge list, weights,
labels). The server keeps a FIFO queue. Whenever a stream slot is free it admits the
longest prefix of the queue whose batch footprint (the workspace the library needs for
exactly that batch, plus the batch's Z outputs) fits the free budget, and launches those
requests as one batch (gee_embed_batch_ws) on that slot's stream. Batches on different
streams overlap on the device; a request that arrives while others run is admitted as
soon as a slot and memory free up. Admission is
strictly FIFO, so a large request at the head waits for memory rather than being passed
(no starvation); a request larger than the whole budget is rejected.

Each request's schedule comes from its own sizes (the autotuned table or the library
default), so its Z is bitwise the same whether it runs alone or batched with others.

Optionally the edges of the batches in flight are capped: a request that would exceed
the cap waits (FIFO) until enough of the device is free, and runs alone when it exceeds
the cap by itself.

The scheduler is host logic over a small backend interface, so it can be driven by the
GPU backend or, in tests, by a simulated one on a virtual clock.
"""

from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence


@dataclass
class Request:
    rid: int
    graph: Dict[str, Any]          # src, dst, w (or None), labels, K, flags[, sched]
    arrival: float                 # scheduled arrival time (server clock, seconds)
    E: int = 0
    N: int = 0
    nbytes: int = 0                # footprint while admitted
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Any = None
    error: Optional[str] = None
    cancelled: bool = False

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


class Backend:
    """What the scheduler needs from a device."""

    slots: int = 1

    def footprint(self, req: Request) -> int:
        raise NotImplementedError

    def batch_footprint(self, reqs: List[Request]) -> int:
        """Bytes a batch of these requests holds while it runs. A batch's workspace can exceed
        the sum of its members' own (its tables are sized by the batch's largest class count
        and partition digits), so a backend that knows better says so here."""
        return sum(r.nbytes for r in reqs)

    def launch(self, reqs: List[Request], slot: int) -> Any:
        """Start one batch on slot `slot`; returns a handle."""
        raise NotImplementedError

    def poll(self, handle: Any) -> bool:
        """True once the batch has finished (results available)."""
        raise NotImplementedError

    def finish(self, handle: Any, reqs: List[Request]) -> None:
        """Hand results to the requests and release the batch's resources."""
        raise NotImplementedError


@dataclass
class _Flight:
    slot: int
    handle: Any
    reqs: List[Request]
    nbytes: int
    edges: int = 0
    bigs: int = 0


class GeeServer:
    def __init__(self, backend: Backend, budget_bytes: int, max_batch: int = 64,
                 clock: Callable[[], float] = time.perf_counter, max_batch_edges: Optional[int] = None,
                 max_inflight_edges: Optional[int] = None,
                 on_done: Optional[Callable[[Request], None]] = None,
                 big_edges: Optional[int] = None, max_big_inflight: int = 1):
        if budget_bytes <= 0 or max_batch < 1:
            raise ValueError("budget and batch size must be positive")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        # A batch finishes as a whole: a cap on its edges keeps small requests from
        # waiting for a large one batched with them (a larger request still runs alone).
        self.max_batch_edges = max_batch_edges
        # Batches in flight share the device: a cap on their edges keeps a large request
        # from being slowed by others running beside it (it waits for the device to empty,
        # as it would in the plain loop, and then runs alone).
        self.max_inflight_edges = max_inflight_edges
        self.inflight_edges = 0
        # Large requests (at least big_edges edges) run at most max_big_inflight at a time:
        # two of them side by side would each be slowed by the other. A large request that
        # has to wait for that lets the smaller requests behind it go first.
        self.big_edges = big_edges
        self.max_big_inflight = int(max_big_inflight)
        self.big_inflight = 0
        self.clock = clock
        # called once per request as it completes (e.g. to check and release its result)
        self.on_done = on_done
        self.queue: Deque[Request] = deque()
        self.flights: List[_Flight] = []
        self.free_slots = list(range(backend.slots))
        self.in_use = 0
        self.peak_in_use = 0
        self.peak_flights = 0
        self.done: List[Request] = []
        self.launch_log: List[List[int]] = []   # request ids of every batch, in launch order

    # --------------------------------------------------------------------- intake
    def hold(self, nbytes: int) -> None:
        """Takes bytes out of the request budget for as long as something else holds them
        (a resident CSR, say); a negative value gives them back."""
        self.budget -= int(nbytes)
        if self.budget <= 0:
            raise ValueError("holding more than the whole budget")

    def submit(self, req: Request) -> None:
        try:
            req.nbytes = int(self.backend.footprint(req))
        except (KeyError, ValueError) as e:  # e.g. a re-embedding of a graph not resident
            req.error = f"invalid request: {e!r}"
            req.t_done = self.clock()
            self.done.append(req)
            return
        if req.nbytes > self.budget:
            req.error = f"request needs {req.nbytes} bytes, more than the whole budget of {self.budget}"
            req.t_done = self.clock()
            self.done.append(req)
            return
        self.queue.append(req)

    def cancel(self, rid: int) -> bool:
        """Cancel a queued (not yet admitted) request."""
        for r in self.queue:
            if r.rid == rid:
                r.cancelled = True
                return True
        return False

    # --------------------------------------------------------------------- scheduling
    def _reap(self) -> int:
        n = 0
        still = []
        for f in self.flights:
            if self.backend.poll(f.handle):
                self.backend.finish(f.handle, f.reqs)
                now = self.clock()
                for r in f.reqs:
                    r.t_done = now
                    self.done.append(r)
                    if self.on_done is not None:
                        self.on_done(r)
                self.in_use -= f.nbytes
                self.inflight_edges -= f.edges
                self.big_inflight -= f.bigs
                self.free_slots.append(f.slot)
                n += 1
            else:
                still.append(f)
        self.flights = still
        return n

    def _admit(self) -> int:
        launched = 0
        while self.free_slots and self.queue:
            while self.queue and self.queue[0].cancelled:
                r = self.queue.popleft()
                r.error = "cancelled"
                r.t_done = self.clock()
                self.done.append(r)
            if not self.queue:
                break
            batch: List[Request] = []
            nbytes = 0
            edges = 0
            bigs = 0
            for r in self.queue:
                if len(batch) >= self.max_batch:
                    break
                if r.cancelled:
                    continue
                big = self.big_edges is not None and r.E >= self.big_edges
                if big and self.big_inflight + bigs >= self.max_big_inflight:
                    continue  # waits for the large request in flight; smaller ones pass it
                # the batch is charged what it holds with r in it, not the sum of its members
                need = self.backend.batch_footprint(batch + [r]) if batch else r.nbytes
                if self.in_use + need > self.budget:
                    break  # FIFO: nothing behind a request that does not fit yet
                if batch and self.max_batch_edges is not None and edges + r.E > self.max_batch_edges:
                    break  # the next batch starts with this request
                if (self.max_inflight_edges is not None and (batch or self.flights)
                        and self.inflight_edges + edges + r.E > self.max_inflight_edges):
                    break  # FIFO: wait until the device has room for this request
                batch.append(r)
                nbytes = need
                edges += r.E
                bigs += 1 if big else 0
            if not batch:
                break
            ids = {id(r) for r in batch}
            self.queue = deque(r for r in self.queue if id(r) not in ids)
            slot = self.free_slots.pop(0)
            now = self.clock()
            for r in batch:
                r.t_admit = now
            handle = self.backend.launch(batch, slot)
            self.flights.append(_Flight(slot, handle, batch, nbytes, edges, bigs))
            self.in_use += nbytes
            self.inflight_edges += edges
            self.big_inflight += bigs
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.peak_flights = max(self.peak_flights, len(self.flights))
            self.launch_log.append([r.rid for r in batch])
            launched += 1
        return launched

    def step(self) -> int:
        """Reap finished batches, then admit and launch; returns the number of events."""
        return self._reap() + self._admit()

    @property
    def idle(self) -> bool:
        return not self.queue and not self.flights

    # --------------------------------------------------------------------- traces
    def run_trace(self, reqs: Sequence[Request], sleep: Callable[[float], None] = time.sleep,
                  poll_interval: float = 20e-6, busy_poll: bool = False) -> List[Request]:
        """Feed requests at their arrival times (relative to now) and run until all are done.
        With busy_poll (a real clock), the loop polls the batches in flight without sleeping
        and waits for the next arrival with wait_until, so neither a completion nor an
        arrival is seen late by a sleep's overshoot."""
        t0 = self.clock()
        pending = sorted(reqs, key=lambda r: r.arrival)
        for r in pending:
            r.arrival += t0
        i = 0
        while i < len(pending) or not self.idle:
            now = self.clock()
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            if self.step() == 0:
                if busy_poll:
                    if self.flights or i >= len(pending):
                        continue
                    if not self.queue:
                        wait_until(pending[i].arrival, self.clock, sleep)
                        continue
                nxt = pending[i].arrival - now if i < len(pending) else poll_interval
                sleep(max(0.0, min(poll_interval, nxt)))
        return list(reqs)


def wait_until(t: float, clock: Callable[[], float] = time.perf_counter,
               sleep: Callable[[float], None] = time.sleep, spin: float = 300e-6) -> None:
    """Returns at clock() >= t: sleeps until `spin` seconds before t (a sleep can overshoot
    by tens of microseconds), then polls the clock."""
    while True:
        dt = t - clock()
        if dt <= 0:
            return
        if dt > spin:
            sleep(dt - spin)


def run_plain(reqs: Sequence[Request], embed_one: Callable[[Request], None],
              clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
              on_done: Optional[Callable[[Request], None]] = None, busy_poll: bool = False):
    """The plain per-request loop: one host thread, FIFO, each request embedded alone and
    waited for before the next one starts (with busy_poll, arrivals are waited for with
    wait_until)."""
    t0 = clock()
    order = sorted(reqs, key=lambda r: r.arrival)
    for r in order:
        r.arrival += t0
    for r in order:
        now = clock()
        if r.arrival > now:
            if busy_poll:
                wait_until(r.arrival, clock, sleep)
            else:
                sleep(r.arrival - now)
        r.t_admit = clock()
        embed_one(r)
        r.t_done = clock()
        if on_done is not None:
            on_done(r)
    return list(reqs)


def percentile(xs: Sequence[float], q: float) -> float:
    """Linear-interpolated percentile (the numpy default), q in [0, 100]."""
    s = sorted(xs)
    if not s:
        return float("nan")
    pos = (len(s) - 1) * q / 100.0
    lo = int(pos)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (pos - lo)


def summarize(reqs: Sequence[Request]) -> Dict[str, float]:
    ok = [r for r in reqs if r.error is None and r.t_done is not None]
    lat = [r.latency for r in ok]
    if not ok:
        return {"completed": 0}
    span = max(r.t_done for r in ok) - min(r.arrival for r in ok)
    return {"completed": len(ok), "rejected": sum(1 for r in reqs if r.error is not None),
            "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
            "mean_ms": sum(lat) / len(lat) * 1e3,
            "edges_per_s": sum(r.E for r in ok) / span if span > 0 else float("nan")}


# ----------------------------------------------------------------------------- GPU backend

class GpuBackend(Backend):
    """Batches run with gee_embed_batch_ws on `slots` torch streams (default priority).
    A batch is charged the library's workspace size for exactly that batch plus its Z
    outputs; the bytes each batch actually allocates are tracked too (peak_actual).
    A batch's data errors are taken in stream order into pinned memory (no stream wait)
    and read when it finishes; when a batch of several requests reports one, each request
    is embedded again alone to find the ones that carry it, and only those get an error.

    Re-embedding: make_resident(gid, ...) builds a graph's CSR (gee_build_csr) and keeps it
    on the device; a request whose graph dict holds {"resident": gid, "labels", "K",
    "flags"} is then embedded from that CSR with its own labels (gee_embed_csr: class
    counts, degrees and the class scatter, no sort), the iterative use of GEE with changing
    labels. Such requests run in the same batches, on the same stream, one call each."""

    def __init__(self, slots: int = 4, table=None, use_plans: bool = False, plan_reserve: int = 256 << 20,
                 sync_inputs: bool = True):
        import torch

        from . import _lib, gee

        self._torch = torch
        self._lib = _lib
        # sync_inputs: each batch's stream first waits for the submitting stream (the requests'
        # inputs may still be in flight there); a caller whose inputs are all complete before
        # they are submitted (a staged pool) can turn it off
        self.sync_inputs = sync_inputs
        # use_plans: each slot keeps one batch plan (a captured launch sequence) and gives it
        # every batch of edge-list requests with gee_batch_plan_update (no allocation while
        # the batch fits the plan's workspace, reserved at plan_reserve bytes or more)
        self.use_plans = use_plans
        self.plan_reserve = int(plan_reserve)
        self._plans = [None] * slots
        # host seconds spent in launch() and finish(), and their calls (for measurements)
        self.host_s = {"launch": 0.0, "finish": 0.0, "launches": 0}
        self._gee = gee
        self.slots = slots
        self._streams = None  # made at the first launch (sizing needs no device)
        self._errs = None     # per slot: pinned int32 the batch's data-error bits land in
        self.table = table
        self.in_use_actual = 0
        self.peak_actual = 0
        self.resident: Dict[Any, Dict[str, Any]] = {}
        self._ws = [None] * slots  # per slot: grow-only workspace (one batch per slot at a time)

    @property
    def streams(self):
        if self._streams is None:
            self._streams = [self._torch.cuda.Stream() for _ in range(self.slots)]
            self._errs = [self._torch.zeros(1, dtype=self._torch.int32, pin_memory=True) for _ in range(self.slots)]
        return self._streams

    # --------------------------------------------------------------- resident CSRs
    def make_resident(self, gid, src, dst, w, N: int, flags: int) -> int:
        """Builds and keeps the CSR of an edge list under `gid`; returns the bytes it holds
        (a server can hold them out of its request budget with GeeServer.hold)."""
        torch = self._torch
        rp, col, val = self._gee.gee_build_csr(src, dst, w, N, flags)
        torch.cuda.synchronize()
        if self._gee.gee_get_data_errors() != 0:
            raise ValueError(f"graph {gid!r}: the edge list has data errors")
        M = int(rp[-1].item())
        col = col[:M].clone()
        val = val[:M].clone() if val is not None else None
        nbytes = rp.numel() * 4 + col.numel() * 4 + (val.numel() * 4 if val is not None else 0)
        self.resident[gid] = dict(rp=rp, col=col, val=val, M=M, N=N, nbytes=nbytes)
        return nbytes

    def release(self, gid) -> int:
        """Drops a resident CSR; returns the bytes it held."""
        return self.resident.pop(gid)["nbytes"]

    def _csr_sched(self, g: Dict[str, Any], res: Dict[str, Any]):
        if g.get("sched") is not None:
            return g["sched"]
        if self.table is None:
            return None
        s = self.table.lookup(res["M"], res["N"], int(g["K"]), int(g["flags"]) & ~8, path="csr")
        return s or None

    def sched_of(self, g: Dict[str, Any]) -> Optional[Dict[str, int]]:
        if g.get("sched") is not None:
            return g["sched"]
        if self.table is None:
            return None
        # the lookup depends on the graph's sizes alone: kept with the graph
        key = ("_gee_sched", id(self.table))
        if key not in g:
            g[key] = self.table.lookup(g["src"].numel(), g["labels"].numel(), int(g["K"]), int(g["flags"])) or None
        return g[key]

    def _struct(self, r: Request, Z):
        """The request's gee_graph with its output Z: the graph's part is checked and built
        once (by the binding) and kept with the graph."""
        g = r.graph
        key = ("_gee_struct", id(self.table))
        if key not in g:
            g[key] = self._gee._graph_struct(dict(g, Z=None, sched=self.sched_of(g)), g["labels"].device,
                                             sizing=True)
        st = self._lib.GeeGraph.from_buffer_copy(g[key])
        st.Z = Z.data_ptr()
        return st

    def _item(self, r: Request, Z=None):
        g = r.graph
        return dict(src=g["src"], dst=g["dst"], w=g.get("w"), labels=g["labels"], K=int(g["K"]),
                    flags=int(g["flags"]), Z=Z, sched=self.sched_of(g))

    def _sizes(self, r: Request):
        g = r.graph
        return (r.E, r.N, int(g["K"]), int(g["flags"]), g.get("w") is not None, self.sched_of(g))

    def _csr_ws_bytes(self, r: Request) -> int:
        g = r.graph
        res = self.resident[g["resident"]]
        return int(self._gee.gee_embed_csr_workspace_bytes(res["M"], res["N"], int(g["K"]),
                                                           int(g["flags"]) & ~8, self._csr_sched(g, res)))

    def footprint(self, r: Request) -> int:
        g = r.graph
        if "resident" in g:
            if (int(g["flags"]) & 16) and (int(g["flags"]) & 2):
                raise ValueError("a resident CSR has no column sums for the directed-degree Laplacian")
            res = self.resident[g["resident"]]
            r.E, r.N = res["M"], res["N"]
        else:
            r.E = int(g["src"].numel())
            r.N = int(g["labels"].numel())
        return self.batch_footprint([r])

    def _ws_bytes(self, reqs: List[Request]) -> int:
        """Workspace of a batch: the library's size for exactly these graphs (a graph alone
        keeps its own size with it)."""
        edge = [r for r in reqs if "resident" not in r.graph]
        if len(edge) == 1:
            g = edge[0].graph
            key = ("_gee_ws1", id(self.table))
            if key not in g:
                g[key] = int(self._gee.batch_workspace_bytes_of_sizes([self._sizes(edge[0])]))
            ws = g[key]
        else:
            ws = int(self._gee.batch_workspace_bytes_of_sizes([self._sizes(r) for r in edge])) if edge else 0
        return ws + sum(self._csr_ws_bytes(r) for r in reqs if "resident" in r.graph)

    def batch_footprint(self, reqs: List[Request]) -> int:
        return self._ws_bytes(reqs) + sum(4 * r.N * int(r.graph["K"]) for r in reqs)

    def _workspace(self, slot: int, nbytes: int, dev):
        w = self._ws[slot]
        if w is None or w.numel() < nbytes:
            w = self._torch.empty(max(nbytes, 1), dtype=self._torch.uint8, device=dev)
            self._ws[slot] = w
        return w

    def _embed_resident(self, r: Request, Z, s):
        g = r.graph
        res = self.resident[g["resident"]]
        ws = self._torch.empty(max(1, self._csr_ws_bytes(r)), dtype=self._torch.uint8, device=Z.device)
        self._gee.gee_embed_csr(res["rp"], res["col"], res["val"], res["M"], g["labels"], int(g["K"]),
                                int(g["flags"]) & ~8, Z=Z, sched=self._csr_sched(g, res), workspace=ws, stream=s)
        return ws

    def launch(self, reqs: List[Request], slot: int):
        t0 = time.perf_counter()
        h = self._launch(reqs, slot)
        self.host_s["launch"] += time.perf_counter() - t0
        self.host_s["launches"] += 1
        return h

    def _launch(self, reqs: List[Request], slot: int):
        torch = self._torch
        s = self.streams[slot]
        dev = reqs[0].graph["labels"].device
        # the requests' inputs were made on the submitting stream
        if self.sync_inputs:
            s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            items, held_ws = [], []
            for r in reqs:
                Z = torch.empty((r.N, int(r.graph["K"])), dtype=torch.float32, device=dev)
                items.append(self._item(r, Z=Z) if "resident" not in r.graph else dict(Z=Z))
            edge = [it for r, it in zip(reqs, items) if "resident" not in r.graph]
            if edge and self.use_plans:
                # the slot's batch plan takes this batch (the previous one on this slot has
                # finished); a plan too small for it is replaced by a larger one
                nbytes = self._ws_bytes([r for r in reqs if "resident" not in r.graph])
                plan = self._plans[slot]
                if plan is not None and plan.workspace_bytes >= nbytes:
                    plan.update(edge)
                else:
                    if plan is not None:
                        plan.destroy()
                    plan = self._gee.BatchPlan(edge, workspace_bytes=max(nbytes, self.plan_reserve))
                    self._plans[slot] = plan
                plan.launch(stream=s)
            elif edge:
                # the slot's own workspace, grown to this batch's size (the library's size
                # for exactly these graphs; the previous batch on this slot has finished)
                er = [r for r in reqs if "resident" not in r.graph]
                nbytes = self._ws_bytes(er)
                ws = self._workspace(slot, nbytes, dev)
                arr = (self._lib.GeeGraph * len(er))(*[self._struct(r, it["Z"]) for r, it in zip(er, edge)])
                rc = self._lib.load().gee_embed_batch_ws(arr, len(er), ws.data_ptr(), nbytes,
                                                         ctypes.c_void_p(s.cuda_stream))
                if rc != 0:
                    raise self._gee.GeeError(rc, "gee_embed_batch_ws")
                held_ws.append(ws[:nbytes])
            for r, it in zip(reqs, items):
                if "resident" in r.graph:
                    held_ws.append(self._embed_resident(r, it["Z"], s))
            # the batch's data-error bits, taken in stream order into pinned memory, so the
            # host reads them at completion without synchronizing the stream
            err = self._errs[slot]
            self._gee.gee_take_data_errors_async(err, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        held = sum(w.numel() for w in held_ws) + sum(it["Z"].numel() * 4 for it in items)
        self.in_use_actual += held
        self.peak_actual = max(self.peak_actual, self.in_use_actual)
        return (ev, items, held_ws, s, held, err)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle, reqs: List[Request]) -> None:
        t0 = time.perf_counter()
        try:
            self._finish(handle, reqs)
        finally:
            self.host_s["finish"] += time.perf_counter() - t0

    def _finish(self, handle, reqs: List[Request]) -> None:
        _, items, _, s, held, err = handle
        self.in_use_actual -= held
        bits = int(err[0])
        for r, it in zip(reqs, items):
            r.result = it["Z"]
        if not bits:
            return
        if len(reqs) == 1:
            reqs[0].error = f"data error (bits {bits:#x})"
            reqs[0].result = None
            return
        for r, it in zip(reqs, items):
            with self._torch.cuda.stream(s):
                if "resident" in r.graph:
                    self._embed_resident(r, it["Z"], s)
                else:
                    self._gee.gee_embed_batch([it], stream=s)
            b = self._gee.gee_get_data_errors(s)
            if b:
                r.error = f"data error (bits {b:#x})"
                r.result = None
