"""Serving loop on the GPU (needs an MI355X): requests of the serving recipe (scaled down)
admitted by budget and batched over streams; every result equals the request embedded
alone (bitwise) and matches the oracle."""

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from gee_workloads.configs import serving_one
from oracle import embed_graph as or_embed_graph
from paper_2406_03726_amd.autotune import ScheduleTable
from paper_2406_03726_amd.serve import GeeServer, GpuBackend, Request, summarize

from gpu_util import assert_close, flags, graph_tensors

pytestmark = pytest.mark.gpu


def _pool(n, e_max):
    gs = [serving_one(g, e_max=e_max) for g in range(n)]
    dev = []
    for g in gs:
        s, d, w, lab = graph_tensors(g)
        dev.append(dict(src=s, dst=d, w=w, labels=lab, K=g.K, flags=flags(g)))
    return gs, dev


@pytest.mark.parametrize("table", [False, True])
def test_served_equals_alone(table):
    print(f"[gpu-test] serving table={table}", flush=True)
    gs, dev = _pool(14, 200_000)
    tab = ScheduleTable.load() if table else None
    be = GpuBackend(slots=3, table=tab)
    budget = sum(be.footprint(Request(i, d, 0.0)) for i, d in enumerate(dev)) // 2
    srv = GeeServer(be, budget, max_batch=6)
    rng = np.random.default_rng(0)
    arr = np.cumsum(rng.exponential(2e-4, size=len(dev)))
    reqs = [Request(i, d, float(a)) for i, (d, a) in enumerate(zip(dev, arr))]
    srv.run_trace(reqs)
    torch.cuda.synchronize()
    assert srv.peak_in_use <= budget
    assert be.peak_actual <= budget  # bytes the batches really allocated
    assert any(len(b) > 1 for b in srv.launch_log), "no batch of several requests"
    assert srv.peak_flights > 1, "batches never overlapped"
    assert all(r.error is None for r in reqs)
    s = summarize(reqs)
    assert s["completed"] == len(reqs)
    for i, (r, g, d) in enumerate(zip(reqs, gs, dev)):
        alone = gee.gee_embed(d["src"], d["dst"], d["w"], d["labels"], d["K"], d["flags"],
                              sched=be.sched_of(d))
        torch.cuda.synchronize()
        assert torch.equal(r.result, alone), f"request {i}"
        if i % 4 == 0:
            assert_close(r.result, or_embed_graph(g), f"request {i} vs oracle")
