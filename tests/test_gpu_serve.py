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


def test_served_large_request_matches_oracle():
    """A request of the serving recipe above 5M edges served among small ones (busy-polled
    loop): equal to its plain call bit for bit and within tolerance of the oracle."""
    big = serving_one(0, e_max=20_000_000)  # request 0 of the pool draws about 5.6M edges
    assert big.E >= 5_000_000
    small = [serving_one(g, e_max=100_000) for g in range(1, 6)]
    gs = small[:3] + [big] + small[3:]
    print(f"[gpu-test] serving large request E={big.E} N={big.N} K={big.K}", flush=True)
    dev = []
    for g in gs:
        s, d, w, lab = graph_tensors(g)
        dev.append(dict(src=s, dst=d, w=w, labels=lab, K=g.K, flags=flags(g)))
    be = GpuBackend(slots=2)
    srv = GeeServer(be, 1 << 36, max_batch=8)
    reqs = [Request(i, d, 1e-4 * i) for i, d in enumerate(dev)]
    srv.run_trace(reqs, busy_poll=True)
    torch.cuda.synchronize()
    assert all(r.error is None for r in reqs)
    r = reqs[3]
    alone = gee.gee_embed(dev[3]["src"], dev[3]["dst"], dev[3]["w"], dev[3]["labels"], dev[3]["K"], dev[3]["flags"])
    torch.cuda.synchronize()
    assert torch.equal(r.result, alone)
    assert_close(r.result, or_embed_graph(big), "large served request vs oracle")


def test_reembed_requests_on_resident_csrs():
    """Re-embedding requests (new labels on a graph whose CSR the backend keeps resident)
    served in the same batches as edge-list requests: each equals gee_embed_csr alone bit
    for bit and the oracle within tolerance; an unknown graph id is an error of that
    request only."""
    from gee_workloads.configs import random_small_graph

    base = [random_small_graph(70 + i, N=3000 + 500 * i, E=40_000, K=6, weighted=bool(i % 2)) for i in range(2)]
    be = GpuBackend(slots=2)
    srv = GeeServer(be, 1 << 32, max_batch=6)
    for i, g in enumerate(base):
        s, d, w, _ = graph_tensors(g)
        srv.hold(be.make_resident(f"g{i}", s, d, w, g.N, flags(g)))
    rng = np.random.default_rng(5)
    reqs, ref_graphs = [], []
    edge_pool = [serving_one(g, e_max=50_000) for g in range(3)]
    for i in range(12):
        if i % 3 == 2:
            x = edge_pool[i % 3]
            s, d, w, lab = graph_tensors(x)
            reqs.append(Request(i, dict(src=s, dst=d, w=w, labels=lab, K=x.K, flags=flags(x)), 1e-4 * i))
            ref_graphs.append(x)
        else:
            b = base[i % 2]
            K = int(rng.integers(2, 40))
            lab = rng.integers(-1, K, size=b.N).astype(np.int32)
            opts = tuple(bool(v) for v in rng.random(3) < 0.5)
            x = type(b)(src=b.src, dst=b.dst, w=b.w, N=b.N, labels=lab, K=K, sym=b.sym).with_options(*opts)
            reqs.append(Request(i, dict(resident=f"g{i % 2}", labels=torch.from_numpy(lab).cuda(), K=K,
                                        flags=flags(x)), 1e-4 * i))
            ref_graphs.append(x)
    reqs.append(Request(99, dict(resident="nope", labels=reqs[0].graph["labels"], K=3, flags=0), 0.0))
    print(f"[gpu-test] serving re-embedding requests: {len(reqs)}", flush=True)
    srv.run_trace(reqs, busy_poll=True)
    torch.cuda.synchronize()
    assert reqs[-1].error is not None and reqs[-1].result is None
    assert any(len(b) > 1 for b in srv.launch_log)
    for i, (r, x) in enumerate(zip(reqs[:-1], ref_graphs)):
        assert r.error is None, f"request {i}: {r.error}"
        g = r.graph
        if "resident" in g:
            res = be.resident[g["resident"]]
            alone = gee.gee_embed_csr(res["rp"], res["col"], res["val"], res["M"], g["labels"], g["K"],
                                      g["flags"] & ~gee.GEE_SYMMETRIZE)
            torch.cuda.synchronize()
            assert torch.equal(r.result, alone), f"re-embedding {i}"
        assert_close(r.result, or_embed_graph(x), f"request {i} vs oracle")


def test_served_through_batch_plans_equals_alone():
    """The backend's plan mode: every batch of a slot goes through that slot's batch plan
    (gee_batch_plan_update, then a graph launch); results equal the plain calls bitwise."""
    gs, dev = _pool(12, 200_000)
    print("[gpu-test] serving through batch plans", flush=True)
    be = GpuBackend(slots=2, use_plans=True, plan_reserve=64 << 20)
    srv = GeeServer(be, 1 << 34, max_batch=5)
    rng = np.random.default_rng(3)
    reqs = [Request(i, d, float(a)) for i, (d, a) in enumerate(zip(dev + dev, np.cumsum(rng.exponential(2e-4, 24))))]
    srv.run_trace(reqs, busy_poll=True)
    torch.cuda.synchronize()
    assert any(len(b) > 1 for b in srv.launch_log)
    for i, r in enumerate(reqs):
        d = r.graph
        assert r.error is None
        alone = gee.gee_embed(d["src"], d["dst"], d["w"], d["labels"], d["K"], d["flags"])
        torch.cuda.synchronize()
        assert torch.equal(r.result, alone), f"request {i}"
