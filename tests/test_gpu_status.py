"""Data-error words per stream, GEE_NO_VALIDATE, and stream-ordered allocations in the
binding (needs an MI355X). Results are checked against the FP64 oracle."""

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from gee_workloads.configs import random_small_graph
from oracle import embed_graph as or_embed_graph

from gpu_util import DEV, assert_close, flags, graph_tensors

pytestmark = pytest.mark.gpu


def _label(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _graph(seed=11):
    return random_small_graph(seed, N=600, E=4000, K=5).with_options(True, True, True)


def test_errors_are_reported_on_their_own_stream():
    _label("data-error words per stream")
    g = _graph()
    s, d, w, lab = graph_tensors(g)
    bad = lab.clone()
    bad[17] = g.K + 3
    bad_d = d.clone()
    bad_d[5] = g.N + 1
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    for st in (s1, s2, s3):
        st.wait_stream(torch.cuda.current_stream())
        gee.gee_get_data_errors(st)  # start clean
    Z1 = gee.gee_embed(s, d, w, lab, g.K, flags(g), stream=s1)
    gee.gee_embed(s, d, w, bad, g.K, flags(g), stream=s2)
    gee.gee_embed(s, bad_d, w, lab, g.K, flags(g), stream=s3)
    assert gee.gee_get_data_errors(s1) == 0
    assert gee.gee_get_data_errors(s2) == gee.GEE_DATA_LABEL
    assert gee.gee_get_data_errors(s3) == gee.GEE_DATA_INDEX
    # reading takes the bits
    assert gee.gee_get_data_errors(s2) == 0 and gee.gee_get_data_errors(s3) == 0
    torch.cuda.synchronize()
    assert_close(Z1, or_embed_graph(g), "good stream")
    # the other entry points report on their stream too
    gee.gee_embed_atomic(s, d, w, bad, g.K, flags(g), stream=s1)
    rp, col, val = gee.gee_build_csr(s, d, w, g.N, flags(g), stream=s2)
    assert gee.gee_get_data_errors(s1) == gee.GEE_DATA_LABEL
    assert gee.gee_get_data_errors(s2) == 0
    M = int(rp[-1].item())
    gee.gee_embed_csr(rp, col, val, M, bad, g.K, flags(g), stream=s3)
    assert gee.gee_get_data_errors(s3) == gee.GEE_DATA_LABEL
    assert gee.gee_get_data_errors(s1) == 0 and gee.gee_get_data_errors(s2) == 0


def test_batch_plan_reports_on_its_launch_stream():
    _label("batch plan data errors")
    g = _graph(12)
    bad = random_small_graph(13, N=100, E=300, K=3)
    bad.labels[7] = 5
    items = []
    for x in (g, bad):
        s, d, w, lab = graph_tensors(x)
        items.append(dict(src=s, dst=d, w=w, labels=lab, K=x.K, flags=flags(x),
                          Z=torch.empty((x.N, x.K), dtype=torch.float32, device=DEV)))
    plan = gee.BatchPlan(items)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for st in (s1, s2):
        st.wait_stream(torch.cuda.current_stream())
        gee.gee_get_data_errors(st)
    plan.launch(stream=s1)
    assert gee.gee_get_data_errors(s1) == gee.GEE_DATA_LABEL
    assert gee.gee_get_data_errors(s2) == 0
    plan.launch(stream=s2)
    assert gee.gee_get_data_errors(s2) == gee.GEE_DATA_LABEL
    assert gee.gee_get_data_errors(s1) == 0
    plan.destroy()
    torch.cuda.synchronize()
    assert_close(items[0]["Z"], or_embed_graph(g), "good graph of the plan")


def test_no_validate():
    _label("GEE_NO_VALIDATE")
    g = _graph(14)
    s, d, w, lab = graph_tensors(g)
    gee.gee_get_data_errors()
    Z0 = gee.gee_embed(s, d, w, lab, g.K, flags(g))
    Z1 = gee.gee_embed(s, d, w, lab, g.K, flags(g) | gee.GEE_NO_VALIDATE)
    torch.cuda.synchronize()
    assert torch.equal(Z0, Z1)
    bad = lab.clone()
    bad[3] = g.K
    bad_w = w.clone()
    bad_w[2] = float("inf")
    gee.gee_embed(s, d, w, bad, g.K, flags(g) | gee.GEE_NO_VALIDATE)
    gee.gee_embed(s, d, bad_w, lab, g.K, flags(g) | gee.GEE_NO_VALIDATE)
    gee.gee_embed_atomic(s, d, w, bad, g.K, flags(g) | gee.GEE_NO_VALIDATE)
    assert gee.gee_get_data_errors() == 0
    gee.gee_embed(s, d, w, bad, g.K, flags(g))
    assert gee.gee_get_data_errors() == gee.GEE_DATA_LABEL


def test_call_on_a_side_stream_keeps_its_workspace():
    """gee_embed on a stream that is not the current one, then at once allocations and
    writes on the current stream: the call's workspace and Z must not be handed out under
    its kernels (the result still matches the oracle)."""
    _label("side-stream allocation")
    from gee_workloads import powerlaw_10m

    g = powerlaw_10m(N=60_000, E=1_000_000, K=20, dmax=8000.0)
    s, d, w, lab = graph_tensors(g)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):
        Z = gee.gee_embed(s, d, w, lab, g.K, flags(g), stream=side)
        outs.append(Z)
        # fill whatever memory the current stream can get right now
        junk = [torch.full((1 << 22,), float(i), device=DEV) for i in range(16)]
        del junk
    side.synchronize()
    torch.cuda.synchronize()
    R = or_embed_graph(g)
    for Z in outs:
        assert_close(Z, R, "side stream")


def test_served_request_errors_are_per_request():
    """A batch of served requests where one carries a bad label: only that request gets an
    error; the others get results equal to their plain calls."""
    _label("serving: per-request errors")
    from paper_2406_03726_amd.serve import GeeServer, GpuBackend, Request

    gs = [random_small_graph(40 + i, N=300 + 40 * i, E=2000, K=4).with_options(True, i % 2 == 0, True)
          for i in range(6)]
    reqs = []
    for i, x in enumerate(gs):
        s, d, w, lab = graph_tensors(x)
        if i == 3:
            lab = lab.clone()
            lab[0] = -7
        reqs.append(Request(i, dict(src=s, dst=d, w=w, labels=lab, K=x.K, flags=flags(x)), 0.0))
    be = GpuBackend(slots=1)
    srv = GeeServer(be, 1 << 30, max_batch=8)
    srv.run_trace(reqs)
    torch.cuda.synchronize()
    assert any(len(b) > 1 for b in srv.launch_log)
    for i, r in enumerate(reqs):
        if i == 3:
            assert r.error is not None and r.result is None
        else:
            assert r.error is None
            assert_close(r.result, or_embed_graph(gs[i]), f"request {i}")


def test_take_data_errors_async_into_pinned_memory():
    """The stream-ordered take without a wait: the bits land in pinned host memory once the
    stream passes the take, per stream, and the word is cleared."""
    _label("async data-error take")
    g = _graph(21)
    s, d, w, lab = graph_tensors(g)
    bad = lab.clone()
    bad[3] = g.K
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for st in (s1, s2):
        st.wait_stream(torch.cuda.current_stream())
        gee.gee_get_data_errors(st)
    h1 = torch.full((1,), -1, dtype=torch.int32, pin_memory=True)
    h2 = torch.full((1,), -1, dtype=torch.int32, pin_memory=True)
    gee.gee_embed(s, d, w, lab, g.K, flags(g), stream=s1)
    gee.gee_embed(s, d, w, bad, g.K, flags(g), stream=s2)
    gee.gee_take_data_errors_async(h1, stream=s1)
    gee.gee_take_data_errors_async(h2, stream=s2)
    e1, e2 = torch.cuda.Event(), torch.cuda.Event()
    e1.record(s1)
    e2.record(s2)
    e1.synchronize()
    e2.synchronize()
    assert int(h1[0]) == 0
    assert int(h2[0]) == gee.GEE_DATA_LABEL
    assert gee.gee_get_data_errors(s2) == 0  # the take cleared the word
    # into device memory too
    dv = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    gee.gee_embed(s, d, w, bad, g.K, flags(g), stream=s1)
    gee.gee_take_data_errors_async(dv, stream=s1)
    s1.synchronize()
    assert int(dv.item()) == gee.GEE_DATA_LABEL
    with pytest.raises(ValueError):
        gee.gee_take_data_errors_async(torch.zeros(1, dtype=torch.int32))  # pageable host memory
