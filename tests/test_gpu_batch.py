"""Batched form through the C ABI (needs an MI355X): many graphs in one launch sequence
and in a captured batch plan. Bars: every graph's Z bitwise equal to its plain call with
the same schedule, and within tolerance of the FP64 oracle."""

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from gee_workloads.configs import batched_one, random_small_graph
from gee_workloads.generators import Graph
from oracle import embed_graph as or_embed_graph

from gpu_util import DEV, assert_close, flags, graph_tensors

pytestmark = pytest.mark.gpu


def _label(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _mixed_graphs(n, seed=0):
    """Uneven graphs: sizes from tiny to tens of thousands of edges, K from 1 to 128
    (both sides of 64), weighted and unweighted, symmetrized and directed, random options,
    isolated nodes, an edge-free graph."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.integers(1, 6000)) if i % 7 else int(rng.integers(1, 40))
        E = int(rng.integers(0, 8 * N + 1)) if i % 11 else 0
        K = int(rng.choice([1, 2, 3, 7, 31, 50, 64, 65, 100, 128]))
        g = random_small_graph(1000 + 37 * seed + i, N=N, E=E, K=K, weighted=bool(rng.random() < 0.7),
                               sym=bool(rng.random() < 0.8), unknown_frac=float(rng.uniform(0, 0.2)))
        d, l, c = (bool(x) for x in rng.random(3) < 0.5)
        out.append(g.with_options(d, l, c))
    return out


def _dev_graphs(gs, scheds=None):
    items = []
    for i, g in enumerate(gs):
        s, d, w, lab = graph_tensors(g)
        items.append(dict(src=s, dst=d, w=w, labels=lab, K=g.K, flags=flags(g),
                          Z=torch.full((g.N, g.K), float("nan"), dtype=torch.float32, device=DEV),
                          sched=None if scheds is None else scheds[i]))
    return items


def _plain(items):
    out = []
    for it in items:
        out.append(gee.gee_embed(it["src"], it["dst"], it["w"], it["labels"], it["K"], it["flags"],
                                 sched=it["sched"]))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_batch_matches_plain_bitwise(seed):
    gs = _mixed_graphs(40, seed)
    rng = np.random.default_rng(seed)
    scheds = [None if rng.random() < 0.5 else dict(wave_entries=int(rng.choice([256, 512, 2048])))
              for _ in gs]
    _label(f"batch of {len(gs)} mixed graphs seed={seed}")
    items = _dev_graphs(gs, scheds)
    gee.gee_embed_batch(items)
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() == 0
    plain = _plain(items)
    for i, (it, zp) in enumerate(zip(items, plain)):
        assert torch.equal(it["Z"], zp), f"graph {i} (N={gs[i].N}, E={gs[i].E}, K={gs[i].K})"
    for i in range(0, len(gs), 5):
        assert_close(items[i]["Z"], or_embed_graph(gs[i]), f"graph {i} vs oracle")


def test_batch_plan_replays():
    """A captured plan replayed several times, with eager work and new input contents in
    between; every replay equals the eager result for the inputs at that time."""
    gs = _mixed_graphs(24, 5)
    _label("batch plan replays")
    items = _dev_graphs(gs)
    plan = gee.BatchPlan(items)
    rng = np.random.default_rng(9)
    for rep in range(4):
        if rep >= 2:  # new labels in place: the plan reads current contents
            for it, g in zip(items, gs):
                lab = rng.integers(-1, g.K, size=g.N).astype(np.int32)
                it["labels"].copy_(torch.from_numpy(lab))
        for it in items:
            it["Z"].fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        eager = _plain(items)
        for i, (it, zp) in enumerate(zip(items, eager)):
            assert torch.equal(it["Z"], zp), f"replay {rep} graph {i}"
        _ = torch.randn(1000, device=DEV).sum().item()  # unrelated eager work between replays
    plan.destroy()


def test_batch_plan_update_to_other_graph_sets():
    """One plan replayed over three different graph sets (other sizes, classes, options and
    counts; the second set changes the launch sequence, the third keeps it): after every
    update the replay equals the plain calls bit for bit and the oracle within tolerance.
    A set that needs more workspace than the plan holds is refused and leaves the plan as
    it was."""
    sets = [_mixed_graphs(12, 21), _mixed_graphs(30, 22), _mixed_graphs(12, 23)]
    big = max(gee.gee_embed_batch_workspace_bytes(_dev_graphs(gs)) for gs in sets)
    _label(f"batch plan update over 3 graph sets (workspace {big} bytes)")
    first = _dev_graphs(sets[0])
    plan = gee.BatchPlan(first, workspace_bytes=big)
    assert plan.workspace_bytes >= big
    for k, gs in enumerate(sets):
        items = first if k == 0 else _dev_graphs(gs)
        if k > 0:
            plan.update(items)
        for rep in range(2):
            for it in items:
                it["Z"].fill_(float("nan"))
            plan.launch()
            torch.cuda.synchronize()
            assert gee.gee_get_data_errors() == 0
            plain = _plain(items)
            for i, (it, zp) in enumerate(zip(items, plain)):
                assert torch.equal(it["Z"], zp), f"set {k} replay {rep} graph {i}"
        for i in range(0, len(gs), 4):
            assert_close(items[i]["Z"], or_embed_graph(gs[i]), f"set {k} graph {i} vs oracle")
    # too large for the plan: refused, and the plan still embeds its last set
    huge = [random_small_graph(900, N=200_000, E=2_000_000, K=64, weighted=True, sym=True)
            .with_options(True, True, True)]
    hi = _dev_graphs(huge)
    assert gee.gee_embed_batch_workspace_bytes(hi) > plan.workspace_bytes
    with pytest.raises(gee.GeeError) as ei:
        plan.update(hi)
    assert ei.value.code == gee.GEE_ERR_WORKSPACE
    for it in items:
        it["Z"].fill_(float("nan"))
    plan.launch()
    torch.cuda.synchronize()
    for i, (it, zp) in enumerate(zip(items, _plain(items))):
        assert torch.equal(it["Z"], zp), f"after a refused update, graph {i}"
    plan.destroy()


def test_batch_plan_update_reports_data_errors_of_the_new_set():
    g = random_small_graph(31, N=300, E=2000, K=4).with_options(True, True, True)
    bad = random_small_graph(32, N=200, E=800, K=3)
    bad.labels[11] = 7
    items = _dev_graphs([g, g])
    plan = gee.BatchPlan(items, workspace_bytes=1 << 24)
    plan.launch()
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() == 0
    plan.update(_dev_graphs([g, bad]))
    plan.launch()
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() & gee.GEE_DATA_LABEL
    plan.destroy()


def test_batch_all_512_recipe_graphs_vs_oracle():
    """Every graph of the 512-graph batched workload (about 232M edges), embedded in one
    batch plan, against the FP64 oracle; a sample also against its plain call bitwise."""
    import multiprocessing as mp

    with mp.get_context("spawn").Pool(min(16, mp.cpu_count())) as pool:
        gs = pool.map(batched_one, range(512), chunksize=4)
    _label(f"all 512 batched graphs: {sum(g.E for g in gs)} edges")
    items = _dev_graphs(gs)
    plan = gee.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() == 0
    plan.destroy()
    worst = 0.0
    for i, (it, g) in enumerate(zip(items, gs)):
        worst = max(worst, assert_close(it["Z"], or_embed_graph(g), f"graph {i}"))
    _label(f"all 512 batched graphs: max relative error {worst:.3e}")
    sample = items[::37]
    for i, (it, zp) in enumerate(zip(sample, _plain(sample))):
        assert torch.equal(it["Z"], zp), f"sample {i}"


def test_batch_recipe_sample():
    """Graphs of the 512-graph batched workload recipe (a sample of them), batched vs plain
    bitwise and vs the oracle."""
    gs = [batched_one(g) for g in range(0, 512, 16)]
    _label(f"batched recipe sample of {len(gs)}")
    items = _dev_graphs(gs)
    gee.gee_embed_batch(items)
    torch.cuda.synchronize()
    plain = _plain(items)
    for i, (it, zp) in enumerate(zip(items, plain)):
        assert torch.equal(it["Z"], zp), f"graph {i}"
    for i in range(0, len(gs), 4):
        assert_close(items[i]["Z"], or_embed_graph(gs[i]), f"graph {i} vs oracle")


def test_batch_single_and_errors():
    g = random_small_graph(3, N=500, E=3000, K=5).with_options(True, True, True)
    items = _dev_graphs([g])
    gee.gee_embed_batch(items)
    torch.cuda.synchronize()
    assert_close(items[0]["Z"], or_embed_graph(g), "batch of one")
    # a bad label in one graph raises the shared data-error bit
    bad = random_small_graph(4, N=100, E=300, K=3)
    bad.labels[7] = 5
    items = _dev_graphs([g, bad])
    gee.gee_embed_batch(items)
    assert gee.gee_get_data_errors() & gee.GEE_DATA_LABEL
    # an empty graph list entry with N = 0 and E = 0 is accepted
    empty = Graph(src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32), w=None, N=0,
                  labels=np.zeros(0, np.int32), K=2)
    items = _dev_graphs([g, empty, g])
    gee.gee_embed_batch(items)
    torch.cuda.synchronize()
    assert torch.equal(items[0]["Z"], items[2]["Z"])


def test_batch_beyond_one_bucket_size_keeps_plain_bits():
    """A batch of more than 2^21 rows (one graph alone above it): every graph still takes
    the bucket size it takes alone, so batched, planned and plain Z agree bit for bit."""
    sizes = [(700_000, 1_400_000, 8), (2_300_000, 3_000_000, 5), (900_000, 1_000_000, 12),
             (600_000, 900_000, 3), (50, 120, 2)]
    gs = [random_small_graph(500 + i, N=N, E=E, K=K, weighted=bool(i % 2), sym=True).with_options(True, True, True)
          for i, (N, E, K) in enumerate(sizes)]
    _label(f"batch beyond 2^21 rows: {sum(g.N for g in gs)} rows")
    items = _dev_graphs(gs)
    gee.gee_embed_batch(items)
    torch.cuda.synchronize()
    plain = _plain(items)
    for i, (it, zp) in enumerate(zip(items, plain)):
        assert torch.equal(it["Z"], zp), f"graph {i} (N={gs[i].N})"
    plan = gee.BatchPlan(items)
    for it in items:
        it["Z"].fill_(float("nan"))
    plan.launch()
    torch.cuda.synchronize()
    for i, (it, zp) in enumerate(zip(items, plain)):
        assert torch.equal(it["Z"], zp), f"planned graph {i}"
    plan.destroy()
    assert_close(items[4]["Z"], or_embed_graph(gs[4]), "small graph vs oracle")
    assert_close(items[3]["Z"], or_embed_graph(gs[3]), "600k-row graph vs oracle")


def test_path_routing_beyond_bucket_limits():
    """gee_embed of a graph above 2^22 rows (the CSR path) and of a graph with K > 64 above
    2^21 rows (64-row buckets with a 100-float class stride), alone and batched with a small
    graph: vs the oracle, and batched equal to plain bit for bit."""
    gs = [random_small_graph(700, N=4_300_000, E=250_000, K=3, weighted=True, sym=True).with_options(True, True, True),
          random_small_graph(701, N=2_200_000, E=300_000, K=100, weighted=False, sym=True).with_options(False, True, True),
          random_small_graph(702, N=3000, E=20_000, K=100, weighted=True, sym=False).with_options(True, False, True)]
    _label("path routing: 4.3M rows K=3, 2.2M rows K=100, small K=100")
    items = _dev_graphs(gs)
    plain = _plain(items)
    for i in range(3):
        assert_close(plain[i], or_embed_graph(gs[i]), f"graph {i} alone vs oracle")
    gee.gee_embed_batch(items)
    torch.cuda.synchronize()
    for i, (it, zp) in enumerate(zip(items, plain)):
        assert torch.equal(it["Z"], zp), f"graph {i}"
