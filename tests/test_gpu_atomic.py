"""The original GEE form (gee_embed_atomic: one pass over the edge list, float atomics)
against the FP64 oracle, through the C ABI (needs an MI355X).

Its Z is not deterministic in the last bits, so every check is against the oracle at the
same bar as the sparse paths: max relative error 1e-5 on the oracle's non-zero entries and
exactly zero elsewhere. Weights are non-negative here (no cancellation)."""

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from gee_workloads import powerlaw_10m, random_small_graph, sbm_small
from gee_workloads.generators import Graph
from oracle import embed_graph as or_embed_graph

from gpu_util import assert_close, flags, graph_tensors, max_rel_error

pytestmark = pytest.mark.gpu

FLAG_COMBOS = [(d, l, c) for d in (False, True) for l in (False, True) for c in (False, True)]


def _label(msg):
    print(f"[gpu-test] {msg}", flush=True)


def embed_atomic(g):
    s, d, w, lab = graph_tensors(g)
    Z = gee.gee_embed_atomic(s, d, w, lab, g.K, flags(g))
    torch.cuda.synchronize()
    return Z


@pytest.mark.parametrize("seed", range(2))
@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("weighted", [True, False])
def test_atomic_random_all_options(seed, sym, weighted):
    base = random_small_graph(seed, N=2500, E=30_000, K=5, weighted=weighted, sym=sym, unknown_frac=0.1)
    for d, l, c in FLAG_COMBOS:
        g = base.with_options(d, l, c)
        _label(f"atomic random seed={seed} sym={sym} w={weighted} opts={(d, l, c)}")
        assert_close(embed_atomic(g), or_embed_graph(g), f"opts={(d, l, c)}")


# K around every lane-group width of the row finish (1, 2, 4, ..., 64 lanes, two columns
# per lane above 64)
@pytest.mark.parametrize("K", [1, 2, 3, 5, 9, 17, 33, 50, 64, 65, 128])
def test_atomic_class_counts_range(K):
    g = random_small_graph(K, N=4000, E=60_000, K=K, weighted=True, unknown_frac=0.05)
    for opts in ((True, True, True), (False, False, False), (False, False, True)):
        gg = g.with_options(*opts)
        _label(f"atomic K={K} opts={opts}")
        assert_close(embed_atomic(gg), or_embed_graph(gg), f"K={K} opts={opts}")


@pytest.mark.parametrize("N,K", [(96, 128), (1500, 5), (4096, 3), (4097, 3), (12288, 1), (12289, 1)])
def test_atomic_small_graphs(N, K):
    """Small graphs with many edge rows per node (contended degree and Z atomics)."""
    base = random_small_graph(N + K, N=N, E=8 * N, K=K, weighted=True, unknown_frac=0.1)
    for d, l, c in FLAG_COMBOS:
        g = base.with_options(d, l, c)
        _label(f"atomic small N={N} K={K} opts={(d, l, c)}")
        assert_close(embed_atomic(g), or_embed_graph(g), f"N={N} K={K} opts={(d, l, c)}")


def test_atomic_small_graph_dense():
    """800 nodes, 400k edge rows: every degree and Z word takes hundreds of atomics."""
    g = random_small_graph(11, N=800, E=400_000, K=4, weighted=True, unknown_frac=0.05)
    for opts in ((False, False, False), (True, True, True)):
        gg = g.with_options(*opts)
        _label(f"atomic small many parts opts={opts}")
        assert_close(embed_atomic(gg), or_embed_graph(gg), f"opts={opts}")


def test_atomic_edge_cases():
    _label("atomic edge cases")
    e0 = np.zeros(0, np.int32)
    lab = np.array([0, 1, -1, 1, 2, 0, 2], np.int32)
    for d, l, c in FLAG_COMBOS:
        g = Graph(src=e0, dst=e0, w=None, N=7, labels=lab, K=3, diag=d, lap=l, cor=c)
        assert_close(embed_atomic(g), or_embed_graph(g), f"empty {(d, l, c)}")
    g = Graph(src=np.array([0], np.int32), dst=np.array([0], np.int32), w=np.array([0.5], np.float32),
              N=1, labels=np.array([0], np.int32), K=1, diag=True, lap=True, cor=False)
    assert_close(embed_atomic(g), or_embed_graph(g), "single node")
    g = random_small_graph(1, N=500, E=3000, K=4, unknown_frac=1.0).with_options(True, True, True)
    assert_close(embed_atomic(g), or_embed_graph(g), "all unknown")
    g = random_small_graph(2, N=20_000, E=2000, K=6, unknown_frac=0.0)
    g.labels[g.labels == 3] = 4  # an empty class, many isolated nodes
    for d, l, c in FLAG_COMBOS:
        gg = g.with_options(d, l, c)
        assert_close(embed_atomic(gg), or_embed_graph(gg), f"isolated {(d, l, c)}")


def test_atomic_unaligned_output():
    """Z starting 4 bytes past a 16-byte boundary, with N*K not a multiple of 4: the
    zeroing pass's scalar head and tail."""
    g = random_small_graph(3, N=1001, E=8000, K=7, weighted=True).with_options(True, True, True)
    s, d, w, lab = graph_tensors(g)
    buf = torch.full((g.N * g.K + 8,), 7.0, dtype=torch.float32, device=s.device)
    Z = buf[1:1 + g.N * g.K]
    gee.gee_embed_atomic(s, d, w, lab, g.K, flags(g), Z=Z)
    torch.cuda.synchronize()
    assert_close(Z, or_embed_graph(g), "unaligned Z")
    assert float(buf[0].item()) == 7.0 and bool((buf[1 + g.N * g.K:] == 7.0).all())


def test_atomic_hub_star():
    """A hub row with 120k entries (atomic contention on one Z row and one degree)."""
    rng = np.random.default_rng(0)
    hub, K, extra = 120_000, 5, 2000
    N = hub + 1
    src = np.concatenate([np.zeros(hub, np.int32), rng.integers(0, N, extra).astype(np.int32)])
    dst = np.concatenate([np.arange(1, N, dtype=np.int32), rng.integers(0, N, extra).astype(np.int32)])
    w = (1.0 - rng.random(src.size, dtype=np.float32)).astype(np.float32)
    lab = rng.integers(-1, K, size=N).astype(np.int32)
    g = Graph(src=src, dst=dst, w=w, N=N, labels=lab, K=K, diag=True, lap=True, cor=True)
    _label("atomic hub star")
    assert_close(embed_atomic(g), or_embed_graph(g), "star")


def test_atomic_data_and_argument_errors():
    _label("atomic data errors")
    gee.gee_get_data_errors()  # clear
    g = random_small_graph(0, N=100, E=500, K=3).with_options(True, True, True)
    s, d, w, lab = graph_tensors(g)
    bad_lab = lab.clone()
    bad_lab[5] = 7
    gee.gee_embed_atomic(s, d, w, bad_lab, 3, flags(g))
    assert gee.gee_get_data_errors() & gee.GEE_DATA_LABEL
    bad_d = d.clone()
    bad_d[3] = 100
    gee.gee_embed_atomic(s, bad_d, w, lab, 3, flags(g))
    assert gee.gee_get_data_errors() & gee.GEE_DATA_INDEX
    bad_w = w.clone()
    bad_w[2] = float("inf")
    gee.gee_embed_atomic(s, d, bad_w, lab, 3, flags(g))
    assert gee.gee_get_data_errors() & gee.GEE_DATA_WEIGHT
    gee.gee_embed_atomic(s, d, w, lab, 3, flags(g))
    assert gee.gee_get_data_errors() == 0
    for K, fl in ((0, flags(g)), (129, flags(g)), (3, 1 << 9)):
        with pytest.raises(gee.GeeError):
            gee.gee_embed_atomic(s, d, w, lab, K, fl)
    from paper_2406_03726_amd import _lib
    import ctypes

    small = torch.empty(16, dtype=torch.uint8, device=s.device)
    Z = torch.empty((g.N, 3), dtype=torch.float32, device=s.device)
    rc = _lib.load().gee_embed_atomic_ws(ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()),
                                         ctypes.c_void_p(w.data_ptr()), g.E, g.N,
                                         ctypes.c_void_p(lab.data_ptr()), 3, flags(g),
                                         ctypes.c_void_p(Z.data_ptr()), ctypes.c_void_p(small.data_ptr()),
                                         16, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -9  # GEE_ERR_WORKSPACE, nothing enqueued


def test_atomic_sbm_small_both_option_sets():
    for opt in ("off", "all"):
        g = sbm_small(opt)
        _label(f"atomic sbm N=2000 options={opt}")
        assert_close(embed_atomic(g), or_embed_graph(g), f"sbm_small {opt}")


def test_atomic_powerlaw_10m_full_matches_oracle_and_sparse_path():
    """The 10M-edge power-law workload at full size, all options: against the oracle, and
    against the deterministic bucket path (gee_embed) on the same input."""
    g = powerlaw_10m()
    _label(f"atomic powerlaw N={g.N} E={g.E} K={g.K}")
    s, d, w, lab = graph_tensors(g)
    Z = gee.gee_embed_atomic(s, d, w, lab, g.K, flags(g))
    Zs = gee.gee_embed(s, d, w, lab, g.K, flags(g))
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() == 0
    R = or_embed_graph(g)
    rel = assert_close(Z, R, "powerlaw_10m atomic")
    _label(f"atomic powerlaw max rel error {rel:.3e}")
    nz = Zs != 0
    assert torch.equal(Z != 0, nz)
    assert float(((Z - Zs).abs()[nz] / Zs.abs()[nz]).max().item()) <= 2e-5
    # a second call: same result within the bar (the last bits may differ)
    Z2 = gee.gee_embed_atomic(s, d, w, lab, g.K, flags(g))
    torch.cuda.synchronize()
    rel2, zero_ok = max_rel_error(Z2, R)
    assert zero_ok and rel2 <= 1e-5
