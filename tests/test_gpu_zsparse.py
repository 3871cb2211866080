"""Z in sparse storage (gee_embed_sparse) against the oracle's sparse storage of its FP64 Z,
through the C ABI (needs an MI355X).

Bars: row_ptr and the class indices bit-exact (the zero pattern of Z is exact on every
path); values within 1e-5 relative of the oracle, and bitwise equal to what gee_embed
writes into a dense Z for the same graph."""

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from gee_workloads import powerlaw_10m, random_small_graph, sbm_small
from gee_workloads.generators import Graph
from oracle import embed_graph as or_embed_graph
from oracle import sparse_rows

from gpu_util import RTOL, flags, graph_tensors

pytestmark = pytest.mark.gpu


def _label(msg):
    print(f"[gpu-test] {msg}", flush=True)


def check_sparse(g, capacity=None):
    s, d, w, lab = graph_tensors(g)
    rp, col, val = gee.gee_embed_sparse(s, d, w, lab, g.K, flags(g), capacity=capacity)
    Zd = gee.gee_embed(s, d, w, lab, g.K, flags(g))
    torch.cuda.synchronize()
    rrp, rcol, rval = sparse_rows(or_embed_graph(g))
    rp = rp.cpu().numpy()
    nnz = int(rp[-1])
    assert np.array_equal(rp, rrp), "row_ptr"
    n = nnz if capacity is None else min(nnz, capacity)
    col = col[:n].cpu().numpy() if n else np.zeros(0, np.int32)
    val = val[:n].cpu().numpy() if n else np.zeros(0, np.float32)
    assert np.array_equal(col, rcol[:n]), "class indices"
    if n:
        rel = np.max(np.abs(val.astype(np.float64) - rval[:n]) / np.abs(rval[:n]))
        assert rel <= RTOL, rel
        rows = np.repeat(np.arange(g.N), np.diff(rp))[:n]
        dense_vals = Zd.cpu().numpy()[rows, col]
        assert np.array_equal(val.view(np.uint32), dense_vals.view(np.uint32)), "values differ from gee_embed"
    return nnz


@pytest.mark.parametrize("K", [1, 2, 3, 5, 9, 17, 33, 50, 64, 65, 128])
def test_sparse_class_counts_range(K):
    # 5,003 rows: nineteen 256-row tiles and a ragged last one
    g = random_small_graph(K, N=5003, E=20_000, K=K, weighted=True, unknown_frac=0.1)
    for opts in ((False, False, False), (True, True, True)):
        _label(f"sparse Z K={K} opts={opts}")
        check_sparse(g.with_options(*opts))


@pytest.mark.parametrize("sym", [True, False])
def test_sparse_all_options(sym):
    g = random_small_graph(7, N=2500, E=30_000, K=6, weighted=True, sym=sym, unknown_frac=0.1)
    for d in (False, True):
        for l in (False, True):
            for c in (False, True):
                _label(f"sparse Z sym={sym} opts={(d, l, c)}")
                check_sparse(g.with_options(d, l, c))


@pytest.mark.parametrize("K", [7, 40])
def test_sparse_capacity_short_and_zero(K):
    # K = 7: a dense Z compacted afterwards; K = 40: the non-zero pairs staged per bucket by
    # the class scatter (used when the staging is at most twice a dense Z's size)
    g = random_small_graph(2, N=3000, E=9000, K=K, weighted=True).with_options(True, True, True)
    s, d, w, lab = graph_tensors(g)
    _label(f"sparse Z capacity K={K}")
    nnz = check_sparse(g)
    cap = nnz // 3
    check_sparse(g, capacity=cap)
    # nothing written past the capacity
    col = torch.full((nnz,), -5, dtype=torch.int32, device=s.device)
    val = torch.full((nnz,), 9.0, dtype=torch.float32, device=s.device)
    rp, _, _ = gee.gee_embed_sparse(s, d, w, lab, g.K, flags(g), capacity=cap, col=col, val=val)
    torch.cuda.synchronize()
    assert int(rp[-1].item()) == nnz
    assert bool((col[cap:] == -5).all()) and bool((val[cap:] == 9.0).all())
    # capacity 0: row pointers alone
    rp0, c0, v0 = gee.gee_embed_sparse(s, d, w, lab, g.K, flags(g), capacity=0)
    torch.cuda.synchronize()
    assert c0 is None and v0 is None and torch.equal(rp0, rp)


def test_sparse_edge_cases():
    _label("sparse Z edge cases")
    e0 = np.zeros(0, np.int32)
    lab = np.array([0, 1, -1, 1, 2, 0, 2], np.int32)
    for d in (False, True):
        g = Graph(src=e0, dst=e0, w=None, N=7, labels=lab, K=3, diag=d, lap=True, cor=True)
        assert check_sparse(g) == (6 if d else 0)
    g = Graph(src=np.array([0], np.int32), dst=np.array([0], np.int32), w=np.array([0.5], np.float32),
              N=1, labels=np.array([0], np.int32), K=1, diag=True, lap=True, cor=False)
    assert check_sparse(g) == 1
    g = random_small_graph(1, N=500, E=3000, K=4, unknown_frac=1.0).with_options(True, True, True)
    assert check_sparse(g) == 0  # all labels unknown: Z = 0


def test_sparse_sbm_small():
    for opt in ("off", "all"):
        g = sbm_small(opt)
        _label(f"sparse Z sbm N=2000 options={opt}")
        assert check_sparse(g) == g.N * g.K  # dense graph: every entry is non-zero


def test_sparse_powerlaw_10m_full():
    g = powerlaw_10m()
    _label(f"sparse Z powerlaw N={g.N} E={g.E} K={g.K}")
    nnz = check_sparse(g)
    _label(f"sparse Z powerlaw nnz={nnz} of {g.N * g.K}")
    assert gee.gee_get_data_errors() == 0


def test_sparse_powerlaw_k128_split_buckets():
    # K = 128: 32-row buckets; hub rows split buckets into several parts, whose combine stages
    # the pairs over all its wavefronts; 100,003 rows end in a ragged bucket and tile
    g = powerlaw_10m(N=100_003, E=800_000, K=128, dmax=20_000.0)
    _label(f"sparse Z powerlaw N={g.N} E={g.E} K={g.K}")
    check_sparse(g)
    check_sparse(g.with_options(False, False, False))


def test_sparse_nan_factor_rows_fill_every_class():
    # a NaN weight makes its rows' Laplacian and correlation factors NaN, so 0 * NaN fills
    # every class of those rows: the staged pairs (K = 40: staged by the class scatter) must
    # hold K pairs for such a row, and the sparse form must list exactly the dense Z's
    # non-zero entries (NaN is not zero), bit for bit
    g = random_small_graph(33, N=3000, E=20_000, K=40, weighted=True).with_options(True, True, True)
    g.w[17] = np.float32("nan")
    s, d, w, lab = graph_tensors(g)
    _label("sparse Z with a NaN weight, K=40")
    gee.gee_get_data_errors()
    rp, col, val = gee.gee_embed_sparse(s, d, w, lab, g.K, flags(g))
    Zd = gee.gee_embed(s, d, w, lab, g.K, flags(g))
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() & gee.GEE_DATA_WEIGHT
    Z = Zd.cpu().numpy()
    nzm = Z != 0.0  # (NaN compares unequal to zero: stored)
    assert np.isnan(Z).any()
    rp = rp.cpu().numpy()
    assert np.array_equal(np.diff(rp), nzm.sum(axis=1)), "row counts"
    nnz = int(rp[-1])
    rows, cls = np.nonzero(nzm)
    assert np.array_equal(col[:nnz].cpu().numpy(), cls.astype(np.int32)), "classes"
    assert np.array_equal(val[:nnz].cpu().numpy().view(np.uint32), Z[rows, cls].view(np.uint32)), "values"
