"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Bars: class counts and CSR bit-exact; Z within 1e-5 max relative error on the oracle's
non-zero entries and exactly zero elsewhere (row-normwise for signed weights); repeated
calls bitwise identical.
"""

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from gee_workloads import powerlaw_10m, random_small_graph, sbm_dense, sbm_small
from gee_workloads.generators import Graph
from oracle import class_counts as or_counts
from oracle import csr as or_csr
from oracle import embed as or_embed
from oracle import embed_graph as or_embed_graph

from gpu_util import assert_close, embed_graph, flags, graph_tensors, to_dev

pytestmark = pytest.mark.gpu

FLAG_COMBOS = [(d, l, c) for d in (False, True) for l in (False, True) for c in (False, True)]


def _label(msg):
    print(f"[gpu-test] {msg}", flush=True)


# ----------------------------------------------------------------------------- counts

@pytest.mark.parametrize("N,K", [(1, 1), (1000, 3), (70_001, 50), (300_000, 128), (5000, 1)])
def test_class_counts_bit_exact(N, K):
    _label(f"class counts N={N} K={K}")
    rng = np.random.default_rng(N + K)
    lab = rng.integers(-1, K, size=N).astype(np.int32)
    c = gee.gee_class_counts(to_dev(lab, torch.int32), K)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy().astype(np.int64), or_counts(lab, K))


# ----------------------------------------------------------------------------- CSR

def _check_csr(g, sched=None):
    s, d, w, _ = graph_tensors(g)
    rp, col, val = gee.gee_build_csr(s, d, w, g.N, gee.flags_of(sym=g.sym), sched=sched)
    torch.cuda.synchronize()
    rrp, rcol, rval = or_csr(g.src, g.dst, g.w, g.N, sym=g.sym)
    M = int(rrp[-1])
    assert np.array_equal(rp.cpu().numpy(), rrp), "row_ptr"
    assert np.array_equal(col[:M].cpu().numpy(), rcol), "col"
    if g.w is not None:
        assert np.array_equal(val[:M].cpu().numpy().view(np.uint32), rval.view(np.uint32)), "val bits"


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("weighted", [True, False])
def test_csr_random_bit_exact(seed, sym, weighted):
    # several pass-1 tiles (16384 entries) and a ragged tail; self-loops and repeats
    g = random_small_graph(seed, N=3000 + 17 * seed, E=50_003 + seed, K=3, weighted=weighted, sym=sym)
    _label(f"csr random seed={seed} sym={sym} weighted={weighted} E={g.E}")
    _check_csr(g)


def test_csr_sbm_small_bit_exact():
    _label("csr sbm N=2000")
    _check_csr(sbm_small("off"))


# bucket sizes: 2 rows (10,000 buckets: both partition passes, tiny buckets), 4096 rows
# (5 buckets of ~48k entries: one partition pass, buckets too large to stage), 128 rows
# (157 staged buckets, one partition pass)
@pytest.mark.parametrize("sched", [dict(tile_entries=4096, bucket_rows_log2=1),
                                   dict(bucket_rows_log2=12),
                                   dict(bucket_rows_log2=7)])
def test_csr_schedules_bit_exact(sched):
    g = random_small_graph(9, N=20_000, E=120_000, K=3, weighted=True)
    _label(f"csr schedule {sched}")
    _check_csr(g, sched=sched)


@pytest.mark.parametrize("sb", [3, 9])
def test_csr_two_partition_passes_with_hubs(sb):
    """Both partition passes (several hundred buckets and more) on a power-law graph whose
    hub rows make some buckets too large to stage."""
    g = powerlaw_10m(N=300_000, E=1_500_000, K=4, dmax=20_000.0)
    _label(f"csr power-law two passes sb={sb}")
    _check_csr(g, sched=dict(bucket_rows_log2=sb))


def test_csr_powerlaw_10m_full_bit_exact():
    """gee_build_csr of the 10M-edge power-law workload (20M entries, hub rows of tens of
    thousands of entries) in its default schedule, bit for bit against the stable sort."""
    g = powerlaw_10m()
    _label(f"csr powerlaw N={g.N} E={g.E}")
    _check_csr(g)


def test_csr_empty_and_isolated():
    _label("csr empty")
    g = Graph(src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32), w=None, N=7,
              labels=np.zeros(7, np.int32), K=1)
    _check_csr(g)


# ----------------------------------------------------------------------------- Z, small

@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("weighted", [True, False])
def test_embed_random_all_options(seed, sym, weighted):
    base = random_small_graph(seed, N=2500, E=30_000, K=5, weighted=weighted, sym=sym, unknown_frac=0.1)
    for d, l, c in FLAG_COMBOS:
        g = base.with_options(d, l, c)
        _label(f"embed random seed={seed} sym={sym} w={weighted} opts={(d, l, c)}")
        assert_close(embed_graph(g), or_embed_graph(g), f"opts={(d, l, c)}")


@pytest.mark.parametrize("K", [1, 2, 3, 31, 50, 64, 65, 100, 128])
def test_embed_class_counts_range(K):
    g = random_small_graph(K, N=4000, E=60_000, K=K, weighted=True, unknown_frac=0.05)
    g = g.with_options(True, True, True)
    _label(f"embed K={K}")
    assert_close(embed_graph(g), or_embed_graph(g), f"K={K}")
    g2 = g.with_options(False, False, False)
    assert_close(embed_graph(g2), or_embed_graph(g2), f"K={K} options off")


def _degree_condition(g, diag):
    """Per-row condition of the Laplacian factors: kappa_j = sum|a_jk| / |d_j| for the row
    itself and every neighbour (d from signed weights, +1 under the diagonal option)."""
    from oracle import degrees as or_degrees

    d = or_degrees(g.src, g.dst, g.w, g.N, diag=diag, sym=g.sym)
    dabs = or_degrees(g.src, g.dst, np.abs(g.w), g.N, diag=diag, sym=g.sym)
    with np.errstate(divide="ignore"):
        kap = np.where(d != 0, dabs / np.abs(d), np.inf)
    worst = kap.copy()
    np.maximum.at(worst, g.src, kap[g.dst])
    np.maximum.at(worst, g.dst, kap[g.src])
    return worst


def test_embed_signed_weights():
    """Signed weights: errors are measured row-normwise (cancellation inside a row), and
    under the Laplacian the bound is scaled by the degree condition number of the row and
    its neighbours, since a degree near zero amplifies FP32 rounding in D^-1/2."""
    g = random_small_graph(4, N=1500, E=20_000, K=4, weighted=True, signed=True)
    for d, l, c in FLAG_COMBOS:
        gg = g.with_options(d, l, c)
        _label(f"embed signed opts={(d, l, c)}")
        Z = embed_graph(gg).cpu().double().numpy()
        R = or_embed_graph(gg)
        rmax = np.max(np.abs(R), axis=1)
        err = np.max(np.abs(Z - R), axis=1)
        tol = np.full(g.N, 1e-5)
        if l:
            tol = 1e-5 * np.maximum(1.0, _degree_condition(gg, d))
        ok = rmax > 0
        assert np.all(err[~ok] == 0), (d, l, c)
        assert np.all(err[ok] <= tol[ok] * rmax[ok]), (d, l, c, float(np.max(err[ok] / rmax[ok])))
        if not l:
            assert float(np.max(err[ok] / rmax[ok])) <= 1e-5


def test_embed_edge_cases():
    _label("embed edge cases")
    # empty graph: zero rows, or the diagonal term alone
    e0 = np.zeros(0, np.int32)
    lab = np.array([0, 1, -1, 1, 2, 0, 2], np.int32)
    for d, l, c in FLAG_COMBOS:
        g = Graph(src=e0, dst=e0, w=None, N=7, labels=lab, K=3, diag=d, lap=l, cor=c)
        assert_close(embed_graph(g), or_embed_graph(g), f"empty {(d, l, c)}")
    # one node, self-loop only
    g = Graph(src=np.array([0], np.int32), dst=np.array([0], np.int32), w=np.array([0.5], np.float32),
              N=1, labels=np.array([0], np.int32), K=1, diag=True, lap=True, cor=False)
    assert_close(embed_graph(g), or_embed_graph(g), "single node")
    # all labels unknown -> Z = 0
    g = random_small_graph(1, N=500, E=3000, K=4, unknown_frac=1.0).with_options(True, True, True)
    assert_close(embed_graph(g), or_embed_graph(g), "all unknown")
    # an empty class and many isolated nodes
    g = random_small_graph(2, N=20_000, E=2000, K=6, unknown_frac=0.0)
    g.labels[g.labels == 3] = 4
    for d, l, c in FLAG_COMBOS:
        gg = g.with_options(d, l, c)
        assert_close(embed_graph(gg), or_embed_graph(gg), f"isolated {(d, l, c)}")


def _star(hub_deg, K=5, extra=2000, seed=0):
    rng = np.random.default_rng(seed)
    N = hub_deg + 1
    leaves = np.arange(1, N, dtype=np.int32)
    src = np.concatenate([np.zeros(hub_deg, np.int32), rng.integers(0, N, extra).astype(np.int32)])
    dst = np.concatenate([leaves, rng.integers(0, N, extra).astype(np.int32)])
    w = (1.0 - rng.random(src.size, dtype=np.float32)).astype(np.float32)
    lab = rng.integers(-1, K, size=N).astype(np.int32)
    return Graph(src=src, dst=dst, w=w, N=N, labels=lab, K=K, diag=True, lap=True, cor=True)


@pytest.mark.parametrize("we", [256, 512, 2048, 16384])
def test_embed_hub_rows_split_across_wavefronts(we):
    g = _star(120_000)
    _label(f"hub rows wave_entries={we}")
    assert_close(embed_graph(g, sched=dict(wave_entries=we)), or_embed_graph(g), f"star WE={we}")


@pytest.mark.parametrize("sched", [dict(wave_entries=256, waves_per_block=1),
                                   dict(wave_entries=1024, waves_per_block=2),
                                   dict(wave_entries=8192, waves_per_block=4, tile_entries=4096)])
def test_embed_schedules(sched):
    g = powerlaw_10m(N=30_000, E=400_000, K=20, dmax=8000.0)
    _label(f"embed schedule {sched}")
    assert_close(embed_graph(g, sched=sched), or_embed_graph(g), str(sched))


@pytest.mark.parametrize("K", [7, 50, 65])
def test_bucket_path_split_buckets(K):
    """Buckets cut into many parts (hub rows, the smallest part size) with K both a
    multiple of 4 and not, every option on: vs the oracle, and bitwise repeatable."""
    g = powerlaw_10m(N=20_000, E=300_000, K=K, dmax=9000.0)
    _label(f"bucket path split buckets K={K}")
    sched = dict(wave_entries=2048)
    Z1 = embed_graph(g, sched=sched)
    _ = torch.randn(1 << 20, device="cuda:0").sum().item()  # other kernels between the calls
    Z2 = embed_graph(g, sched=sched)
    assert torch.equal(Z1, Z2)
    assert_close(Z1, or_embed_graph(g), f"K={K}")


@pytest.mark.parametrize("sched", [dict(wave_entries=256, waves_per_block=1),
                                   dict(wave_entries=1024, waves_per_block=2),
                                   dict(wave_entries=8192, waves_per_block=4)])
def test_embed_csr_schedules(sched):
    """The CSR path's embed schedules on a resident CSR."""
    g = powerlaw_10m(N=30_000, E=400_000, K=20, dmax=8000.0)
    _label(f"embed_csr schedule {sched}")
    s, d, w, lab = graph_tensors(g)
    f = flags(g)
    rp, col, val = gee.gee_build_csr(s, d, w, g.N, f)
    M = int(rp[-1].item())
    Z = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f, sched=sched)
    torch.cuda.synchronize()
    assert_close(Z, or_embed_graph(g), str(sched))


# ----------------------------------------------------------------------------- resident CSR

def test_embed_csr_matches_embed():
    """The resident-CSR path (row-ordered sums) and the edge-list bucket path (sums in
    bucket order) round differently; both meet the oracle bar, and the entries the oracle
    gives as zero are zero on both."""
    g = powerlaw_10m(N=50_000, E=600_000, K=50, dmax=10_000.0)
    _label("embed_csr vs embed")
    s, d, w, lab = graph_tensors(g)
    f = flags(g)
    Z1 = gee.gee_embed(s, d, w, lab, g.K, f)
    rp, col, val = gee.gee_build_csr(s, d, w, g.N, f)
    M = int(rp[-1].item())
    Z2 = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f)
    torch.cuda.synchronize()
    R = or_embed_graph(g)
    assert_close(Z1, R, "embed")
    assert_close(Z2, R, "embed_csr")


def test_embed_csr_new_labels():
    """Re-embedding a resident CSR with different labels (the iterative use of GEE)."""
    g = random_small_graph(6, N=5000, E=80_000, K=8, weighted=True).with_options(True, True, True)
    s, d, w, lab = graph_tensors(g)
    rp, col, val = gee.gee_build_csr(s, d, w, g.N, flags(g))
    M = int(rp[-1].item())
    rng = np.random.default_rng(3)
    for it in range(3):
        lab2 = rng.integers(-1, g.K, size=g.N).astype(np.int32)
        _label(f"re-embed iteration {it}")
        Z = gee.gee_embed_csr(rp, col, val, M, to_dev(lab2, torch.int32), g.K, flags(g))
        torch.cuda.synchronize()
        R = or_embed(g.src, g.dst, g.w, g.N, lab2, g.K, diag=True, lap=True, cor=True)
        assert_close(Z, R, f"re-embed {it}")


# ----------------------------------------------------------------------------- determinism

def test_determinism_and_symmetrize_equivalence():
    g = powerlaw_10m(N=40_000, E=500_000, K=30, dmax=9000.0)
    _label("determinism")
    Z1 = embed_graph(g)
    Z2 = embed_graph(g)
    assert torch.equal(Z1, Z2)
    # the symmetrized list == the explicit interleaved list of rows and mirrors
    keep = g.src != g.dst
    E = g.E
    s2 = np.empty(2 * E, np.int32)
    d2 = np.empty(2 * E, np.int32)
    s2[0::2], s2[1::2] = g.src, g.dst
    d2[0::2], d2[1::2] = g.dst, g.src
    m = np.ones(2 * E, bool)
    m[1::2] = keep
    w2 = np.repeat(g.w, 2)[m]
    gx = Graph(src=s2[m], dst=d2[m], w=w2, N=g.N, labels=g.labels, K=g.K, diag=g.diag, lap=g.lap,
               cor=g.cor, sym=False)
    assert torch.equal(Z1, embed_graph(gx))


# ----------------------------------------------------------------------------- data errors

def test_data_errors_are_reported():
    _label("data errors")
    gee.gee_get_data_errors()  # clear
    g = random_small_graph(0, N=100, E=500, K=3)
    s, d, w, lab = graph_tensors(g)
    bad_lab = lab.clone()
    bad_lab[5] = 7
    gee.gee_embed(s, d, w, bad_lab, 3, flags(g))
    assert gee.gee_get_data_errors() & gee.GEE_DATA_LABEL
    bad_d = d.clone()
    bad_d[3] = 100
    gee.gee_embed(s, bad_d, w, lab, 3, flags(g))
    assert gee.gee_get_data_errors() & gee.GEE_DATA_INDEX
    bad_w = w.clone()
    bad_w[2] = float("nan")
    gee.gee_embed(s, d, bad_w, lab, 3, flags(g))
    assert gee.gee_get_data_errors() & gee.GEE_DATA_WEIGHT
    gee.gee_embed(s, d, w, lab, 3, flags(g))
    assert gee.gee_get_data_errors() == 0


def test_argument_errors():
    g = random_small_graph(0, N=100, E=500, K=3)
    s, d, w, lab = graph_tensors(g)
    with pytest.raises(gee.GeeError):
        gee.gee_embed(s, d, w, lab, 0, flags(g))
    with pytest.raises(gee.GeeError):
        gee.gee_embed(s, d, w, lab, 129, flags(g))
    with pytest.raises(gee.GeeError):
        gee.gee_embed(s, d, w, lab, 3, 1 << 9)


def test_unread_hip_error_of_the_caller_is_not_a_launch_failure():
    """A HIP error the application left unread (here: elapsed time of events never
    recorded) is not taken for a failed launch of the next call."""
    import ctypes
    import os

    hip = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipEventCreate(ctypes.byref(a)) == 0 and hip.hipEventCreate(ctypes.byref(b)) == 0
    ms = ctypes.c_float()
    assert hip.hipEventElapsedTime(ctypes.byref(ms), a, b) != 0  # leaves the thread's last error set
    g = random_small_graph(5, N=300, E=2000, K=4).with_options(True, True, True)
    Z = embed_graph(g)
    torch.cuda.synchronize()
    hip.hipEventDestroy(a)
    hip.hipEventDestroy(b)
    assert_close(Z, or_embed_graph(g), "after an unread HIP error")


# ----------------------------------------------------------------------------- full sizes

def test_sbm_small_both_option_sets():
    for opt in ("off", "all"):
        g = sbm_small(opt)
        _label(f"sbm N=2000 options={opt}")
        assert_close(embed_graph(g), or_embed_graph(g), f"sbm_small {opt}")


def test_sbm_dense_all_options():
    g = sbm_dense()
    _label(f"sbm N=10000 E={g.E}")
    assert_close(embed_graph(g), or_embed_graph(g), "sbm_dense")


def test_powerlaw_10m_full():
    """The 10M-edge power-law workload at full size, in the launch configuration the
    benchmark times (default schedule)."""
    g = powerlaw_10m()
    _label(f"powerlaw N={g.N} E={g.E} K={g.K}")
    Z = embed_graph(g)
    assert gee.gee_get_data_errors() == 0
    R = or_embed_graph(g)
    rel = assert_close(Z, R, "powerlaw_10m")
    _label(f"powerlaw max rel error {rel:.3e}")
    # unit row norms under correlation
    nr = torch.linalg.vector_norm(Z.double(), dim=1).cpu().numpy()
    nz = np.linalg.norm(R, axis=1) > 0
    assert np.all(np.abs(nr[nz] - 1) < 1e-5)
