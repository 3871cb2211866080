"""CPU checks of the canonical CSR reference and of the input generators."""

import json
import os

import numpy as np

from gee_workloads import (chung_lu_edges, edge_density, random_small_graph, rng_for,
                           sbm_expected_edges, sbm_small, zipf_labels)
from gee_workloads.configs import SBM_P_IN, SBM_P_OUT, SBM_PRIOR, batched_one, serving_one
from oracle import csr

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_csr_section3_example():
    """P6: the Section 3 prose example of index_pointers / col_indices / data."""
    with open(os.path.join(GOLDEN, "csr_section3_example.json")) as f:
        fx = json.load(f)
    rows = np.array(fx["directed_rows"], dtype=np.float64)
    rp, col, val = csr(rows[:, 0].astype(np.int32), rows[:, 1].astype(np.int32),
                       rows[:, 2].astype(np.float32), fx["num_rows"], sym=False)
    ex = fx["expect"]
    assert len(rp) == ex["index_pointers_len"]
    assert rp[2] == ex["index_pointers_2"] and rp[3] == ex["index_pointers_3"]
    assert list(col[3:5]) == ex["col_indices_3_5"]
    assert list(val[3:5]) == ex["data_3_5"]


def _brute_csr(src, dst, w, N, sym):
    rows = [[] for _ in range(N)]
    for e, (s, d) in enumerate(zip(src, dst)):
        rows[s].append((d, None if w is None else w[e]))
        if sym and s != d:
            rows[d].append((s, None if w is None else w[e]))
    rp = [0]
    col, val = [], []
    for r in rows:
        for c, v in r:
            col.append(c)
            val.append(v)
        rp.append(len(col))
    return np.array(rp), np.array(col, dtype=np.int64), val


def test_csr_matches_loop():
    for seed in range(5):
        for sym in (True, False):
            for weighted in (True, False):
                g = random_small_graph(seed, N=40, E=150, K=3, weighted=weighted, sym=sym)
                rp, col, val = csr(g.src, g.dst, g.w, g.N, sym=sym)
                brp, bcol, bval = _brute_csr(g.src, g.dst, g.w, g.N, sym)
                assert np.array_equal(rp, brp)
                assert np.array_equal(col, bcol)
                if weighted:
                    assert np.array_equal(val, np.array(bval, dtype=np.float32))
                else:
                    assert val is None


def test_csr_empty_and_isolated():
    rp, col, val = csr(np.zeros(0, np.int32), np.zeros(0, np.int32), None, 5, sym=True)
    assert list(rp) == [0] * 6 and col.size == 0


def test_table2_density():
    """P7: Eq. (2) reproduces the printed density column of Table 2 to within one unit of
    the last printed digit (the table truncates Citeseer's 0.000855 to 0.00085 but rounds
    PubMed's 0.000228 to 0.00023, so neither rounding rule fits every row)."""
    with open(os.path.join(GOLDEN, "table2_density.json")) as f:
        fx = json.load(f)
    for row in fx["rows"]:
        d = edge_density(row["nodes"], row["edges"])
        assert abs(d - row["density"]) < 1e-5, row["dataset"]


def test_sbm_generator_statistics():
    g = sbm_small("off")
    assert g.N == 2000 and g.K == 3 and g.w is None
    exp = sbm_expected_edges(2000, SBM_PRIOR, SBM_P_IN, SBM_P_OUT)
    assert abs(g.E - exp) < 5 * np.sqrt(exp)
    assert abs(exp - 222_700) < 200  # "~220k" edges for the N=2,000 configuration
    frac = np.bincount(g.labels, minlength=3) / g.N
    assert np.allclose(frac, SBM_PRIOR, atol=0.04)
    # no self-loops, no repeated pairs, shuffled orientation
    assert not np.any(g.src == g.dst)
    key = np.minimum(g.src, g.dst).astype(np.int64) * g.N + np.maximum(g.src, g.dst)
    assert np.unique(key).size == g.E
    assert 0.45 < np.mean(g.src < g.dst) < 0.55
    # the paper's 10k-node graph has ~5.6M edges (Section 4.1)
    assert abs(sbm_expected_edges(10_000, SBM_PRIOR, SBM_P_IN, SBM_P_OUT) - 5.57e6) < 1e4


def test_chung_lu_generator():
    rng = rng_for(99)
    s, d = chung_lu_edges(5000, 40_000, 2.1, 800.0, rng)
    assert s.size == 40_000
    assert not np.any(s == d)
    key = np.minimum(s, d).astype(np.int64) * 5000 + np.maximum(s, d)
    assert np.unique(key).size == 40_000
    deg = np.bincount(s, minlength=5000) + np.bincount(d, minlength=5000)
    assert deg.max() <= 800 * 1.2 and deg.max() > 200  # heavy tail up to ~dmax
    assert np.median(deg) < deg.mean()  # skewed


def test_zipf_labels():
    lab = zipf_labels(10_000, 50, 1.1, 0.1, rng_for(98))
    assert (lab == -1).sum() == 1000
    c = np.bincount(lab[lab >= 0], minlength=50)
    assert c.sum() == 9000 and np.all(np.diff(c) <= 0) and c[-1] > 0


def test_batched_and_serving_recipes():
    g = batched_one(0)
    assert 100 <= g.N <= 50_000 and 2 <= g.K <= 64 and g.w is not None
    assert g.labels.min() >= 0
    s = serving_one(0, e_max=200_000)
    assert 2 <= s.K <= 128 and s.E >= 900
    assert s.labels.min() >= -1


def test_generators_are_deterministic():
    a = random_small_graph(5, N=100, E=300)
    b = random_small_graph(5, N=100, E=300)
    assert np.array_equal(a.src, b.src) and np.array_equal(a.w, b.w)
