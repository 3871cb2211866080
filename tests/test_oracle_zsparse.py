"""The oracle's sparse storage of Z pinned outside itself (CPU only): the Section 3 CSR
prose example, scipy.sparse's CSR of the same dense matrix, and the round trip."""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from gee_workloads import random_small_graph
from oracle import dense_of, embed_graph, sparse_rows

HERE = os.path.dirname(os.path.abspath(__file__))


def test_section3_prose_example():
    ex = json.load(open(os.path.join(HERE, "golden", "csr_section3_example.json")))
    R = ex["num_rows"]
    M = np.zeros((R, 6))
    for r, c, v in ex["directed_rows"]:
        M[r, c] = v
    rp, col, val = sparse_rows(M)
    e = ex["expect"]
    assert len(rp) == e["index_pointers_len"]
    assert rp[2] == e["index_pointers_2"] and rp[3] == e["index_pointers_3"]
    assert list(col[3:5]) == e["col_indices_3_5"]
    assert list(val[3:5]) == e["data_3_5"]


@pytest.mark.parametrize("seed", range(4))
def test_matches_scipy_csr(seed):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((300, 17))
    Z[rng.random(Z.shape) < 0.6] = 0.0
    Z[0, :] = 0.0  # an empty row
    Z[5, 3] = -0.0  # a negative zero is not stored
    rp, col, val = sparse_rows(Z)
    ref = sp.csr_matrix(Z)
    ref.sort_indices()
    assert np.array_equal(rp, ref.indptr) and np.array_equal(col, ref.indices)
    assert np.array_equal(val, ref.data)


def test_round_trip_on_embeddings():
    g = random_small_graph(3, N=400, E=2000, K=9, weighted=True, unknown_frac=0.1)
    for opts in ((False, False, False), (True, True, True)):
        Z = embed_graph(g.with_options(*opts))
        rp, col, val = sparse_rows(Z)
        assert rp[-1] == np.count_nonzero(Z)
        assert np.all(val != 0)
        assert np.array_equal(dense_of(rp, col, val, g.N, g.K), Z)
        # classes increase inside each row
        for i in range(g.N):
            assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)


def test_mistakes_fail():
    """A column-major walk or a dropped last row would not pass the pins above."""
    rng = np.random.default_rng(9)
    Z = rng.standard_normal((20, 5))
    Z[rng.random(Z.shape) < 0.5] = 0.0
    ref = sp.csr_matrix(Z)
    cols_t, rows_t = np.nonzero(Z.T)  # column-major order
    assert not np.array_equal(rows_t * 5 + cols_t, np.repeat(np.arange(20), np.diff(ref.indptr)) * 5 + ref.indices)
    rp, _, _ = sparse_rows(Z[:-1])
    assert len(rp) != len(ref.indptr)
