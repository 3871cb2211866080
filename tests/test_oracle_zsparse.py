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


# Plausible mistakes, each planted in a copy of the storage routine: every one must fail
# at least one of the pins above (the Section 3 example or the scipy comparison).
def _column_major(Z):
    keep = Z != 0
    rp = np.zeros(Z.shape[0] + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=rp[1:])
    cols, rows = np.nonzero(keep.T)  # walks Z column by column
    return rp, cols.astype(np.int64), Z[rows, cols]


def _pointers_shifted(Z):
    rp, col, val = sparse_rows(Z)
    return np.concatenate([rp[1:], rp[-1:]]), col, val


def _keeps_negative_zero(Z):
    keep = np.signbit(Z) | (Z != 0)
    rp = np.zeros(Z.shape[0] + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=rp[1:])
    rows, cols = np.nonzero(keep)
    return rp, cols.astype(np.int64), Z[rows, cols]


def _classes_decreasing(Z):
    rp, col, val = sparse_rows(Z)
    col, val = col.copy(), val.copy()
    for i in range(Z.shape[0]):
        col[rp[i]:rp[i + 1]] = col[rp[i]:rp[i + 1]][::-1]
        val[rp[i]:rp[i + 1]] = val[rp[i]:rp[i + 1]][::-1]
    return rp, col, val


def _drops_last_row(Z):
    rp, col, val = sparse_rows(Z[:-1])
    return np.concatenate([rp, rp[-1:]]), col, val


def _pins_pass(fn):
    ex = json.load(open(os.path.join(HERE, "golden", "csr_section3_example.json")))
    M = np.zeros((ex["num_rows"], 6))
    for r, c, v in ex["directed_rows"]:
        M[r, c] = v
    rp, col, val = fn(M)
    e = ex["expect"]
    ok = (len(rp) == e["index_pointers_len"] and rp[2] == e["index_pointers_2"] and rp[3] == e["index_pointers_3"]
          and list(col[3:5]) == e["col_indices_3_5"] and list(val[3:5]) == e["data_3_5"])
    for seed in range(4):
        rng = np.random.default_rng(seed)
        Z = rng.standard_normal((300, 17))
        Z[rng.random(Z.shape) < 0.6] = 0.0
        Z[0, :] = 0.0
        Z[5, 3] = -0.0
        Z[-1, :] = 0.0
        Z[-1, 2] = 1.5  # the last row holds one entry
        rp, col, val = fn(Z)
        ref = sp.csr_matrix(Z)
        ref.sort_indices()
        ok = ok and (np.array_equal(rp, ref.indptr) and np.array_equal(col, ref.indices)
                     and np.array_equal(val, ref.data))
    return ok


def test_pins_hold_for_the_oracle():
    assert _pins_pass(sparse_rows)


@pytest.mark.parametrize("mutant", [_column_major, _pointers_shifted, _keeps_negative_zero, _classes_decreasing,
                                    _drops_last_row])
def test_planted_mistakes_fail(mutant):
    assert not _pins_pass(mutant), mutant.__name__
