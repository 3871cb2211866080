"""Seeded graph and label generators (inputs only; no embedding arithmetic).

Recipes follow the workloads of the paper's evaluation: stochastic block model
graphs with a class prior and within/between block probabilities (Section 4,
simulated datasets), and Chung-Lu power-law graphs standing in for the
Network-Repository "CL-100K-1d8-*" graphs of Table 2, whose files are not
available here.

Conventions shared by every generator:
  * node ids are int32 in [0, N), labels are int32 in [-1, K) with -1 = unknown;
  * an undirected graph is returned as one (src, dst) row per unordered pair, in
    shuffled order and with each row's orientation flipped with probability 1/2,
    so that no consumer ever sees pre-sorted input;
  * edge weights, when present, are float32 drawn as 1 - U with U uniform on
    [0, 1), i.e. in (0, 1].
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_ROOT = 240603726


def rng_for(config: int, graph: int = 0, salt: int = 0) -> np.random.Generator:
    """Canonical generator for (config, graph) so every consumer sees the same input."""
    return np.random.default_rng([SEED_ROOT, int(config), int(graph), int(salt)])


@dataclasses.dataclass
class Graph:
    """One embedding request: an edge list, labels and the three GEE options."""

    src: np.ndarray  # int32[E]
    dst: np.ndarray  # int32[E]
    w: Optional[np.ndarray]  # float32[E] or None (every weight is 1)
    N: int
    labels: np.ndarray  # int32[N], -1 = unknown
    K: int
    diag: bool = False
    lap: bool = False
    cor: bool = False
    sym: bool = True  # each row is one undirected edge
    deg_io: bool = False  # Laplacian with out-degrees on the left, in-degrees on the right
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def E(self) -> int:
        return int(self.src.shape[0])

    def with_options(self, diag: bool, lap: bool, cor: bool, name: str | None = None) -> "Graph":
        return dataclasses.replace(self, diag=diag, lap=lap, cor=cor, name=name or self.name)


# ----------------------------------------------------------------------------- labels

def iid_labels(N: int, prior, rng: np.random.Generator) -> np.ndarray:
    """Labels drawn independently from a class prior (the SBM setup of Section 4)."""
    prior = np.asarray(prior, dtype=np.float64)
    prior = prior / prior.sum()
    return rng.choice(len(prior), size=N, p=prior).astype(np.int32)


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    quota = weights / weights.sum() * total
    base = np.floor(quota).astype(np.int64)
    short = total - int(base.sum())
    if short > 0:
        order = np.argsort(-(quota - base), kind="stable")
        base[order[:short]] += 1
    return base


def zipf_labels(N: int, K: int, s: float, unknown_frac: float, rng: np.random.Generator) -> np.ndarray:
    """Class sizes proportional to (k+1)^-s over the labelled nodes (largest-remainder
    rounding), a fraction of nodes left unknown (-1), then randomly placed over nodes."""
    n_unknown = int(round(unknown_frac * N))
    labelled = N - n_unknown
    sizes = _largest_remainder(np.arange(1, K + 1, dtype=np.float64) ** (-s), labelled)
    lab = np.concatenate([np.repeat(np.arange(K, dtype=np.int32), sizes),
                          np.full(n_unknown, -1, dtype=np.int32)])
    rng.shuffle(lab)
    return lab


def uniform_weights(E: int, rng: np.random.Generator) -> np.ndarray:
    """float32 weights in (0, 1]."""
    return (np.float32(1.0) - rng.random(E, dtype=np.float32)).astype(np.float32)


# ----------------------------------------------------------------------------- helpers

def _sample_distinct(P: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """`count` distinct integers from [0, P), uniformly."""
    if count <= 0:
        return np.zeros(0, dtype=np.int64)
    if count > P:
        raise ValueError("more samples than population")
    if P <= 50_000_000 and count * 4 > P:
        return rng.choice(P, size=count, replace=False).astype(np.int64)
    have = np.zeros(0, dtype=np.int64)
    while have.size < count:
        need = count - have.size
        draw = rng.integers(0, P, size=int(need * 1.05) + 16, dtype=np.int64)
        have = np.unique(np.concatenate([have, draw]))
    # keep a uniformly random subset of the right size
    keep = rng.choice(have.size, size=count, replace=False)
    return have[np.sort(keep)]


def _decode_upper_pair(t: np.ndarray, n: int):
    """Index t in [0, n(n-1)/2) -> (i, j), i < j, row-major over the strict upper triangle."""
    t = t.astype(np.int64)
    b = 2 * n - 1
    i = np.floor((b - np.sqrt(np.maximum(b * b - 8.0 * t, 0.0))) / 2.0).astype(np.int64)
    i = np.clip(i, 0, n - 2)

    def start(r):
        return r * (2 * n - r - 1) // 2

    for _ in range(2):
        i = np.where(start(i) > t, i - 1, i)
        i = np.where(start(i + 1) <= t, i + 1, i)
    j = t - start(i) + i + 1
    return i, j


def shuffle_and_orient(src: np.ndarray, dst: np.ndarray, w: Optional[np.ndarray], rng: np.random.Generator):
    """Random row order, and each row's (src, dst) swapped with probability 1/2."""
    E = src.shape[0]
    order = rng.permutation(E)
    s = src[order]
    d = dst[order]
    flip = rng.random(E) < 0.5
    s2 = np.where(flip, d, s).astype(np.int32)
    d2 = np.where(flip, s, d).astype(np.int32)
    w2 = None if w is None else w[order].astype(np.float32)
    return s2, d2, w2


# ----------------------------------------------------------------------------- SBM

def sbm_expected_edges(N: int, prior, p_in: float, p_out: float) -> float:
    """Expected unordered-pair edge count when labels are i.i.d. from `prior`."""
    prior = np.asarray(prior, dtype=np.float64)
    prior = prior / prior.sum()
    same = float((prior ** 2).sum())
    return N * (N - 1) / 2.0 * (same * p_in + (1.0 - same) * p_out)


def sbm_edges(labels: np.ndarray, K: int, B, rng: np.random.Generator):
    """Undirected SBM: every unordered pair (i, j) with i != j is an edge independently
    with probability B[y_i, y_j]. Nodes labelled -1 take no part. Returns (src, dst)
    grouped by block pair; callers shuffle with `shuffle_and_orient`."""
    B = np.asarray(B, dtype=np.float64)
    members = [np.flatnonzero(labels == k).astype(np.int64) for k in range(K)]
    srcs, dsts = [], []
    for a in range(K):
        na = members[a].size
        for b in range(a, K):
            nb = members[b].size
            p = float(B[a, b])
            if a == b:
                P = na * (na - 1) // 2
            else:
                P = na * nb
            if P == 0 or p <= 0.0:
                continue
            cnt = int(rng.binomial(P, min(p, 1.0)))
            t = _sample_distinct(P, cnt, rng)
            if a == b:
                i, j = _decode_upper_pair(t, na)
                srcs.append(members[a][i])
                dsts.append(members[a][j])
            else:
                srcs.append(members[a][t // nb])
                dsts.append(members[b][t % nb])
    if not srcs:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    return np.concatenate(srcs).astype(np.int32), np.concatenate(dsts).astype(np.int32)


def sbm_block_matrix(K: int, p_in: float, p_out: float) -> np.ndarray:
    B = np.full((K, K), p_out, dtype=np.float64)
    np.fill_diagonal(B, p_in)
    return B


# ----------------------------------------------------------------------------- Chung-Lu

def chung_lu_expected_degrees(N: int, E: int, gamma: float, dmax: float) -> np.ndarray:
    """Expected degrees w_i = c (i + i0)^(-1/(gamma-1)), with (c, i0) chosen so that
    w_0 = dmax and sum_i w_i = 2E."""
    alpha = 1.0 / (gamma - 1.0)
    idx = np.arange(N, dtype=np.float64)
    target = 2.0 * E
    if N * dmax < target:
        raise ValueError("dmax too small for the requested edge count")

    def total(i0):
        return dmax * np.sum((i0 / (idx + i0)) ** alpha)

    lo, hi = 1e-9, 1.0
    while total(hi) < target:
        hi *= 2.0
        if hi > 1e15:
            raise ValueError("cannot reach the requested edge count")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < target:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-12 * hi:
            break
    i0 = 0.5 * (lo + hi)
    return dmax * (i0 / (idx + i0)) ** alpha


def chung_lu_edges(N: int, E: int, gamma: float, dmax: float, rng: np.random.Generator,
                   permute: bool = True):
    """Chung-Lu graph with exactly E distinct undirected edges and no self-loops.

    Endpoints are drawn independently with probability proportional to the expected
    degree; self-loops are rejected, repeated unordered pairs collapse to one, and the
    draw tops up until E distinct pairs exist. Node ids are then randomly permuted so
    that high-degree nodes are scattered over the id range."""
    if E > N * (N - 1) // 2:
        raise ValueError("too many edges for N")
    wdeg = chung_lu_expected_degrees(N, E, gamma, dmax)
    P = N * (N - 1) // 2
    keys = np.zeros(0, dtype=np.int64)
    if P <= 20_000_000 and E * 8 > P:
        # Dense small graph: rejection would stall, so draw E distinct pairs with
        # probability proportional to w_u w_v by weighted sampling without replacement
        # (Efraimidis-Spirakis keys log(U) / weight, keep the E largest).
        iu, ju = np.triu_indices(N, k=1)
        pw = wdeg[iu] * wdeg[ju]
        score = np.log(rng.random(P)) / pw
        top = np.argpartition(-score, E - 1)[:E]
        keys = np.sort(iu[top].astype(np.int64) * N + ju[top].astype(np.int64))
    cdf = np.cumsum(wdeg)
    cdf /= cdf[-1]
    while keys.size < E:
        need = E - keys.size
        m = int(need * 1.15) + 64
        u = np.searchsorted(cdf, rng.random(m), side="right")
        v = np.searchsorted(cdf, rng.random(m), side="right")
        u = np.minimum(u, N - 1)
        v = np.minimum(v, N - 1)
        ok = u != v
        lo = np.minimum(u, v)[ok].astype(np.int64)
        hi = np.maximum(u, v)[ok].astype(np.int64)
        fresh = lo * N + hi
        keys = np.unique(np.concatenate([keys, fresh]))
    if keys.size > E:
        keep = rng.choice(keys.size, size=E, replace=False)
        keys = keys[np.sort(keep)]
    lo = (keys // N).astype(np.int64)
    hi = (keys % N).astype(np.int64)
    if permute:
        perm = rng.permutation(N).astype(np.int64)
        lo = perm[lo]
        hi = perm[hi]
    return lo.astype(np.int32), hi.astype(np.int32)


# ----------------------------------------------------------------------------- Eq. 2

def edge_density(num_nodes: int, num_edges: int) -> float:
    """Edge density of an undirected graph, Section 4 Eq. (2): d = 2|E| / (|V| (|V| - 1))."""
    if num_nodes < 2:
        return 0.0
    return 2.0 * num_edges / (num_nodes * (num_nodes - 1.0))


def loguniform_int(lo: float, hi: float, rng: np.random.Generator) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
