"""The synthetic workloads the GEE path is tested and measured on.

* ``sbm_small``   - SBM, N=2,000, K=3, prior [0.2, 0.3, 0.5], p_in 0.13, p_out 0.10,
                    unweighted, undirected (about 222.7k edges); options off or all on.
* ``sbm_dense``   - the same SBM at N=10,000 (about 5.57M edges, the largest simulated
                    graph of Section 4.1), unweighted, all options on.
* ``powerlaw_10m`` - Chung-Lu, N=600,000, E=10,000,000, exponent 2.1, max expected
                    degree 50,000, weights in (0, 1], K=50 with Zipf(1.1) class sizes and
                    10% unknown labels, all options on. It stands in for the 10M-edge
                    "CL-100K-1d8-L5" graph of Tables 2-4, which is not available here.
* ``batched_graphs`` - 512 independent uneven graphs (Chung-Lu exponent 2.5).
* ``serving_pool`` - a pool of mixed SBM / power-law requests for the serving loop.
"""

from __future__ import annotations

import math

import numpy as np

from .generators import (
    Graph,
    chung_lu_edges,
    iid_labels,
    loguniform_int,
    rng_for,
    sbm_block_matrix,
    sbm_edges,
    shuffle_and_orient,
    uniform_weights,
    zipf_labels,
)

CONFIG_NAMES = {
    1: "sbm_n2000_k3",
    2: "sbm_n10000_k3",
    3: "chunglu_n600k_e10m_k50",
    4: "batched_512_chunglu",
    5: "serving_mixed_pool",
}

SBM_PRIOR = (0.2, 0.3, 0.5)
SBM_P_IN = 0.13
SBM_P_OUT = 0.10


def _sbm(N: int, cfg: int, graph: int = 0) -> Graph:
    rng = rng_for(cfg, graph)
    K = len(SBM_PRIOR)
    labels = iid_labels(N, SBM_PRIOR, rng)
    s, d = sbm_edges(labels, K, sbm_block_matrix(K, SBM_P_IN, SBM_P_OUT), rng)
    s, d, _ = shuffle_and_orient(s, d, None, rng)
    return Graph(src=s, dst=d, w=None, N=N, labels=labels, K=K, sym=True)


def sbm_small(options: str = "off") -> Graph:
    """SBM N=2,000 (options "off" or "all")."""
    g = _sbm(2000, 1)
    on = options == "all"
    return g.with_options(on, on, on, name=f"{CONFIG_NAMES[1]}_{options}")


def sbm_dense() -> Graph:
    """SBM N=10,000, all options on."""
    return _sbm(10_000, 2).with_options(True, True, True, name=CONFIG_NAMES[2])


def powerlaw_10m(N: int = 600_000, E: int = 10_000_000, K: int = 50, dmax: float = 50_000.0) -> Graph:
    """Chung-Lu power-law graph, all options on. Smaller sizes reuse the same recipe."""
    rng = rng_for(3, 0 if (N, E, K) == (600_000, 10_000_000, 50) else N ^ (E << 1) ^ (K << 40))
    s, d = chung_lu_edges(N, E, 2.1, dmax, rng)
    w = uniform_weights(E, rng)
    s, d, w = shuffle_and_orient(s, d, w, rng)
    labels = zipf_labels(N, K, 1.1, 0.10, rng)
    name = CONFIG_NAMES[3] if (N, E, K) == (600_000, 10_000_000, 50) else f"chunglu_n{N}_e{E}_k{K}"
    return Graph(src=s, dst=d, w=w, N=N, labels=labels, K=K, sym=True,
                 diag=True, lap=True, cor=True, name=name)


def batched_one(g: int, cfg: int = 4) -> Graph:
    """Graph `g` of the batched workload: N log-uniform in [100, 50,000], average degree
    uniform in [5, 200] (capped at (N-1)/2), Chung-Lu exponent 2.5 with max expected
    degree sqrt(N d), K uniform in {2..64}, labels uniform with no unknowns, weights in
    (0, 1], and each option an independent fair coin."""
    rng = rng_for(cfg, g)
    N = loguniform_int(100, 50_000, rng)
    d = float(rng.uniform(5.0, 200.0))
    d = min(d, (N - 1) / 2.0)
    E = max(1, int(round(N * d / 2.0)))
    dmax = math.sqrt(N * d)
    K = int(rng.integers(2, 65))
    diag, lap, cor = (bool(x) for x in rng.random(3) < 0.5)
    s, dd = chung_lu_edges(N, E, 2.5, dmax, rng)
    w = uniform_weights(E, rng)
    s, dd, w = shuffle_and_orient(s, dd, w, rng)
    labels = rng.integers(0, K, size=N).astype(np.int32)
    return Graph(src=s, dst=dd, w=w, N=N, labels=labels, K=K, sym=True,
                 diag=diag, lap=lap, cor=cor, name=f"batched_g{g}")


def batched_graphs(G: int = 512, cfg: int = 4):
    return [batched_one(g, cfg) for g in range(G)]


def serving_one(g: int, cfg: int = 5, e_max: int = 20_000_000) -> Graph:
    """Request `g` of the serving pool: E log-uniform in [1k, e_max], SBM or Chung-Lu
    (exponent 2.1) 50/50, average degree uniform in [5, 200], N = max(2E/d, 2 sqrt(E)+1),
    K uniform in {2..128}, 0-20% unknown labels, weights in (0, 1], random options."""
    rng = rng_for(cfg, g)
    E = loguniform_int(1_000, e_max, rng)
    d = float(rng.uniform(5.0, 200.0))
    N = int(max(round(2 * E / d), math.ceil(2 * math.sqrt(E)) + 1))
    K = int(rng.integers(2, 129))
    unk = float(rng.uniform(0.0, 0.2))
    diag, lap, cor = (bool(x) for x in rng.random(3) < 0.5)
    kind = "sbm" if rng.random() < 0.5 else "powerlaw"
    if kind == "sbm":
        labels = rng.integers(0, K, size=N).astype(np.int32)
        # p_in / p_out = 1.3 and expected degree d over a uniform prior
        p_out = d / ((N - 1) * (1.3 / K + (K - 1) / K))
        s, dd = sbm_edges(labels, K, sbm_block_matrix(K, 1.3 * p_out, p_out), rng)
        unknown = rng.random(N) < unk
        labels = np.where(unknown, -1, labels).astype(np.int32)
    else:
        dmax = min(N - 1.0, max(math.sqrt(N * d) * 4.0, d * 2.0))
        s, dd = chung_lu_edges(N, E, 2.1, dmax, rng)
        labels = rng.integers(0, K, size=N).astype(np.int32)
        unknown = rng.random(N) < unk
        labels = np.where(unknown, -1, labels).astype(np.int32)
    E = int(s.shape[0])
    w = uniform_weights(E, rng)
    s, dd, w = shuffle_and_orient(s, dd, w, rng)
    return Graph(src=s, dst=dd, w=w, N=N, labels=labels, K=K, sym=True,
                 diag=diag, lap=lap, cor=cor, name=f"serve_{kind}_g{g}",
                 meta={"kind": kind})


def serving_pool(n: int = 64, cfg: int = 5, e_max: int = 20_000_000):
    return [serving_one(g, cfg, e_max) for g in range(n)]


def random_small_graph(seed: int, N: int = 50, E: int = 200, K: int = 4, weighted: bool = True,
                       self_loops: bool = True, duplicates: bool = True, unknown_frac: float = 0.1,
                       sym: bool = True, diag: bool = False, lap: bool = False, cor: bool = False,
                       signed: bool = False) -> Graph:
    """Small adversarial graph for parity tests: uniform endpoints with optional
    self-loops and repeated pairs, optional unknown labels, optional signed weights."""
    rng = rng_for(100, seed)
    s = rng.integers(0, max(N, 1), size=E).astype(np.int32) if N > 0 else np.zeros(0, np.int32)
    d = rng.integers(0, max(N, 1), size=E).astype(np.int32) if N > 0 else np.zeros(0, np.int32)
    if not self_loops and E > 0:
        clash = s == d
        d = np.where(clash, (d + 1) % max(N, 1), d).astype(np.int32)
    if not duplicates and E > 0:
        key = np.minimum(s, d).astype(np.int64) * N + np.maximum(s, d)
        _, first = np.unique(key, return_index=True)
        first = np.sort(first)
        s, d = s[first], d[first]
    w = None
    if weighted:
        w = uniform_weights(s.shape[0], rng)
        if signed:
            w = np.where(rng.random(s.shape[0]) < 0.3, -w, w).astype(np.float32)
    labels = rng.integers(0, K, size=N).astype(np.int32)
    if unknown_frac > 0:
        labels = np.where(rng.random(N) < unknown_frac, -1, labels).astype(np.int32)
    return Graph(src=s.astype(np.int32), dst=d.astype(np.int32), w=w, N=N, labels=labels, K=K,
                 sym=sym, diag=diag, lap=lap, cor=cor, name=f"random_s{seed}")
