"""Checks that pin the FP64 oracle to facts outside itself.

Each function takes an oracle library handle (``oracle.oracle.load()`` or a mutated
build) and raises AssertionError when the oracle disagrees with:
  * the dense matrix form of Table 1 evaluated with numpy (brute force, tiny graphs);
  * the scipy.sparse route, the library the paper builds sparse GEE on (Section 3);
  * closed forms worked by hand (golden fixture, complete graph, regular graph, star,
    empty graph);
  * invariants the definition fixes (class counts, integer counts, column sums, unit
    row norms, symmetrization, linearity, permutations, symmetry of the Laplacian).
"""

from __future__ import annotations

import json
import os

import numpy as np

from gee_workloads import random_small_graph
from oracle import oracle as orc
from oracle.scipy_route import scipy_route

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

FLAG_COMBOS = [(d, l, c) for d in (False, True) for l in (False, True) for c in (False, True)]


# ----------------------------------------------------------------------------- references

def dense_brute_force(src, dst, w, N, labels, K, diag, lap, cor, sym, deg_io=False):
    """Table 1 in matrix form with dense numpy arrays (N small). `deg_io`: the Laplacian
    takes the row sums on the left and the column sums on the right."""
    A = np.zeros((N, N), dtype=np.float64)
    wv = np.ones(len(src)) if w is None else np.asarray(w, dtype=np.float64)
    for s, d, v in zip(src, dst, wv):
        A[s, d] += v
        if sym and s != d:
            A[d, s] += v
    if diag:
        A = A + np.eye(N)
    if lap:
        def inv_sqrt(deg):
            return np.where(deg > 0, 1.0 / np.sqrt(np.where(deg > 0, deg, 1.0)), 0.0)

        left = inv_sqrt(A.sum(axis=1))
        right = inv_sqrt(A.sum(axis=0)) if deg_io else left
        A = np.diag(left) @ A @ np.diag(right)
    W = np.zeros((N, K), dtype=np.float64)
    nk = np.array([(labels == k).sum() for k in range(K)], dtype=np.float64)
    for j in range(N):
        if labels[j] >= 0:
            W[j, labels[j]] = 1.0 / nk[labels[j]]
    Z = A @ W
    if cor:
        nr = np.linalg.norm(Z, axis=1, keepdims=True)
        Z = np.where(nr > 0, Z / np.where(nr > 0, nr, 1.0), 0.0)
    return Z


def _embed(lib, g, **over):
    kw = dict(diag=g.diag, lap=g.lap, cor=g.cor, sym=g.sym, deg_io=g.deg_io)
    kw.update(over)
    return orc.embed(g.src, g.dst, g.w, g.N, g.labels, g.K, lib=lib, **kw)


def _close(a, b, tol=1e-11, what=""):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, f"{what}: shape {a.shape} vs {b.shape}"
    err = np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))) if a.size else 0.0
    assert err <= tol, f"{what}: max error {err:.3e} > {tol:.1e}"


# ----------------------------------------------------------------------------- pins

def pin_brute_force(lib, seeds=range(6)):
    """P1: oracle == dense Table 1 on adversarial tiny graphs, every option combination,
    symmetrized and directed, weighted, unweighted and signed."""
    for seed in seeds:
        for sym in (True, False):
            for weighted, signed in ((False, False), (True, False), (True, True)):
                g = random_small_graph(seed, N=23, E=70, K=4, weighted=weighted, signed=signed,
                                       sym=sym, unknown_frac=0.15)
                for diag, lap, cor in FLAG_COMBOS:
                    for io in ((False, True) if lap else (False,)):
                        Z = _embed(lib, g, diag=diag, lap=lap, cor=cor, deg_io=io)
                        R = dense_brute_force(g.src, g.dst, g.w, g.N, g.labels, g.K, diag, lap, cor, sym,
                                              deg_io=io)
                        _close(Z, R, 1e-11, f"brute force seed={seed} sym={sym} w={weighted} "
                                            f"signed={signed} opts={(diag, lap, cor)} in/out={io}")


def pin_scipy_route(lib, graphs):
    """P2: oracle == scipy.sparse CSR products (the paper's library) on given graphs."""
    for g in graphs:
        Z = _embed(lib, g)
        R = scipy_route(g.src, g.dst, g.w, g.N, g.labels, g.K, g.diag, g.lap, g.cor, g.sym,
                        deg_io=g.deg_io)
        _close(Z, R, 1e-10, f"scipy route {g.name}")


def pin_hand_worked(lib):
    """Closed forms worked by hand (tests/golden/hand_worked_small.json)."""
    with open(os.path.join(GOLDEN, "hand_worked_small.json")) as f:
        fx = json.load(f)
    gg = fx["graph"]
    e = np.array(gg["undirected_edges"], dtype=np.int32)
    lab = np.array(gg["labels"], dtype=np.int32)
    opts = {"off": (0, 0, 0), "diag": (1, 0, 0), "lap": (0, 1, 0), "cor": (0, 0, 1), "all": (1, 1, 1)}
    for name, (d, l, c) in opts.items():
        Z = orc.embed(e[:, 0], e[:, 1], None, gg["N"], lab, gg["K"], diag=bool(d), lap=bool(l),
                      cor=bool(c), sym=True, lib=lib)
        _close(Z, fx["expect"][name], 1e-12, f"hand worked {name}")
        # the same graph given with the other orientation of every row
        Z2 = orc.embed(e[:, 1], e[:, 0], None, gg["N"], lab, gg["K"], diag=bool(d), lap=bool(l),
                       cor=bool(c), sym=True, lib=lib)
        _close(Z2, fx["expect"][name], 1e-12, f"hand worked reversed {name}")
    dg = fx["directed"]["graph"]
    r = np.array(dg["directed_rows"], dtype=np.int32)
    for name, l in (("off", False), ("lap", True)):
        Z = orc.embed(r[:, 0], r[:, 1], None, dg["N"], np.array(dg["labels"], np.int32), dg["K"],
                      lap=l, sym=False, lib=lib)
        _close(Z, fx["directed"]["expect"][name], 1e-12, f"hand worked directed {name}")


def pin_directed_degrees(lib):
    """The two degree readings of the Laplacian on a directed graph, worked by hand
    (tests/golden/directed_degrees.json), the in-degrees themselves, and that on symmetric
    input the in/out reading equals the row-sum reading."""
    with open(os.path.join(GOLDEN, "directed_degrees.json")) as f:
        fx = json.load(f)
    gg = fx["graph"]
    rows = np.array(gg["directed_rows"], dtype=np.float64)
    s, d, w = rows[:, 0].astype(np.int32), rows[:, 1].astype(np.int32), rows[:, 2]
    lab = np.array(gg["labels"], dtype=np.int32)
    N, K = gg["N"], gg["K"]
    cases = {"lap_rowsum": (False, False), "lap_inout": (False, True), "diag_lap_inout": (True, True)}
    for name, (diag, io) in cases.items():
        Z = orc.embed(s, d, w, N, lab, K, diag=diag, lap=True, sym=False, deg_io=io, lib=lib)
        _close(Z, fx["expect"][name], 1e-12, f"directed degrees {name}")
    _close(orc.in_degrees(s, d, w, N, sym=False, lib=lib), fx["expect"]["in_degrees"], 1e-14, "in-degrees")
    _close(orc.in_degrees(s, d, w, N, diag=True, sym=False, lib=lib), fx["expect"]["in_degrees_diag"], 1e-14,
           "in-degrees with A + I")
    for seed in range(3):
        g = random_small_graph(seed, N=40, E=150, K=3, weighted=True, sym=True)
        for diag, cor in ((False, False), (True, True)):
            a = orc.embed(g.src, g.dst, g.w, g.N, g.labels, g.K, diag=diag, lap=True, cor=cor, lib=lib)
            b = orc.embed(g.src, g.dst, g.w, g.N, g.labels, g.K, diag=diag, lap=True, cor=cor, deg_io=True,
                          lib=lib)
            _close(a, b, 1e-12, "in/out degrees on symmetric input")


def pin_closed_forms(lib):
    """P4: empty graph, complete graph, regular graph and star graph."""
    rng = np.random.default_rng(7)
    # (a) E = 0
    N, K = 40, 5
    lab = rng.integers(-1, K, size=N).astype(np.int32)
    nk = np.array([(lab == k).sum() for k in range(K)])
    e0 = np.zeros(0, dtype=np.int32)
    for d, l, c in FLAG_COMBOS:
        Z = orc.embed(e0, e0, None, N, lab, K, diag=d, lap=l, cor=c, lib=lib)
        R = np.zeros((N, K))
        if d:
            for i in range(N):
                if lab[i] >= 0:
                    R[i, lab[i]] = 1.0 if c else 1.0 / nk[lab[i]]
        _close(Z, R, 1e-14, f"empty graph opts={(d, l, c)}")
    # (b) complete graph, unweighted, options off: Z[i,k] = (n_k - [y_i = k]) / n_k
    N, K = 30, 3
    lab = np.array([i % K for i in range(N)], dtype=np.int32)
    lab[:4] = 0
    nk = np.array([(lab == k).sum() for k in range(K)], dtype=np.float64)
    iu, ju = np.triu_indices(N, 1)
    Z = orc.embed(iu.astype(np.int32), ju.astype(np.int32), None, N, lab, K, lib=lib)
    R = np.array([[(nk[k] - (lab[i] == k)) / nk[k] for k in range(K)] for i in range(N)])
    _close(Z, R, 1e-13, "complete graph")
    # (c) r-regular ring lattice (circulant, r = 6): Laplacian divides by r, and by r+1
    # with the diagonal added.
    N, r, K = 50, 6, 4
    src, dst = [], []
    for i in range(N):
        for off in range(1, r // 2 + 1):
            src.append(i)
            dst.append((i + off) % N)
    src = np.array(src, np.int32)
    dst = np.array(dst, np.int32)
    lab = rng.integers(0, K, size=N).astype(np.int32)
    w_plain = orc.embed(src, dst, None, N, lab, K, lib=lib)
    w_lap = orc.embed(src, dst, None, N, lab, K, lap=True, lib=lib)
    _close(w_lap, w_plain / r, 1e-13, "regular graph laplacian")
    w_dplain = orc.embed(src, dst, None, N, lab, K, diag=True, lib=lib)
    w_dlap = orc.embed(src, dst, None, N, lab, K, diag=True, lap=True, lib=lib)
    _close(w_dlap, w_dplain / (r + 1), 1e-13, "regular graph diag+laplacian")
    # (d) star: hub 0 with leaves 1..L; hub row holds (#leaves of class k) / n_k, and each
    # leaf row holds 1/n_{y_0} at the hub's class.
    L, K = 25, 3
    lab = np.array([1] + [k % K for k in range(L)], dtype=np.int32)
    N = L + 1
    nk = np.array([(lab == k).sum() for k in range(K)], dtype=np.float64)
    src = np.zeros(L, np.int32)
    dst = np.arange(1, L + 1, dtype=np.int32)
    Z = orc.embed(dst, src, None, N, lab, K, lib=lib)
    leaves = lab[1:]
    hub = [(leaves == k).sum() / nk[k] for k in range(K)]
    _close(Z[0], hub, 1e-13, "star hub")
    R = np.zeros((L, K))
    R[:, lab[0]] = 1.0 / nk[lab[0]]
    _close(Z[1:], R, 1e-13, "star leaves")


def pin_invariants(lib, g):
    """P3 on one graph g (any size): I1-I8."""
    K, N = g.K, g.N
    lab = g.labels
    # I1: class counts are exact and exclude unknown labels.
    nk = orc.class_counts(lab, K, lib=lib)
    assert int(nk.sum()) + int((lab < 0).sum()) == N, "I1 class counts"
    assert np.array_equal(nk, np.bincount(lab[lab >= 0], minlength=K)), "I1 bincount"
    # I2: unweighted, options off: Z[i,k] n_k is the number of class-k neighbours.
    Z = orc.embed(g.src, g.dst, None, N, lab, K, sym=g.sym, lib=lib)
    cnt = np.zeros((N, K))
    src = g.src.astype(np.int64)
    dst = g.dst.astype(np.int64)
    ls, ld = lab[src], lab[dst]
    m = ld >= 0
    np.add.at(cnt, (src[m], ld[m]), 1.0)
    if g.sym:
        m2 = (ls >= 0) & (src != dst)
        np.add.at(cnt, (dst[m2], ls[m2]), 1.0)
    scaled = Z * np.where(nk > 0, nk, 1)[None, :]
    assert np.max(np.abs(scaled - cnt)) < 1e-9, "I2 integer neighbour counts"
    # I3: options off: sum_i Z[i,k] = sum_{j in class k} colsum_j / n_k.
    Zw = orc.embed(g.src, g.dst, g.w, N, lab, K, sym=g.sym, lib=lib)
    wv = np.ones(g.E) if g.w is None else g.w.astype(np.float64)
    colsum = np.zeros(N)
    np.add.at(colsum, dst, wv)
    if g.sym:
        np.add.at(colsum, src[src != dst], wv[src != dst])
    expect = np.array([colsum[lab == k].sum() / nk[k] if nk[k] else 0.0 for k in range(K)])
    _close(Zw.sum(axis=0), expect, 1e-9, "I3 column sums")
    # I4: correlation rows have unit norm (or are zero).
    Zc = orc.embed(g.src, g.dst, g.w, N, lab, K, diag=True, lap=True, cor=True, sym=g.sym, lib=lib)
    nr = np.linalg.norm(Zc, axis=1)
    nz = nr > 0
    assert np.all(np.abs(nr[nz] - 1.0) < 1e-12), "I4 unit row norms"
    raw = orc.embed(g.src, g.dst, g.w, N, lab, K, diag=True, lap=True, sym=g.sym, lib=lib)
    assert np.array_equal(nz, np.linalg.norm(raw, axis=1) > 0), "I4 zero rows stay zero"
    # I5: symmetrize == explicit mirror rows without symmetrization.
    if g.sym:
        keep = g.src != g.dst
        s2 = np.concatenate([g.src, g.dst[keep]])
        d2 = np.concatenate([g.dst, g.src[keep]])
        w2 = None if g.w is None else np.concatenate([g.w, g.w[keep]])
        for d, l, c in ((False, False, False), (True, True, True)):
            a = orc.embed(g.src, g.dst, g.w, N, lab, K, diag=d, lap=l, cor=c, sym=True, lib=lib)
            b = orc.embed(s2, d2, w2, N, lab, K, diag=d, lap=l, cor=c, sym=False, lib=lib)
            _close(a, b, 1e-12, "I5 symmetrize vs mirrored rows")
    # I6: linearity with options off.
    h = g.E // 2
    w1 = None if g.w is None else g.w[:h]
    w2 = None if g.w is None else g.w[h:]
    za = orc.embed(g.src[:h], g.dst[:h], w1, N, lab, K, sym=g.sym, lib=lib)
    zb = orc.embed(g.src[h:], g.dst[h:], w2, N, lab, K, sym=g.sym, lib=lib)
    _close(Zw, za + zb, 1e-11, "I6 linearity")
    # I7: node permutation permutes rows; class relabelling permutes columns; row order
    # does not matter.
    rng = np.random.default_rng(11)
    perm = rng.permutation(N)
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N)
    lab_p = np.empty(N, dtype=np.int32)
    lab_p[perm] = lab
    zp = orc.embed(perm[g.src].astype(np.int32), perm[g.dst].astype(np.int32), g.w, N, lab_p, K,
                   diag=True, lap=True, cor=True, sym=g.sym, lib=lib)
    _close(zp[perm], Zc, 1e-11, "I7 node permutation")
    cperm = rng.permutation(K)
    lab_c = np.where(lab >= 0, cperm[np.maximum(lab, 0)], -1).astype(np.int32)
    zc = orc.embed(g.src, g.dst, g.w, N, lab_c, K, diag=True, lap=True, cor=True, sym=g.sym, lib=lib)
    _close(zc[:, cperm], Zc, 1e-11, "I7 class permutation")
    order = rng.permutation(g.E)
    zo = orc.embed(g.src[order], g.dst[order], None if g.w is None else g.w[order], N, lab, K,
                   diag=True, lap=True, cor=True, sym=g.sym, lib=lib)
    _close(zo, Zc, 1e-11, "I7 row order")


def pin_laplacian_symmetric(lib, seeds=range(3)):
    """I8: with one class per node (W = I), Z equals the normalized adjacency, which is
    symmetric for undirected input and equals D^-1/2 A D^-1/2 entrywise."""
    for seed in seeds:
        g = random_small_graph(seed, N=17, E=60, K=17, weighted=True, unknown_frac=0.0)
        lab = np.arange(g.N, dtype=np.int32)
        for diag in (False, True):
            Z = orc.embed(g.src, g.dst, g.w, g.N, lab, g.N, diag=diag, lap=True, sym=True, lib=lib)
            _close(Z, Z.T, 1e-13, "I8 symmetric normalized adjacency")
            deg = orc.degrees(g.src, g.dst, g.w, g.N, diag=diag, sym=True, lib=lib)
            A = np.zeros((g.N, g.N))
            for s, d, v in zip(g.src, g.dst, g.w):
                A[s, d] += v
                if s != d:
                    A[d, s] += v
            if diag:
                A += np.eye(g.N)
            dm = np.where(deg > 0, 1 / np.sqrt(np.abs(deg) + (deg <= 0)), 0)
            _close(Z, dm[:, None] * A * dm[None, :], 1e-12, "I8 entrywise")


def pin_degrees(lib, seeds=range(3)):
    """Row sums of A (+ I) against a direct loop."""
    for seed in seeds:
        for sym in (True, False):
            g = random_small_graph(seed, N=31, E=90, K=3, weighted=True, sym=sym)
            for diag in (False, True):
                deg = orc.degrees(g.src, g.dst, g.w, g.N, diag=diag, sym=sym, lib=lib)
                ref = np.zeros(g.N)
                for s, d, v in zip(g.src, g.dst, g.w.astype(np.float64)):
                    ref[s] += v
                    if sym and s != d:
                        ref[d] += v
                if diag:
                    ref += 1.0
                _close(deg, ref, 1e-12, "degrees")


def pin_sbm_statistics(lib, g, B_in, B_out):
    """P5: on an SBM with options off, the class-conditional mean of Z[i,k] equals
    B[y_i,k] (n_k - [y_i = k]) / n_k up to sampling error."""
    Z = orc.embed(g.src, g.dst, None, g.N, g.labels, g.K, sym=True, lib=lib)
    nk = np.bincount(g.labels, minlength=g.K).astype(np.float64)
    for a in range(g.K):
        rows = Z[g.labels == a]
        for k in range(g.K):
            p = B_in if a == k else B_out
            expect = p * (nk[k] - (a == k)) / nk[k]
            # per-row count is Binomial(n_k - [a=k], p); standard error of the mean of
            # count/n_k over n_a rows
            se = np.sqrt(p * (1 - p) * (nk[k] - (a == k))) / nk[k] / np.sqrt(len(rows))
            assert abs(rows[:, k].mean() - expect) < 6 * se + 1e-12, f"P5 block ({a},{k})"


ALL_CHEAP_PINS = ("pin_brute_force", "pin_hand_worked", "pin_closed_forms", "pin_laplacian_symmetric",
                  "pin_degrees", "pin_directed_degrees")
