"""The paper's own design on the CPU: sparse GEE as scipy.sparse CSR matrices and sparse
products (Section 3; Table 1's formulas with A, D, I and W all sparse).

TEST INFRASTRUCTURE ONLY. It is a second CPU route, written independently of the C edge
loop in gee_oracle.c (library sparse products instead of a loop over the entries): the
tests pin the oracle against it, and the benchmark's CPU-baseline leg times it as the
paper's design on the host. The product path never imports it.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def scipy_route(src, dst, w, N, labels, K, diag, lap, cor, sym, deg_io=False):
    """The paper's own library design: CSR matrices and sparse products (Section 3).
    `deg_io`: the Laplacian as D_out^-1/2 A D_in^-1/2 (row sums left, column sums right)."""
    E = len(src)
    wv = np.ones(E) if w is None else np.asarray(w, dtype=np.float64)
    A = sp.coo_matrix((wv, (np.asarray(src), np.asarray(dst))), shape=(N, N)).tocsr()
    A.sum_duplicates()
    if sym:
        A = (A + A.T - sp.diags(A.diagonal())).tocsr()
    if diag:
        A = (A + sp.identity(N, format="csr")).tocsr()
    if lap:
        def inv_sqrt(d):
            out = np.zeros(N)
            pos = d > 0
            out[pos] = 1.0 / np.sqrt(d[pos])
            return out

        Dl = sp.diags(inv_sqrt(np.asarray(A.sum(axis=1)).ravel()))
        Dr = sp.diags(inv_sqrt(np.asarray(A.sum(axis=0)).ravel())) if deg_io else Dl
        A = (Dl @ A @ Dr).tocsr()
    lab = np.asarray(labels)
    nk = np.bincount(lab[lab >= 0], minlength=K).astype(np.float64)
    rows = np.flatnonzero(lab >= 0)
    W = sp.csr_matrix((1.0 / nk[lab[rows]], (rows, lab[rows])), shape=(N, K))
    Z = (A @ W).toarray()
    if cor:
        nr = np.sqrt((Z * Z).sum(axis=1))
        pos = nr > 0
        Z[pos] /= nr[pos, None]
    return Z
