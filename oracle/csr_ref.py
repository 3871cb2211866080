"""Canonical CSR of an edge list (test infrastructure only).

Section 3 fixes the CSR layout: ``index_pointers`` of length R + 1, and for each row
in turn the column indices and the data values of its non-zero entries. The paper does
not fix the order of the entries inside a row; the reading used here is that row i lists
the other endpoint of every edge row touching i in increasing input row index, the row
itself (A[s, d]) before its mirror (A[d, s]) under symmetrization, a self-loop once, and
the data value being the untouched input weight. That order is exactly a stable sort by
row of the entry sequence fwd(0), rev(0), fwd(1), rev(1), ...; a stable library sort is
used for it.
"""

from __future__ import annotations

import numpy as np


def csr(src, dst, w, N: int, sym: bool = True):
    """Return (row_ptr int32[N+1], col int32[M], val float32[M] or None)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    E = src.shape[0]
    if sym:
        rows = np.empty(2 * E, dtype=np.int64)
        cols = np.empty(2 * E, dtype=np.int64)
        rows[0::2] = src
        rows[1::2] = dst
        cols[0::2] = dst
        cols[1::2] = src
        keep = np.ones(2 * E, dtype=bool)
        keep[1::2] = src != dst  # a self-loop appears once
        eidx = np.repeat(np.arange(E), 2)
        rows, cols, eidx = rows[keep], cols[keep], eidx[keep]
    else:
        rows, cols, eidx = src, dst, np.arange(E)
    order = np.argsort(rows, kind="stable")
    counts = np.bincount(rows, minlength=N) if rows.size else np.zeros(N, dtype=np.int64)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[order].astype(np.int32)
    val = None
    if w is not None:
        val = np.asarray(w, dtype=np.float32)[eidx[order]]
    return row_ptr.astype(np.int32), col, val


def csr_graph(g):
    return csr(g.src, g.dst, g.w, g.N, sym=g.sym)
