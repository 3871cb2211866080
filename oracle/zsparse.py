"""Sparse storage of the embedding matrix (test infrastructure only).

The paper keeps the embedding matrix in CSR (Section 3 layout: ``index_pointers`` of
length R + 1, then for each row in turn the column indices and the data values of its
non-zero entries). For Z that means: row i lists the classes k with Z[i, k] != 0, in
increasing k, with their values. This is that definition written out over a dense Z
(as the oracle's ``embed`` returns it); no entry order beyond row-major is involved.
"""

from __future__ import annotations

import numpy as np


def sparse_rows(Z):
    """(row_ptr int64[N+1], col int64[nnz], val[nnz]) of the non-zero entries of Z, row by
    row with classes increasing. An entry equal to zero (also -0.0) is not stored."""
    Z = np.asarray(Z)
    keep = Z != 0
    row_ptr = np.zeros(Z.shape[0] + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=row_ptr[1:])
    rows, cols = np.nonzero(keep)  # row-major order for a C-ordered array
    return row_ptr, cols.astype(np.int64), Z[rows, cols]


def dense_of(row_ptr, col, val, N: int, K: int):
    """The dense N x K matrix of a sparse storage (the inverse of ``sparse_rows``)."""
    Z = np.zeros((N, K), dtype=np.asarray(val).dtype if len(val) else np.float64)
    for i in range(N):
        Z[i, col[row_ptr[i]:row_ptr[i + 1]]] = val[row_ptr[i]:row_ptr[i + 1]]
    return Z
