"""FP64 CPU oracle for the sparse GEE hot path.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package; the product path never does. It shares
no code with the HIP implementation.

* ``embed``        - Z of Eq. (1) with the Section 2 / Table 1 options (C, float64).
* ``class_counts`` - exact integer n_k (C).
* ``degrees``      - row sums of A (or A + I), float64 (C).
* ``csr``          - the canonical CSR of an edge list (numpy stable sort).
* ``sparse_rows``  - Z in sparse storage (its non-zero entries in the Section 3 CSR layout).
"""

from .oracle import (  # noqa: F401
    build_oracle,
    class_counts,
    degrees,
    embed,
    embed_graph,
    lib_path,
)
from .csr_ref import csr, csr_graph  # noqa: F401
from .zsparse import dense_of, sparse_rows  # noqa: F401
