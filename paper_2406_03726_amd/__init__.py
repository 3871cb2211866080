"""MI355X-native sparse Graph Encoder Embedding (Qin & Shen, Sections 2-3).

The hot path (edge list -> CSR -> degrees -> Laplacian rescale -> per-row class
scatter -> correlation) runs in hand-written HIP kernels for gfx950 behind the C ABI
of include/gee.h (libgee.so); this package is the thin Python binding over it.
"""

from .gee import (  # noqa: F401
    BatchPlan,
    GEE_CORRELATION,
    GEE_DATA_CSR,
    GEE_DATA_INDEX,
    GEE_DATA_INTERNAL,
    GEE_DATA_LABEL,
    GEE_DATA_WEIGHT,
    GEE_DIAG,
    GEE_ERR_WORKSPACE,
    GEE_DIRECTED_DEGREES,
    GEE_LAPLACIAN,
    GEE_NO_VALIDATE,
    GEE_SYMMETRIZE,
    GeeError,
    flags_of,
    gee_abi_version,
    gee_build_csr,
    gee_build_csr_workspace_bytes,
    gee_class_counts,
    gee_csr_capacity,
    gee_default_schedule,
    gee_embed,
    gee_embed_atomic,
    gee_embed_atomic_workspace_bytes,
    gee_embed_sparse,
    gee_embed_sparse_workspace_bytes,
    gee_embed_batch,
    gee_embed_batch_workspace_bytes,
    gee_embed_csr,
    gee_embed_csr_workspace_bytes,
    gee_embed_workspace_bytes,
    gee_embed_noalloc,
    gee_scratch_bytes,
    gee_get_data_errors,
    gee_take_data_errors_async,
    gee_init,
    schedule,
)
