"""Seeded synthetic graph workloads for the sparse GEE hot path.

This package only draws inputs: edge lists, edge weights, node labels and the
per-graph option choices. It holds none of the embedding arithmetic, so both the
FP64 oracle and the HIP path can consume the same inputs without sharing code.

Every generator takes an explicit ``numpy.random.Generator``; ``rng_for`` builds
the canonical one for a (config, graph) pair.
"""

from .generators import (  # noqa: F401
    Graph,
    rng_for,
    iid_labels,
    zipf_labels,
    uniform_weights,
    sbm_edges,
    chung_lu_edges,
    chung_lu_expected_degrees,
    shuffle_and_orient,
    sbm_expected_edges,
    edge_density,
)
from .configs import (  # noqa: F401
    CONFIG_NAMES,
    sbm_small,
    sbm_dense,
    powerlaw_10m,
    batched_graphs,
    serving_pool,
    random_small_graph,
)
