"""Seeded synthetic input graphs shared by the oracle side and the device side.

This package only draws random numbers and turns them into edge lists.  It
holds none of the pattern-mining arithmetic: no CSR canonicalisation beyond
what a generator's own stopping rule needs, no orientation, no counting.

Every random number comes from one counter-based generator (splitmix64 over a
counter, Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), evaluated with numpy uint64 arithmetic, so that a
(seed, stream) pair yields the same bytes on every machine.
"""
from .rng import splitmix64, stream_u64, stream_uniform
from .graphs import (
    EdgeList,
    BatchEdgeLists,
    erdos_renyi,
    rmat,
    rgg_batch,
    complete_graph,
    star_graph,
    cycle_graph,
    path_graph,
    complete_bipartite,
    complete_multipartite,
    relabel,
    disjoint_union,
)

__all__ = [
    "splitmix64", "stream_u64", "stream_uniform",
    "EdgeList", "BatchEdgeLists", "erdos_renyi", "rmat", "rgg_batch",
    "complete_graph", "star_graph", "cycle_graph", "path_graph",
    "complete_bipartite", "complete_multipartite", "relabel", "disjoint_union",
]
