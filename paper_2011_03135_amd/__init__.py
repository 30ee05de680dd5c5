"""MI355X (gfx950) graph pattern mining: Python binding of libgpmhip.so.

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory (caller-owned buffers) and the stream.  The
binding raises if the built library is missing; there is no fallback.

    import paper_2011_03135_amd as gpm
    g = gpm.Graph.build(n, u, v)            # u, v: int32 CUDA tensors
    gpm.count(g, gpm.clique(4))             # exact int
    gpm.motif_count(g, 4)                   # 6 induced 4-motif counts
    gpm.motif_count_enum(g, 5)              # 21 induced 5-motif counts
"""
from .binding import (  # noqa: F401
    GpmError,
    Graph,
    Pattern,
    BatchConfig,
    batch_autotune,
    batch_default_config,
    batch_motif_count,
    batch_motif_count_static,
    clique,
    clique_counts,
    count,
    diamond,
    cycle4,
    library_path,
    list_embeddings,
    matching_order,
    load,
    motif_count,
    motif_classes,
    motif_class_pattern,
    motif_count_enum,
    motif_count_formula,
    motif_formula_workspace_bytes,
    motif_enum_workspace_bytes,
    motif_workspace_bytes,
    pattern,
    timing_enable,
    timing_read,
    workspace_bytes,
    ORIENT_DEGREE,
    ORIENT_CORE,
    MOTIF3_NAMES,
    MOTIF4_NAMES,
    VERTEX_INDUCED,
    EDGE_INDUCED,
    LIST,
)
