"""Ray reordering and closest-hit tracing on AMD Instinct MI355X (gfx950).

A from-scratch HIP implementation of the data-parallel path of Meister et al.,
"On Ray Reordering Techniques for Faster GPU Ray Tracing" (I3D 2020): sort
keys (the layouts of the paper's key figure, Two Point with fixed, adaptive
and real termination estimates), a stable key/index radix sort, the ray
gather and a closest-hit BVH trace, behind the C ABI of include/rr.h.  The
Python layer only marshals arguments; PyTorch supplies device memory and
streams.
"""
from .rr import (  # noqa: F401
    EXPORTS, KeyParams, RRError, Scene,
    RR_KEY_NONE, RR_KEY_ORIGIN_DIRECTION, RR_KEY_ORIGIN_TERMINATION, RR_KEY_ORIGIN, RR_KEY_DIRECTION_ORIGIN,
    RR_KEY_AILA, RR_KEY_AILA_COMPACT, RR_KEY_OCTAHEDRON, RR_KEY_TWO_POINT_ADAPTIVE, RR_KEY_TWO_POINT_REAL,
    RR_LENGTH_CELLS, RR_HITS_ORIGINAL_ORDER, RR_INDIRECT, RR_LOCAL_SORT_1024, RR_LOCAL_SORT_2048,
    RR_LOCAL_SORT_4096, RR_ANY_HIT, RR_SORT_MSD, LengthTable,
    coherence_m64, hits_to_numpy, key_params, keys_workspace_size, load, reorder_workspace_size, sort_workspace_size,
    rr_compute_keys, rr_sort, rr_local_sort, rr_gather, rr_scatter_hits, rr_trace, rr_trace_any, rr_trace_profile, rr_reorder_and_trace, rr_reorder_and_trace_noalloc,
    workspace,
)
from .batch import (  # noqa: F401
    EXTRA_EXPORTS, RR_BATCH_EAGER, RR_TILES_COUNTER, RR_TILES_FIXED, Batch, Server, load_tuned, save_tuned, segment,
    tuning_db_path,
)
