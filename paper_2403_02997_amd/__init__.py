"""Cover-edge triangle counting on AMD Instinct MI355X (gfx950).

Method: Bader, Li, Du et al., "Cover Edge-Based Novel Triangle Counting"
(arXiv 2403.02997): BFS levels restarted per component, the horizontal (same-level)
edges as cover-edge set, and one sorted-list intersection per cover edge with the
paper's level/order rule.  The kernels live in ``csrc/`` and are reached through the
C ABI of ``include/tc.h``; :mod:`.tc` is the Python binding with the same names, and
:mod:`.autotune` picks the intersection class thresholds on the caller's own input.
"""
from .tc import (  # noqa: F401
    EXPORTS,
    NOALLOC_SCRATCH_BYTES,
    Server,
    ServeResult,
    Stats,
    TCError,
    as_u64,
    load,
    tc_count,
    tc_count_batch,
    tc_count_batch_noalloc,
    tc_count_batch_workspace_size,
    tc_count_ex,
    tc_count_per_vertex,
    tc_count_split,
    tc_local_clustering,
    tc_get_forward_threshold,
    tc_get_hub_params,
    tc_get_isect_params,
    tc_last_call_info,
    tc_profile_enable,
    tc_profile_read,
    tc_set_forward_threshold,
    tc_set_hub_params,
    tc_set_isect_params,
    tc_validate_csr,
    tc_version,
    to_device,
)
