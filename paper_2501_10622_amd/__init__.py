"""MI355X-native hot path of the CWT halo finder (arXiv:2501.10622).

Stages (HIP kernels in libhf.so, C ABI in include/hf.h): CIC deposit, grid CWT
by FFT (or by the paper's truncated real-space stencil), 26-neighbour maxima,
steepest-ascent segmentation, particle labels, the group statistics and
density filter that follow them, the cross-scale check, and the
identification loop over scales on one grid or on per-scale grids.
"""
from .hf import (  # noqa: F401
    CWT_BATCH_MAX, EXPORTS, HFError, LIB_PATH, NOALLOC_SCRATCH_BYTES, STENCIL_MAX_HALF_WIDTH, Context, context,
    cross_scale, cwt, cwt_batch, cwt_batch_ws_bytes, cwt_scales, cwt_stencil, deposit, find_halos, find_halos_async,
    find_halos_filtered_async, find_halos_group_async, find_halos_noalloc_async, find_halos_scales_async, groups,
    identify_async, identify_buffers, identify_grids_async, identify_grids_buffers, job_buffers, label, load_library,
    maxima, paper_grid, peaks, scales_buffers, segment, stencil_half_width, status_str, sync, unbind,
    workspace_size,
)
