"""MI355X-native single-scale hot path of the CWT halo finder (arXiv:2501.10622).

Stages (HIP kernels in libhf.so, C ABI in include/hf.h): CIC deposit, grid CWT
by FFT, 26-neighbour maxima, steepest-ascent segmentation, particle labels.
"""
from .hf import (  # noqa: F401
    EXPORTS, HFError, LIB_PATH, Context, context, cwt, deposit, find_halos, label, load_library, maxima,
    segment, status_str, sync, workspace_size,
)
