"""Shared helpers for the GPU parity tests (inputs, tolerances, tie certification)."""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cwthf as O  # noqa: E402
import synth  # noqa: E402

# FP32 CWT against the FP64 oracle: max |C32 - C64| <= 1e-5 max |C64|.
CWT_RTOL = 1e-5
# particle-label agreement required when the input is not certified tie-free
LABEL_AGREEMENT = 0.9999


def ensure_built():
    from paper_2501_10622_amd import hf
    if not os.path.exists(hf.LIB_PATH):
        from paper_2501_10622_amd import build
        build.build(verbose=False)


def cuda(t):
    return torch.as_tensor(t).cuda()


def small_box(n, box_len, np_, n_halos, dtype, seed):
    return synth.make_box(box_len, np_, n_halos, dtype, seed).numpy()


def cwt_error(c32, c64):
    return float(np.max(np.abs(c32.astype(np.float64) - c64)) / np.max(np.abs(c64)))


def tie_free(c64, eps, tau=0.0):
    """True if every pair of 26-neighbours differs by more than 2 eps and every
    local maximum is more than 2 eps from tau: then an FP32 field within eps of
    c64 orders every comparison the maxima and segmentation make the same way."""
    for (dz, dy, dx) in O.neighbour_offsets()[:13]:  # each unordered pair once
        nb = np.roll(c64, (-dz, -dy, -dx), axis=(0, 1, 2))
        if np.any(np.abs(c64 - nb) <= 2 * eps):
            return False
    mx = O.maxima(c64, -np.inf)  # every root, above tau or not
    return not np.any(np.abs(c64.ravel()[mx] - tau) <= 2 * eps)
