"""Pins for the oracle's cross-scale maximum check (step 8).

A brute force walks the 27 periodic neighbours with explicit index arithmetic.
The Gaussian blob fixes the outcome from its closed-form CWT: at the blob's
centre C(w) is proportional to w^1.5 (1 + w^2 s^2 / 2)^(-5/2) (the transform
of Eq. (4) times the Gaussian's), which rises with w up to w* = sqrt(6/7)/s and
falls beyond; so the centre is a maximum across scale against a smaller scale
(larger w) exactly when both scales lie above w*.
"""
import math

import numpy as np
import pytest

from oracle import cwthf as O


def _brute(cs, cm, roots):
    n = cs.shape[0]
    out = []
    for r in roots:
        z, y, x = r // (n * n), (r // n) % n, r % n
        best = max(cm[(z + dz) % n, (y + dy) % n, (x + dx) % n]
                   for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
        out.append(bool(cs[z, y, x] > best))
    return out


@pytest.mark.parametrize("seed,n", [(1, 8), (2, 9), (3, 12)])
def test_matches_brute_force(seed, n):
    rng = np.random.default_rng(seed)
    cm = rng.normal(size=(n, n, n))
    cs = cm + rng.normal(scale=0.7, size=(n, n, n))
    roots = O.maxima(cs, -np.inf)
    got = O.cross_scale(cs, cm, roots)
    assert got.tolist() == _brute(cs, cm, roots)
    assert got.any() and not got.all()


def test_strict_and_same_field():
    rng = np.random.default_rng(4)
    c = rng.normal(size=(8, 8, 8))
    roots = O.maxima(c, -np.inf)
    # a maximum equals itself at the other scale: never strictly above
    assert not O.cross_scale(c, c, roots).any()
    assert O.cross_scale(c + 1e-9, c, roots).all()


def _centre_value(w, s):
    return w ** 1.5 * (1 + w * w * s * s / 2) ** -2.5


@pytest.mark.parametrize("a_large,a_small,expect", [
    (4.0, 3.0, False),   # both scales below w* (coarser than the blob): the response still grows
    (3.0, 2.5, False),
    (1.5, 1.0, True),    # both above w*: the centre beats the finer scale everywhere near it
    (1.2, 1.0, True),
])
def test_gaussian_blob_closed_form(a_large, a_small, expect):
    n, s, centre = 64, 2.0, (30, 31, 33)
    g = np.arange(n)
    d = lambda c0: ((g - c0 + n // 2) % n - n // 2).astype(float)
    r2 = d(centre[0])[:, None, None] ** 2 + d(centre[1])[None, :, None] ** 2 + d(centre[2])[None, None, :] ** 2
    f = np.exp(-r2 / (2 * s * s))
    w1, w2 = 1.0 / a_large, 1.0 / a_small
    wstar = math.sqrt(6.0 / 7.0) / s
    assert (min(w1, w2) > wstar) if expect else (max(w1, w2) < wstar)  # the case is the one named
    assert (_centre_value(w1, s) > _centre_value(w2, s)) == expect
    c1 = O.cwt_field(f, float(n), w1, "sampled")
    c2 = O.cwt_field(f, float(n), w2, "sampled")
    root = (centre[0] * n + centre[1]) * n + centre[2]
    assert root in set(O.maxima(c1).tolist())
    assert O.cross_scale(c1, c2, [root]).tolist() == [expect]
