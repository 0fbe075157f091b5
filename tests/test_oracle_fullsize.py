"""Pins for the oracle pieces that serve the full-size (1024^3) parity checks.

- The C deposit (oracle/cic.c) equals the NumPy deposit bit for bit (itself
  pinned by mass conservation, textbook cases and brute force) on clustered
  boxes with FP32 and FP64 positions, positions outside the box, several B and
  any split into plane ranges; it conserves mass exactly, reports the exact
  2^63 overflow boundary and bad positions.
- ``is_maximum_at`` and ``follow`` are ``maxima`` and ``segment`` evaluated at
  chosen cells: on whole small fields they give exactly the same sets and
  labels, including engineered ties and signed zeros.
- The stencil evaluated at single cells with a half-width of 12 scale lengths
  equals the FFT oracle's sampled transform to 1e-10 of its peak, so the
  full-size CWT check may use it as the FFT path's reference.
"""
import math

import numpy as np
import pytest

import synth
from oracle import cic
from oracle import cwthf as O


@pytest.mark.parametrize("n,L,np_,dtype,bits,threads", [
    (32, 40.0, 60000, "f32", 15, 1), (48, 60.0, 200000, "f32", 12, 5), (64, 100.0, 300000, "f64", 15, 8),
    (24, 30.0, 50000, "f64", 17, 3), (16, 16.0, 20000, "f32", 8, 16)])
def test_c_deposit_equals_numpy(n, L, np_, dtype, bits, threads):
    pos = synth.make_box(L, np_, 40, dtype, n + bits).numpy()
    pos[:100] += L * np.array([1.0, -2.0, 3.0], dtype=pos.dtype)  # outside the box: wraps
    want = O.deposit(pos, L, n, bits)
    got = cic.deposit_c(pos, L, n, bits, threads=threads)
    assert np.array_equal(got, want)
    assert O.total_mass(got) == np_ << (3 * bits)


def test_c_deposit_overflow_and_bad_input():
    rho = cic.deposit_c(np.zeros((7, 3)), 8.0, 8, 20)
    assert rho[0, 0, 0] == 7 * (1 << 60)
    with pytest.raises(O.DepositOverflow):
        cic.deposit_c(np.zeros((8, 3)), 8.0, 8, 20)
    with pytest.raises(O.DepositOverflow):
        cic.deposit_c(np.zeros((8, 3), np.float32), 8.0, 8, 20, threads=4)
    with pytest.raises(ValueError):
        cic.deposit_c(np.array([[0.0, np.nan, 0.0]], np.float32), 8.0, 8, 15)
    with pytest.raises(ValueError):
        cic.deposit_c(np.array([[0.0, 0.0, np.inf]]), 8.0, 8, 15, threads=2)


def _field(seed, n, ties=False):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(n, n, n)).astype(np.float32)
    if ties:  # plateaus of equal values and signed zeros exercise the index tie-break
        c = np.round(c * 2) / 2
        c[c == 0] = np.where(rng.random((c == 0).sum()) < 0.5, -0.0, 0.0)
    return c


@pytest.mark.parametrize("seed,n,ties,tau", [(1, 8, False, 0.0), (2, 12, True, 0.0), (3, 16, True, -0.5),
                                             (4, 10, False, 0.3)])
def test_pointwise_maxima_and_paths_equal_whole_field(seed, n, ties, tau):
    c = _field(seed, n, ties)
    cells = np.arange(n ** 3)
    assert np.flatnonzero(O.is_maximum_at(c, cells, tau)).tolist() == O.maxima(c, tau).tolist()
    assert O.follow(c, cells, tau).tolist() == O.segment(c, tau).ravel().tolist()
    some = np.random.default_rng(seed).integers(0, n ** 3, 50)
    assert O.follow(c, some, tau).tolist() == O.segment(c, tau).ravel()[some].tolist()


@pytest.mark.parametrize("a", [1.0, 2.0])
def test_stencil_at_twelve_scale_lengths_is_the_sampled_transform(a):
    n, L = 64, 64.0
    pos = synth.make_box(L, 200000, 80, "f32", 11).numpy()
    rho = O.deposit(pos, L, n)
    kw = n / (1000.0 * a)
    full = O.cwt(rho, L, kw)
    h = int(math.ceil(12 * a))
    cells = np.concatenate([np.argsort(full.ravel())[-16:], np.random.default_rng(2).integers(0, n ** 3, 48)])
    got = O.stencil_cwt_at(rho, L, kw, h, cells)
    assert np.max(np.abs(got - full.ravel()[cells])) <= 1e-10 * np.abs(full).max()
