"""Pins for the oracle's real-space truncated-stencil CWT (Sec. 2.1; Table 1's
gdw_resolution, kept at its physical extent on the paper's grid N_g).

- On the paper's own grid the default half-width is Table 1's count; on any
  grid it spans at least ten scale lengths, and the stencil then sums to zero
  (the Mexican hat's zero mean) to 1e-7 of its peak at the 1024^3 box's
  scales, where Table 1's count taken in the box's cells leaves a sum 21.6 and
  661 times the peak (a = 2 and 4 cells).  The sums use the one-dimensional
  factorisation, not the oracle's stencil.

- A pure-Python gather over every (target, source) pair and every stencil
  offset congruent to their separation fixes the direction of the shifts, the
  periodic wrap and the double counting of a stencil wider than the box.
- A stencil wide enough to hold the wavelet reproduces the FFT oracle (itself
  pinned by brute force), through entirely different code.
- A uniform field gives the stencil's sum everywhere, which for a cube of
  offsets factorises into one-dimensional sums (a closed form the oracle does
  not use).
- A unit point gives the stencil itself and nothing outside it.
"""
import math

import numpy as np
import pytest

from oracle import cwthf as O


@pytest.mark.parametrize("kw,h", [(0.1, 20), (2.5, 5), (0.5, 8), (1.0, 6), (1.5, 6), (0.3, 10)])
def test_gdw_resolution_table1(kw, h):
    # Int(1.5 / k_w + 5); the two ends of Table 1's k_w range give 20 and 5
    assert O.gdw_resolution(kw) == h


@pytest.mark.parametrize("kw", [0.1, 0.2, 0.35, 0.5, 1.0, 2.5])
def test_default_half_width_on_the_paper_grid_is_table1(kw):
    ng = int(400.0 * kw + 150.0)  # the flowchart's N_g
    assert O.paper_grid(kw) == ng
    assert O.stencil_half_width(kw, ng) == O.gdw_resolution(kw)


def _stencil_sum_over_peak(n, box_len, kw, h):
    # sum over the cube |d_i| <= h of dx^3 Psi(w, d dx), Psi = w^1.5 (6 - u) e^(-u/4)
    # with u = w^2 r^2, factorises into 1D sums: 6 G^3 - 3 G^2 H, G = sum e^(-u_d/4),
    # H = sum u_d e^(-u_d/4); the peak tap is 6 dx^3 w^1.5
    w = 1000.0 * kw / box_len
    u = (w * np.arange(-h, h + 1) * (box_len / n)) ** 2
    G, H = np.sum(np.exp(-u / 4)), np.sum(u * np.exp(-u / 4))
    return (6 * G ** 3 - 3 * G * G * H) / 6.0


@pytest.mark.parametrize("a,h_expect,raw_sum", [(1.0, 11, 2.9e-3), (2.0, 21, 21.6), (4.0, 41, 661.5)])
def test_default_stencil_keeps_zero_mean_at_the_1024_box(a, h_expect, raw_sum):
    n, box_len = 1024, 1000.0
    kw = n / (1000.0 * a)
    h = O.stencil_half_width(kw, n)
    assert h == h_expect
    assert h * (1000.0 * kw / box_len) * (box_len / n) >= 10.0  # at least ten scale lengths
    assert abs(_stencil_sum_over_peak(n, box_len, kw, h)) < 1e-7
    raw = _stencil_sum_over_peak(n, box_len, kw, O.gdw_resolution(kw))
    assert raw == pytest.approx(raw_sum, rel=2e-2)


@pytest.mark.parametrize("n,kw", [(64, 0.02), (96, 0.05), (256, 0.1), (512, 0.3), (1024, 0.8), (150, 0.0)])
def test_default_half_width_spans_ten_scale_lengths(n, kw):
    if kw == 0.0:  # the paper's smallest grid at its largest default scale
        kw, n = 0.1, 190
    h = O.stencil_half_width(kw, n)
    a_cells = n / (1000.0 * kw)
    assert h / a_cells >= 10.0
    assert (h - 1) / a_cells < 12.2  # and not much more (ceil of at most 12 scale lengths)


def _brute(f, box_len, w, h):
    n = f.shape[0]
    dx = box_len / n
    out = np.zeros_like(f)
    rng = range(-h, h + 1)
    for jz in range(n):
        for jy in range(n):
            for jx in range(n):
                acc = 0.0
                for gz in range(n):
                    for gy in range(n):
                        for gx in range(n):
                            fg = f[gz, gy, gx]
                            if fg == 0.0:
                                continue
                            for dz in rng:
                                if (jz - gz - dz) % n:
                                    continue
                                for dy in rng:
                                    if (jy - gy - dy) % n:
                                        continue
                                    for dxo in rng:
                                        if (jx - gx - dxo) % n:
                                            continue
                                        r2 = (dz * dz + dy * dy + dxo * dxo) * dx * dx
                                        u = w * w * r2
                                        acc += fg * dx ** 3 * w ** 1.5 * (6.0 - u) * math.exp(-u / 4.0)
                out[jz, jy, jx] = acc
    return out


@pytest.mark.parametrize("n,h,seed", [(4, 1, 0), (5, 2, 1), (4, 3, 2), (3, 2, 3)])
def test_matches_brute_force_gather(n, h, seed):
    # (4, 3) and (3, 2): the stencil is wider than the box and wraps onto itself
    rng = np.random.default_rng(seed)
    f = rng.random((n, n, n)) * (rng.random((n, n, n)) < 0.6)
    box_len, w = 7.0, 0.9
    np.testing.assert_allclose(O.stencil_cwt_field(f, box_len, w, h), _brute(f, box_len, w, h),
                               rtol=1e-12, atol=1e-12 * np.abs(f).sum())


@pytest.mark.parametrize("n,a_cells,h", [(24, 1.2, 11), (32, 1.5, 15)])
def test_wide_stencil_equals_fft_oracle(n, a_cells, h):
    # beyond h cells the wavelet is below exp(-(h/a)^2/4) ~ 1e-11 of its peak
    rng = np.random.default_rng(n)
    f = rng.gamma(0.5, size=(n, n, n))
    box_len = 100.0
    w = n / (a_cells * box_len)
    c_st = O.stencil_cwt_field(f, box_len, w, h)
    c_fft = O.cwt_field(f, box_len, w)
    assert np.abs(c_st - c_fft).max() <= 1e-8 * np.abs(c_fft).max()


@pytest.mark.parametrize("n,h,a_cells", [(8, 3, 0.46), (10, 2, 1.0), (12, 5, 2.0)])
def test_uniform_field_is_the_factorised_stencil_sum(n, h, a_cells):
    box_len = 50.0
    dx = box_len / n
    w = 1.0 / (a_cells * dx)
    c = O.stencil_cwt_field(np.ones((n, n, n)), box_len, w, h)
    # the cube sum of (6 - u_x - u_y - u_z) e^{-(u_x + u_y + u_z)/4}
    u = [(w * d * dx) ** 2 for d in range(-h, h + 1)]
    g = sum(math.exp(-x / 4.0) for x in u)
    hh = sum(x * math.exp(-x / 4.0) for x in u)
    expect = dx ** 3 * w ** 1.5 * (6.0 * g ** 3 - 3.0 * g * g * hh)
    np.testing.assert_allclose(c, expect, rtol=1e-12, atol=1e-14 * abs(6.0 * g ** 3) * dx ** 3 * w ** 1.5)


def test_unit_point_is_the_stencil_and_nothing_else():
    n, h, box_len, kw = 16, 3, 20.0, 0.4
    rho = np.zeros((n, n, n), dtype=np.int64)
    rho[5, 9, 14] = 1 << 45
    c = O.stencil_cwt(rho, box_len, kw, h)
    w = O.scale_w(kw, box_len)
    s = O.stencil(n, box_len, w, h) * n ** 3  # f = n^3 at the point
    idx = np.ix_([(5 + d) % n for d in range(-h, h + 1)], [(9 + d) % n for d in range(-h, h + 1)],
                 [(14 + d) % n for d in range(-h, h + 1)])
    np.testing.assert_allclose(c[idx], s, rtol=1e-13)
    mask = np.ones_like(c, dtype=bool)
    mask[idx] = False
    assert (c[mask] == 0.0).all()
    # the centre holds 6 dx^3 w^1.5 n^3: Eq. (4) at r = 0
    assert c[5, 9, 14] == pytest.approx(6.0 * (box_len / n) ** 3 * w ** 1.5 * n ** 3, rel=1e-14)


def test_translation_equivariance_and_linearity():
    rng = np.random.default_rng(5)
    n, h, box_len, w = 12, 4, 30.0, 0.5
    f = rng.random((n, n, n))
    g = rng.random((n, n, n))
    c = O.stencil_cwt_field(f, box_len, w, h)
    shifted = O.stencil_cwt_field(np.roll(f, (3, -5, 7), axis=(0, 1, 2)), box_len, w, h)
    np.testing.assert_allclose(shifted, np.roll(c, (3, -5, 7), axis=(0, 1, 2)), rtol=1e-12, atol=1e-12)
    both = O.stencil_cwt_field(2.0 * f - g, box_len, w, h)
    np.testing.assert_allclose(both, 2.0 * c - O.stencil_cwt_field(g, box_len, w, h), rtol=1e-11, atol=1e-11)


def test_default_half_width_and_normalisation():
    rng = np.random.default_rng(9)
    n, box_len, kw = 12, 40.0, 0.9
    rho = rng.integers(0, 1 << 40, size=(n, n, n))
    c = O.stencil_cwt(rho, box_len, kw)
    f = rho / (rho.sum() / n ** 3)
    h = O.stencil_half_width(kw, n)
    assert h == 1  # Int(1.5 / 0.9 + 5) = 6 cells of N_g = 510 cover 0.14 of these 12 cells
    np.testing.assert_allclose(c, O.stencil_cwt_field(f, box_len, O.scale_w(kw, box_len), h),
                               rtol=1e-13, atol=1e-13)
    with pytest.raises(ValueError):
        O.stencil_cwt(rho, box_len, kw, -1)


@pytest.mark.parametrize("n,h", [(10, 3), (6, 4)])
def test_pointwise_windows_equal_the_superposition(n, h):
    # (6, 4): 2h + 1 = 9 > 6, so windows repeat cells, as the wrapped stencil does
    rng = np.random.default_rng(n + h)
    rho = rng.integers(0, 1 << 44, size=(n, n, n)) * (rng.random((n, n, n)) < 0.7)
    box_len, kw = 25.0, 0.35
    full = O.stencil_cwt(rho, box_len, kw, h)
    cells = np.arange(n ** 3)
    np.testing.assert_allclose(O.stencil_cwt_at(rho, box_len, kw, h, cells), full.ravel(), rtol=1e-12,
                               atol=1e-12 * np.abs(full).max())


def test_cwt_stencil_mode_is_the_stencil_with_table1_extent():
    rng = np.random.default_rng(11)
    n, box_len, kw = 24, 20.0, 0.05  # Int(30 + 5) = 35 cells of N_g = 170: ceil(35 * 24 / 170) = 5
    rho = rng.integers(0, 1 << 40, size=(n, n, n))
    np.testing.assert_array_equal(O.cwt(rho, box_len, kw, "stencil"), O.stencil_cwt(rho, box_len, kw, 5))
