"""Pins for the oracle's grid CWT (Eqs. (2)-(4), Sec. 2.1).

The wavelet and its transform are pinned by mathematics that does not reuse the
oracle's formulas: the Fourier pair by radial quadrature, the zero mean that a
positive peak with a negative ring requires, the paper's statement that the
wavelet comes from a w-derivative of a Gaussian, and the closed-form CWT of a
Gaussian blob.  The FFT convolution is pinned by an O(N^6) brute-force sum.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import cwthf as O


def test_fourier_pair_by_quadrature():
    for w in (0.7, 2.3):
        for k in (0.2 * w, w, 1.9 * w):
            f = lambda r: float(O.wavelet(w, r * r)) * 4 * math.pi * r * r * math.sin(k * r) / (k * r)
            val, _ = integrate.quad(f, 0.0, 40.0 / w, limit=400, epsabs=0, epsrel=1e-12)
            assert val == pytest.approx(float(O.wavelet_hat(w, k)), rel=1e-9)


def test_zero_mean():
    # a positive peak with a negative ring integrates to zero (admissible wavelet)
    w = 1.3
    f = lambda r: float(O.wavelet(w, r * r)) * 4 * math.pi * r * r
    val, _ = integrate.quad(f, 0.0, 40.0 / w, limit=400, epsabs=0, epsrel=1e-13)
    pos, _ = integrate.quad(f, 0.0, math.sqrt(6) / w, limit=200)
    assert abs(val) < 1e-11 * pos
    assert float(O.wavelet_hat(w, 0.0)) == 0.0


def test_first_w_derivative_of_gaussian():
    # Sec. 2.1: the wavelet derives from the first derivative of a Gaussian with
    # respect to w; in Fourier space Psi_hat ~ w^-1/2 d/dw exp(-k^2/w^2).
    ratios = []
    for w in (0.5, 1.0, 3.0):
        for k in (0.3, 1.0, 2.5):
            h = 1e-5 * w
            d = (math.exp(-k * k / (w + h) ** 2) - math.exp(-k * k / (w - h) ** 2)) / (2 * h)
            ratios.append(float(O.wavelet_hat(w, k)) * math.sqrt(w) / d)
    assert np.allclose(ratios, ratios[0], rtol=1e-7)
    assert ratios[0] == pytest.approx(16 * math.pi ** 1.5, rel=1e-7)


def test_zero_crossing_of_wavelet():
    w = 0.8
    r0 = math.sqrt(6.0) / w
    assert float(O.wavelet(w, (r0 * 0.999) ** 2)) > 0 > float(O.wavelet(w, (r0 * 1.001) ** 2))


def _brute_force_cwt(f, box_len, w, images):
    n = f.shape[0]
    dx = box_len / n
    g = np.arange(n) * dx
    out = np.zeros_like(f)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    for gz in range(n):
        for gy in range(n):
            for gx in range(n):
                if f[gz, gy, gx] == 0.0:
                    continue
                acc = np.zeros_like(f)
                for mz in range(-images, images + 1):
                    for my in range(-images, images + 1):
                        for mx in range(-images, images + 1):
                            r2 = ((X - gx * dx + mx * box_len) ** 2 + (Y - gy * dx + my * box_len) ** 2
                                  + (Z - gz * dx + mz * box_len) ** 2)
                            u = w * w * r2
                            acc += w ** 1.5 * (6.0 - u) * np.exp(-u / 4.0)
                out += f[gz, gy, gx] * acc * dx ** 3
    return out


def test_brute_force_periodic_sum_8cubed():
    rng = np.random.default_rng(3)
    f = rng.random((8, 8, 8))
    f[f < 0.6] = 0.0  # sparse, so the brute force stays cheap
    w = 1.0 / 1.5  # a = 1.5 cells, L = 8
    ref = _brute_force_cwt(f, 8.0, w, images=3)
    got = O.cwt_field(f, 8.0, w, "sampled")
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_single_point_is_the_wavelet():
    n, L = 32, 32.0
    pos = np.array([[10.0, 20.0, 5.0]])
    rho = O.deposit(pos, L, n)
    a = 3.0
    kw = n / (1000 * a)
    w = O.scale_w(kw, L)
    g = np.arange(n)
    d = lambda c0: ((g - c0 + n // 2) % n - n // 2).astype(float)
    expect = np.zeros((n, n, n))
    for m in np.ndindex(5, 5, 5):  # periodic images within two boxes
        mz, my, mx = (np.array(m) - 2) * L
        r2 = ((d(5) + mz)[:, None, None] ** 2 + (d(20) + my)[None, :, None] ** 2
              + (d(10) + mx)[None, None, :] ** 2)
        expect += L ** 3 * w ** 1.5 * (6 - w * w * r2) * np.exp(-w * w * r2 / 4)
    for mode, tol in (("sampled", 1e-12), ("analytic", 1e-10)):
        c = O.cwt(rho, L, kw, mode)
        assert np.max(np.abs(c - expect)) < tol * expect.max(), mode


@pytest.mark.parametrize("a", [2.0, 3.0])
def test_sampled_matches_analytic_when_resolved(a):
    rng = np.random.default_rng(5)
    f = rng.random((24, 24, 24))
    w = 1.0 / a
    s = O.cwt_field(f, 24.0, w, "sampled")
    an = O.cwt_field(f, 24.0, w, "analytic")
    assert np.max(np.abs(s - an)) < 1e-11 * np.max(np.abs(s))


def test_uniform_field_is_flat_zero():
    n, L = 32, 64.0
    g = (np.arange(n) * (L / n))
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    rho = O.deposit(pos, L, n)
    assert np.all(rho == rho.flat[0])
    kw = n / (1000 * 1.0)
    w = O.scale_w(kw, L)
    peak = L ** 3 * 6 * w ** 1.5  # CWT of one particle at its own node
    assert np.max(np.abs(O.cwt(rho, L, kw, "sampled"))) < 1e-10 * peak
    assert np.max(np.abs(O.cwt(rho, L, kw, "analytic"))) < 1e-12 * peak


def _blob(n, s, centre):
    g = np.arange(n)
    d = lambda c0: ((g - c0 + n // 2) % n - n // 2).astype(float)
    r2 = d(centre[0])[:, None, None] ** 2 + d(centre[1])[None, :, None] ** 2 + d(centre[2])[None, None, :] ** 2
    return np.exp(-r2 / (2 * s * s)), r2


def test_gaussian_blob_closed_form():
    # rho = A exp(-r^2/2s^2)  ->  C(r) = A (2 pi s^2)^1.5 w^-3.5 W^5 (6 - W^2 r^2) exp(-W^2 r^2/4),
    # 1/W^2 = 1/w^2 + s^2/2  (Gaussian times the transform of Eq. (4), inverted)
    n, s, a = 64, 2.0, 2.0
    f, r2 = _blob(n, s, (30, 31, 33))
    w = 1.0 / a
    W = (1.0 / w ** 2 + s * s / 2) ** -0.5
    expect = (2 * math.pi * s * s) ** 1.5 * w ** -3.5 * W ** 5 * (6 - W * W * r2) * np.exp(-W * W * r2 / 4)
    for mode in ("sampled", "analytic"):
        c = O.cwt_field(f, float(n), w, mode)
        assert np.max(np.abs(c - expect)) < 1e-9 * expect.max(), mode
    # zero crossing at sqrt(6)/W and the valley (basin edge) at sqrt(10)/W
    r = np.sqrt(r2)
    c = O.cwt_field(f, float(n), w, "sampled")
    assert np.all(c[r < math.sqrt(6) / W - 0.5] > 0) and np.all(c[(r > math.sqrt(6) / W + 0.5) & (r < 20)] < 0)


def test_linearity_and_translation():
    rng = np.random.default_rng(9)
    f, g = rng.random((2, 16, 16, 16))
    w = 0.5
    cf, cg = O.cwt_field(f, 16.0, w), O.cwt_field(g, 16.0, w)
    np.testing.assert_allclose(O.cwt_field(2 * f - 3 * g, 16.0, w), 2 * cf - 3 * cg, atol=1e-12 * np.abs(cf).max())
    shifted = O.cwt_field(np.roll(f, (3, -5, 7), axis=(0, 1, 2)), 16.0, w)
    np.testing.assert_allclose(shifted, np.roll(cf, (3, -5, 7), axis=(0, 1, 2)), atol=1e-12 * np.abs(cf).max())


def test_normalisation_is_resolution_free():
    # f is in mean-density units and the kernel carries dx^3, so refining the grid
    # of a smooth field leaves C at shared nodes unchanged (up to sampling error).
    n1, n2, L, a_phys = 16, 32, 16.0, 3.0
    w = 1.0 / a_phys
    def field(n):
        g = np.arange(n) * (L / n)
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        return 1.0 + 0.5 * np.sin(2 * math.pi * X / L) * np.cos(2 * math.pi * Y / L)
    c1 = O.cwt_field(field(n1), L, w)
    c2 = O.cwt_field(field(n2), L, w)
    np.testing.assert_allclose(c2[::2, ::2, ::2], c1, atol=1e-8 * np.abs(c1).max())
