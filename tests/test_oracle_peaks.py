"""Pins for the oracle's peak correction (step 4, App. B).

A field that is a sum of per-axis parabolas around a point off the grid has
its top recovered exactly by the per-axis quadratic fits: the vertex of each
axis's parabola is the point's coordinate, and the corrections add the
missing k_d delta_d^2 to the grid value.  Symmetric neighbours leave the
maximum where it is.
"""
import numpy as np
import pytest

from oracle import cwthf as O


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_quadratic_peak_recovered_exactly(seed):
    rng = np.random.default_rng(seed)
    n, L = 16, 32.0
    x0 = np.array([7.0, 9.0, 4.0]) + rng.uniform(-0.49, 0.49, 3)  # (x, y, z) in cells
    k = rng.uniform(0.5, 2.0, 3)
    V = 50.0
    g = np.arange(n, dtype=np.float64)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    c = V - k[0] * (X - x0[0]) ** 2 - k[1] * (Y - x0[1]) ** 2 - k[2] * (Z - x0[2]) ** 2
    root = int((np.round(x0[2]) * n + np.round(x0[1])) * n + np.round(x0[0]))
    assert root in set(O.maxima(c).tolist())
    pos, val = O.peaks(c, [root], L)
    np.testing.assert_allclose(pos[0], x0 * (L / n), rtol=0, atol=1e-12)
    np.testing.assert_allclose(val[0], V, rtol=1e-14)


def test_symmetric_and_flat_neighbours():
    n, L = 8, 8.0
    c = np.zeros((n, n, n))
    c[3, 4, 5] = 2.0  # symmetric neighbours on every axis
    pos, val = O.peaks(c, [(3 * n + 4) * n + 5], L)
    assert pos[0].tolist() == [5.0, 4.0, 3.0] and val[0] == 2.0
    flat = np.ones((n, n, n))
    pos, val = O.peaks(flat, [0], L)
    assert pos[0].tolist() == [0.0, 0.0, 0.0] and val[0] == 1.0


def test_tie_with_a_neighbour_puts_the_peak_half_way():
    n, L = 8, 8.0
    c = np.zeros((n, n, n))
    c[2, 2, 2] = c[2, 2, 3] = 1.0  # equal neighbour along +x
    pos, val = O.peaks(c, [(2 * n + 2) * n + 2], L)
    assert pos[0].tolist() == [2.5, 2.0, 2.0]
    assert val[0] == 1.0 + 1.0 / 8.0  # l1 = l2 = 1: l1^2 / (16 l2 - 8 l1)


def test_periodic_wrap():
    n, L = 8, 8.0
    c = np.zeros((n, n, n))
    c[0, 0, 0], c[0, 0, n - 1] = 3.0, 1.0  # larger neighbour across the x boundary
    pos, _ = O.peaks(c, [0], L)
    assert 7.5 < pos[0][0] < 8.0 and pos[0][1] == 0.0
