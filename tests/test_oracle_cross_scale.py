"""Pins for the oracle's cross-scale maximum check (step 8, with step 4's
correction of each maximum for the grid, App. B).

- A field that is a paraboloid around a point off the grid has its top value
  and position recovered exactly by the per-axis quadratic fits (pinned in
  test_oracle_peaks.py).  Against a flat smaller-scale field placed between the
  raw grid maximum and the true top, the check must pass; placed just above the
  true top, it must fail.  The raw-value reading decides both the other way.
- For a paraboloid V - sum_d k_d (x_d - x0_d)^2 sampled on a grid of spacing
  dx2, every axis has 2 l2 - l1 = 2 k_d dx2^2 whatever the offset, so App. B's
  cube-size term (3/5 removed) is (5/8) mean(k) (dx2^2 - dx1^2) in closed form.
  A flat finer-grid field between the corrected value with and without that
  term flips the decision.
- Across grids, "near" is found at the corrected position: a spike on the
  finer grid two of its cells from the raw node's image but next to the
  corrected position fails the maximum, and one on the other side does not.
- Brute force walks the 27 periodic neighbours with explicit wrap, taking the
  corrected value and position from ``peaks``.
- The Gaussian blob centred on a node (symmetric neighbours: no correction)
  fixes the outcome from its closed-form CWT: at the centre C(w) is
  proportional to w^1.5 (1 + w^2 s^2 / 2)^(-5/2), which rises with w up to
  w* = sqrt(6/7)/s and falls beyond.
"""
import math

import numpy as np
import pytest

from oracle import cwthf as O


def _paraboloid(n, x0, k, V, dxc=1.0):
    """V - sum k_d (g_d - x0_d)^2 dxc^2 on an n^3 grid ([z][y][x]); x0 in cells (x, y, z)."""
    g = np.arange(n, dtype=np.float64)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    return V - (k[0] * (X - x0[0]) ** 2 + k[1] * (Y - x0[1]) ** 2 + k[2] * (Z - x0[2]) ** 2) * dxc * dxc


def _root_of(n, x0):
    r = np.round(np.asarray(x0)).astype(int)
    return int((r[2] * n + r[1]) * n + r[0])


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_off_grid_peak_decision_flips_with_the_correction(seed):
    rng = np.random.default_rng(seed)
    n = 16
    x0 = np.array([6.0, 9.0, 5.0]) + rng.uniform(0.15, 0.45, 3) * rng.choice([-1, 1], 3)
    k = rng.uniform(0.5, 2.0, 3)
    V = 40.0
    c = _paraboloid(n, x0, k, V)
    root = _root_of(n, x0)
    assert root in set(O.maxima(c).tolist())
    B = c.ravel()[root]
    assert B < V - 0.05  # the grid misses the top by a visible margin
    between = np.full_like(c, 0.5 * (B + V))  # above the raw value, below the true top
    above = np.full_like(c, V + 1e-9)
    assert O.cross_scale(c, between, [root]).tolist() == [True]
    assert O.cross_scale(c, above, [root]).tolist() == [False]
    # the raw grid value alone would reject the first case
    assert not B > between.max()


@pytest.mark.parametrize("n2,n1,seed", [(12, 24, 5), (16, 20, 6), (10, 30, 7)])
def test_cube_size_term_closed_form(n2, n1, seed):
    rng = np.random.default_rng(seed)
    x0 = np.array([4.0, 5.0, 3.0]) + rng.uniform(-0.4, 0.4, 3)
    k = rng.uniform(0.5, 2.0, 3)
    V, L = 30.0, float(n2)  # one cell of the coarse grid is one box unit
    c = _paraboloid(n2, x0, k, V)
    root = _root_of(n2, x0)
    shift, value, l1bar, l2bar = O._peak_fits(c, [root])
    dx2, dx1 = L / n2, L / n1
    expect = 0.625 * k.mean() * (dx2 ** 2 - dx1 ** 2)
    got = float(O.cube_size_term(l1bar, l2bar, n2, n1)[0])
    assert got == pytest.approx(expect, rel=1e-12)
    assert float(O.cube_size_term(l1bar, l2bar, n2, n2)[0]) == 0.0
    np.testing.assert_allclose(value[0], V, rtol=1e-13)
    # a flat finer field between V and V + term: passes only with the term
    fine = np.full((n1, n1, n1), V + 0.5 * expect)
    assert O.cross_scale(c, fine, [root]).tolist() == [True]
    fine_hi = np.full((n1, n1, n1), V + 1.5 * expect)
    assert O.cross_scale(c, fine_hi, [root]).tolist() == [False]


def test_near_points_follow_the_corrected_position_across_grids():
    n2, n1 = 16, 32  # the smaller scale's grid is twice as fine
    x0 = np.array([7.0 + 0.4, 8.0, 6.0])  # true top 0.4 coarse cells (0.8 fine) up x
    k = np.array([1.0, 1.0, 1.0])
    c = _paraboloid(n2, x0, k, 20.0)
    root = _root_of(n2, x0)  # coarse node (7, 8, 6)
    shift, _, _, _ = O._peak_fits(c, [root])
    assert shift[0][0] == pytest.approx(0.4, abs=1e-12)
    # corrected position on the fine grid: x = 2 * 7.4 = 14.8 -> node 15; raw node image 14
    low = np.zeros((n1, n1, n1))
    spike_far = low.copy()
    spike_far[12, 16, 16] = 100.0  # x = 16: next to node 15, two fine cells from 14
    assert O.cross_scale(c, spike_far, [root]).tolist() == [False]
    spike_behind = low.copy()
    spike_behind[12, 16, 13] = 100.0  # x = 13: next to 14 only
    assert O.cross_scale(c, spike_behind, [root]).tolist() == [True]


def _brute(cs, cm, roots):
    n2, n1 = cs.shape[0], cm.shape[0]
    pos, val = O.peaks(cs, roots, float(n2))  # box of n2 units: positions in coarse cells
    _, _, l1b, l2b = O._peak_fits(cs, roots)
    out = []
    for i, r in enumerate(roots):
        v = val[i] + float(O.cube_size_term(l1b[i:i + 1], l2b[i:i + 1], n2, n1)[0])
        node = [int(math.floor(pos[i][a] * n1 / n2 + 0.5)) % n1 for a in range(3)]  # x, y, z
        best = max(cm[(node[2] + dz) % n1, (node[1] + dy) % n1, (node[0] + dx) % n1]
                   for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
        out.append(bool(v > best))
    return out


@pytest.mark.parametrize("seed,n2,n1", [(1, 8, 8), (2, 9, 9), (3, 12, 12), (4, 8, 12), (5, 10, 16)])
def test_matches_brute_force(seed, n2, n1):
    rng = np.random.default_rng(seed)
    cs = rng.normal(size=(n2, n2, n2))
    g = np.linspace(0, n2, n1, endpoint=False)
    cm = rng.normal(scale=0.7, size=(n1, n1, n1)) + 0.6 * cs[np.ix_(g.astype(int), g.astype(int), g.astype(int))]
    roots = O.maxima(cs, -np.inf)
    got = O.cross_scale(cs, cm, roots)
    assert got.tolist() == _brute(cs, cm, roots)
    assert got.any() and not got.all()


def test_symmetric_maximum_never_beats_its_own_field():
    n = 8
    c = np.zeros((n, n, n))
    c[3, 4, 5] = 2.0  # symmetric on every axis: no correction, V = B
    assert O.cross_scale(c, c, [(3 * n + 4) * n + 5]).tolist() == [False]
    assert O.cross_scale(c + 1e-9, c, [(3 * n + 4) * n + 5]).tolist() == [True]


def test_against_the_zero_grid():
    rng = np.random.default_rng(9)
    c = rng.normal(size=(8, 8, 8))
    roots = O.maxima(c, -np.inf)
    got = O.cross_scale(c, np.zeros_like(c), roots)
    _, val = O.peaks(c, roots, 8.0)
    assert got.tolist() == (val > 0).tolist()


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
    _, val = O.peaks(c1, [root], float(n))
    assert abs(val[0] - c1.ravel()[root]) < 1e-12 * abs(val[0])  # centred: no correction
    assert O.cross_scale(c1, c2, [root]).tolist() == [expect]
