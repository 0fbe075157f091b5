"""Pins for the oracle's maxima (step 4), segmentation (step 5, Sec. 2.3) and
particle labels (step 6).

Brute-force references are literal pure-Python loops over the definitions
(tuple comparison for the (value, index) order, sequential path following), so
they share no vectorised machinery with the oracle.  The Gaussian blob ties the
segmentation to the closed-form valley radius of its CWT.
"""
import math

import numpy as np
import pytest

from oracle import cwthf as O

OFFS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _key(c, n, z, y, x):
    v = float(c[z % n, y % n, x % n])
    return (v + 0.0, ((z % n) * n + (y % n)) * n + (x % n))  # -0.0 + 0.0 == +0.0


def _brute_parent(c):
    n = c.shape[0]
    par = {}
    for z in range(n):
        for y in range(n):
            for x in range(n):
                best = max(_key(c, n, z + dz, y + dy, x + dx) for dz, dy, dx in OFFS)
                par[(z * n + y) * n + x] = best[1]
    return par


def _brute_maxima(c, tau):
    n = c.shape[0]
    out = []
    for z in range(n):
        for y in range(n):
            for x in range(n):
                me = _key(c, n, z, y, x)
                if me[0] > tau and all(me > _key(c, n, z + dz, y + dy, x + dx)
                                       for dz, dy, dx in OFFS if (dz, dy, dx) != (0, 0, 0)):
                    out.append(me[1])
    return out


def _brute_segment(c, tau):
    par = _brute_parent(c)
    flat = c.ravel()
    lab = []
    for j in range(c.size):
        r = j
        while par[r] != r:
            r = par[r]
        lab.append(r if flat[r] > tau else -1)
    return np.array(lab).reshape(c.shape)


def _smooth_field(n, seed, sigma=1.2):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n))
    k = np.fft.fftfreq(n)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    return np.fft.ifftn(np.fft.fftn(f) * np.exp(-2 * (math.pi * sigma) ** 2 * k2)).real


@pytest.mark.parametrize("n,seed,dtype", [(8, 1, np.float64), (8, 2, np.float32), (16, 3, np.float32)])
def test_maxima_and_segment_brute_force(n, seed, dtype):
    c = _smooth_field(n, seed).astype(dtype)
    tau = 0.0
    np.testing.assert_array_equal(O.maxima(c, tau), _brute_maxima(c, tau))
    np.testing.assert_array_equal(O.segment(c, tau), _brute_segment(c, tau))
    par = O.parents(c)
    bp = _brute_parent(c)
    assert all(par[j] == bp[j] for j in range(c.size))


def test_ties_break_on_index():
    rng = np.random.default_rng(4)
    c = rng.integers(0, 3, (8, 8, 8)).astype(np.float32)  # three levels: many ties
    c[rng.random(c.shape) < 0.3] *= -1.0  # includes -0.0 cells
    for tau in (-1.0, 0.0, 1.0):
        np.testing.assert_array_equal(O.maxima(c, tau), _brute_maxima(c, tau))
        np.testing.assert_array_equal(O.segment(c, tau), _brute_segment(c, tau))


def test_signed_zeros_compare_equal():
    rng = np.random.default_rng(6)
    c = np.where(rng.random((8, 8, 8)) < 0.5, -0.0, 0.0).astype(np.float32)
    # every value equal: only the largest index beats all its neighbours
    np.testing.assert_array_equal(O.maxima(c, -1.0), [8 ** 3 - 1])
    assert np.all(O.segment(c, -1.0) == 8 ** 3 - 1)


def test_nan_rejected():
    c = np.zeros((8, 8, 8))
    c[1, 2, 3] = np.nan
    with pytest.raises(ValueError):
        O.maxima(c)
    with pytest.raises(ValueError):
        O.segment(c)


def test_invariants_on_random_field():
    c = _smooth_field(24, 8).astype(np.float32)
    lab = O.segment(c, 0.0).ravel()
    mx = O.maxima(c, 0.0)
    par = O.parents(c)
    flat = c.ravel()
    assert set(np.unique(lab[lab >= 0])) <= set(mx.tolist())
    assert np.all(lab[mx] == mx)
    idx = np.arange(c.size)
    assert np.all((flat[par] > flat[idx]) | ((flat[par] == flat[idx]) & (par >= idx)))
    # each basin is 26-connected: flood from its root inside the basin reaches all of it
    n = c.shape[0]
    lab3 = lab.reshape(c.shape)
    for root in mx[:10]:
        seen = {int(root)}
        todo = [int(root)]
        while todo:
            j = todo.pop()
            z, y, x = j // (n * n), (j // n) % n, j % n
            for dz, dy, dx in OFFS:
                k = (((z + dz) % n) * n + (y + dy) % n) * n + (x + dx) % n
                if k not in seen and lab3.flat[k] == root:
                    seen.add(k)
                    todo.append(k)
        assert len(seen) == int(np.sum(lab == root))


def test_blob_single_maximum_and_valley_basin():
    # box small enough that the blob's negative tail stays far above FP64 rounding
    # everywhere, so no rounding-noise maxima appear
    n, s, a = 32, 2.0, 2.0
    g = np.arange(n)
    d = lambda c0: ((g - c0 + n // 2) % n - n // 2).astype(float)
    cz, cy, cx = 12, 17, 15
    r2 = d(cz)[:, None, None] ** 2 + d(cy)[None, :, None] ** 2 + d(cx)[None, None, :] ** 2
    f = 50.0 * np.exp(-r2 / (2 * s * s))
    c = O.cwt_field(f, float(n), 1.0 / a)
    centre = (cz * n + cy) * n + cx
    np.testing.assert_array_equal(O.maxima(c, 0.0), [centre])
    W = (a * a + s * s / 2) ** -0.5
    r_valley = math.sqrt(10.0) / W  # where the basin of the blob ends (closed form)
    lab = O.segment(c, 0.0)
    r = np.sqrt(r2)
    assert np.all(lab[r < r_valley - math.sqrt(3)] == centre)
    assert np.all(lab[r > r_valley + math.sqrt(3)] != centre)


def test_two_blobs_split_at_the_valley():
    n, s = 48, 1.5
    g = np.arange(n)
    d = lambda c0: ((g - c0 + n // 2) % n - n // 2).astype(float)
    def r2(c):
        return d(c[0])[:, None, None] ** 2 + d(c[1])[None, :, None] ** 2 + d(c[2])[None, None, :] ** 2
    c1, c2 = (24, 24, 18), (24, 24, 29)
    f = 1.0 + 40.0 * np.exp(-r2(c1) / (2 * s * s)) + 20.0 * np.exp(-r2(c2) / (2 * s * s))
    c = O.cwt_field(f, float(n), 1.0 / 2.0)
    m1, m2 = (c1[0] * n + c1[1]) * n + c1[2], (c2[0] * n + c2[1]) * n + c2[2]
    mx = set(O.maxima(c, 0.0).tolist())
    assert {m1, m2} <= mx
    lab = O.segment(c, 0.0)
    row = lab[24, 24, :]
    assert row[18] == m1 and row[29] == m2
    # along the line joining them the labels switch once, at the CWT minimum between the peaks
    seg = row[18:30]
    switch = int(np.argmax(seg == m2))
    assert np.all(seg[:switch] == m1) and np.all(seg[switch:] == m2)
    valley = 18 + int(np.argmin(c[24, 24, 18:30]))
    assert abs((18 + switch) - valley) <= 1


def test_label_brute_force_and_nodes():
    rng = np.random.default_rng(10)
    n, L, bits = 8, 8.0, 15
    cell = rng.integers(-1, 500, (n, n, n))
    pos = rng.random((300, 3)) * 10.0 - 1.0
    got = O.label(pos, L, n, cell, bits)
    scale = n * (1 << bits) / L
    for p, lab in zip(pos, got):
        node = []
        for a in range(3):
            q = int(np.floor(p[a] * scale)) % (n << bits)
            u, frac = divmod(q, 1 << bits)
            node.append((u + (1 if 2 * frac >= (1 << bits) else 0)) % n)
        assert lab == cell[node[2], node[1], node[0]]
    on_nodes = rng.integers(0, n, (50, 3)).astype(float)
    np.testing.assert_array_equal(O.label(on_nodes, L, n, cell, bits),
                                  cell[on_nodes[:, 2].astype(int), on_nodes[:, 1].astype(int),
                                       on_nodes[:, 0].astype(int)])
