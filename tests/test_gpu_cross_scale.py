"""GPU parity of the cross-scale maximum check (step 8, each maximum corrected
for the grid as step 4 asks, App. B) and of the group filter that uses it,
against the oracle, through the C ABI.  Both sides decide on the same FP32
fields, which the oracle produces (stage-isolated), so the flags and labels
must agree bit for bit, on one grid and across grids of different size."""
import numpy as np
import pytest
import torch

from gpu_helpers import O, cuda, ensure_built, small_box

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


def hfm():
    import paper_2501_10622_amd as m
    return m


def oracle_fields(n, L, np_, halos, seed, scales):
    pos = small_box(n, L, np_, halos, "f32", seed)
    rho = O.deposit(pos, L, n)
    return pos, [O.cwt(rho, L, n / (1000.0 * a)).astype(np.float32) for a in scales]


@pytest.mark.parametrize("n,L,np_,halos,seed,scales", [
    (32, 40.0, 40000, 60, 61, (1.0, 0.75)),
    (64, 100.0, 64 ** 3, 200, 62, (1.5, 1.0)),
    (96, 96.0, 400000, 300, 63, (1.5, 1.0)),   # radix-3 grid
])
def test_cross_scale_matches_oracle(n, L, np_, halos, seed, scales):
    _, (c1, c2) = oracle_fields(n, L, np_, halos, seed, scales)
    roots = O.maxima(c1)
    print(f"cross scale n={n} roots={len(roots)}", flush=True)
    got = hfm().cross_scale(cuda(c1), cuda(c2), cuda(roots.astype(np.int32)))
    hfm().sync()
    want = O.cross_scale(c1, c2, roots)
    np.testing.assert_array_equal(got.cpu().numpy().astype(bool), want)
    assert want.any() and not want.all()


@pytest.mark.parametrize("n2,n1,L,np_,seed,a2,a1", [
    # scales 2-3% apart in box units, so that some maxima pass and some fail
    (48, 64, 60.0, 200000, 71, 2.0, 2.6),    # finer grid for the smaller scale, ratio 4/3
    (32, 96, 40.0, 100000, 72, 1.5, 4.4),    # three times finer
    (64, 48, 64.0, 300000, 73, 1.5, 1.1),    # coarser (the cube-size term changes sign)
])
def test_cross_scale_across_grids_matches_oracle(n2, n1, L, np_, seed, a2, a1):
    pos = small_box(max(n1, n2), L, np_, 200, "f32", seed)
    c2 = O.cwt(O.deposit(pos, L, n2), L, n2 / (1000.0 * a2)).astype(np.float32)
    c1 = O.cwt(O.deposit(pos, L, n1), L, n1 / (1000.0 * a1)).astype(np.float32)
    roots = O.maxima(c2)
    print(f"cross scale across grids n2={n2} n1={n1} roots={len(roots)}", flush=True)
    got = hfm().cross_scale(cuda(c2), cuda(c1), cuda(roots.astype(np.int32)))
    hfm().sync()
    want = O.cross_scale(c2, c1, roots)
    np.testing.assert_array_equal(got.cpu().numpy().astype(bool), want)
    assert want.any() and not want.all()


@pytest.mark.parametrize("seed", [1, 2])
def test_cross_scale_off_grid_paraboloid(seed):
    # the raw grid value is below the flat smaller-scale field, the corrected top above it
    rng = np.random.default_rng(seed)
    n = 16
    x0 = np.array([6.0, 9.0, 5.0]) + rng.uniform(0.2, 0.45, 3) * rng.choice([-1, 1], 3)
    k = rng.uniform(0.5, 2.0, 3)
    g = np.arange(n, dtype=np.float64)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    c = (40.0 - k[0] * (X - x0[0]) ** 2 - k[1] * (Y - x0[1]) ** 2 - k[2] * (Z - x0[2]) ** 2).astype(np.float32)
    r = np.round(x0).astype(int)
    root = np.array([(r[2] * n + r[1]) * n + r[0]], dtype=np.int32)
    B = float(c.ravel()[root[0]])
    for level, expect in ((0.5 * (B + 40.0), 1), (40.0 + 0.01, 0)):
        flat = np.full((n, n, n), level, np.float32)
        assert O.cross_scale(c, flat, root).tolist() == [bool(expect)]
        got = hfm().cross_scale(cuda(c), cuda(flat), cuda(root))
        hfm().sync()
        assert got.cpu().tolist() == [expect]


def test_cross_scale_blob():
    n, s, centre = 64, 2.0, (30, 31, 33)
    g = np.arange(n)
    d = lambda c0: ((g - c0 + n // 2) % n - n // 2).astype(float)
    r2 = d(centre[0])[:, None, None] ** 2 + d(centre[1])[None, :, None] ** 2 + d(centre[2])[None, None, :] ** 2
    f = np.exp(-r2 / (2 * s * s))
    root = np.array([(centre[0] * n + centre[1]) * n + centre[2]], dtype=np.int32)
    for a1, a2, expect in ((4.0, 3.0, 0), (1.5, 1.0, 1)):
        c1 = O.cwt_field(f, float(n), 1 / a1).astype(np.float32)
        c2 = O.cwt_field(f, float(n), 1 / a2).astype(np.float32)
        got = hfm().cross_scale(cuda(c1), cuda(c2), cuda(root))
        hfm().sync()
        assert got.cpu().tolist() == [expect]


def test_cross_scale_nan_reported():
    from paper_2501_10622_amd import HFError, hf
    c = np.zeros((8, 8, 8), np.float32)
    c[0, 0, 0] = 1.0
    c2 = c.copy()
    c2[0, 0, 1] = np.nan
    hfm().cross_scale(cuda(c), cuda(c2), cuda(np.array([0], np.int32)))
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == hf.HF_ERR_INPUT


def test_groups_with_cross_scale_filter():
    # steps 5-8 at one scale against the next smaller one, all on the oracle's fields
    n, L, np_, halos, seed = 64, 100.0, 64 ** 3, 200, 64
    pos, (c1, c2) = oracle_fields(n, L, np_, halos, seed, (0.8, 0.6))
    roots = O.maxima(c1)
    cell = O.segment(c1)
    plab = O.label(pos, L, n, cell)
    ok = O.cross_scale(c1, c2, roots)
    want = O.group_stats(cell, plab, roots, n, np_, 1.0, 15, root_ok=ok)
    flags = hfm().cross_scale(cuda(c1), cuda(c2), cuda(roots.astype(np.int32)))
    got = hfm().groups(cuda(cell.astype(np.int32)), cuda(plab.astype(np.int32)), cuda(roots.astype(np.int32)), np_,
                       1.0, 15, root_ok=flags)
    hfm().sync()
    np.testing.assert_array_equal(got["keep"].cpu().numpy().astype(bool), want["keep"])
    np.testing.assert_array_equal(got["particle_label"].cpu().numpy(), want["particle_label"])
    np.testing.assert_array_equal(got["cell_label"].cpu().numpy(), want["cell_label"])
    base = O.group_stats(cell, plab, roots, n, np_, 1.0, 15)
    assert 0 < want["keep"].sum() < base["keep"].sum()  # the cross-scale test disposes of some groups
