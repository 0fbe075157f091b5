"""GPU parity of step 4's peak correction (App. B) against the oracle on the
same FP32 fields: both compute in FP64 with every operation rounded as written,
so positions and values must agree bit for bit."""
import numpy as np
import pytest

from gpu_helpers import O, cuda, ensure_built, small_box

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


def hfm():
    import paper_2501_10622_amd as m
    return m


@pytest.mark.parametrize("n,L,np_,halos,a,seed", [
    (32, 40.0, 40000, 60, 1.5, 71),
    (64, 100.0, 64 ** 3, 200, 2.0, 72),
    (96, 96.0, 400000, 300, 1.0, 73),
])
def test_peaks_match_oracle(n, L, np_, halos, a, seed):
    pos = small_box(n, L, np_, halos, "f32", seed)
    c = O.cwt(O.deposit(pos, L, n), L, n / (1000.0 * a)).astype(np.float32)
    roots = O.maxima(c)
    print(f"peaks n={n} roots={len(roots)}", flush=True)
    gp, gv = hfm().peaks(cuda(c), cuda(roots.astype(np.int32)), L)
    hfm().sync()
    wp, wv = O.peaks(c, roots, L)
    np.testing.assert_array_equal(gp.cpu().numpy(), wp)
    np.testing.assert_array_equal(gv.cpu().numpy(), wv)
    # the corrected peak is never below the grid maximum and within half a cell of it
    cells = np.stack([roots % n, (roots // n) % n, roots // (n * n)], axis=1) * (L / n)
    d = (wp - cells + L / 2) % L - L / 2
    assert np.all(np.abs(d) <= 0.5 * L / n + 1e-12)
    assert np.all(wv >= c.ravel()[roots])


def test_peaks_quadratic_and_wrap():
    n, L = 16, 32.0
    x0 = np.array([7.3, 8.8, 0.2])  # near the z = 0 face: the fit reaches across the boundary
    g = np.arange(n, dtype=np.float64)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    dz = (Z - x0[2] + n / 2) % n - n / 2
    c = (50.0 - 1.5 * (X - x0[0]) ** 2 - 0.7 * (Y - x0[1]) ** 2 - 1.1 * dz ** 2).astype(np.float32)
    roots = O.maxima(c)
    gp, gv = hfm().peaks(cuda(c), cuda(roots.astype(np.int32)), L)
    hfm().sync()
    wp, wv = O.peaks(c, roots, L)
    np.testing.assert_array_equal(gp.cpu().numpy(), wp)
    np.testing.assert_array_equal(gv.cpu().numpy(), wv)
    np.testing.assert_allclose(wp[0], x0 * (L / n), atol=2e-4 * L / n)  # FP32 field: close, not exact


def test_peaks_arguments_and_nan():
    from paper_2501_10622_amd import HFError, hf
    c = np.zeros((8, 8, 8), np.float32)
    c[0, 0, 1] = np.nan  # the +x neighbour of cell 0, which the fit reads
    hfm().peaks(cuda(c), cuda(np.array([0], np.int32)), 8.0)
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == hf.HF_ERR_INPUT
    p, v = hfm().peaks(cuda(np.zeros((8, 8, 8), np.float32)), cuda(np.zeros(0, np.int32)), 8.0)
    hfm().sync()
    assert p.shape == (0, 3) and v.shape == (0,)
