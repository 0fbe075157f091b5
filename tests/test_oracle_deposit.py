"""Pins for the oracle's CIC deposit (Eq. (1), Sec. 2.1).

Each check is fixed by the definition of cloud-in-cell assignment, not by the
oracle's own code: mass conservation, the two textbook special cases (particle
on a node, particle at a cube centre), periodic wrap, order independence, the
exact overflow boundary, and a brute-force tent-function sum over every node.
"""
import numpy as np
import pytest

from oracle import cwthf as O
from synth import make_box

B = 15
ONE = 1 << B


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_mass_conservation(dtype):
    pos = make_box(40.0, 5000, 10, "f64", seed=11).numpy().astype(dtype)
    rho = O.deposit(pos, 40.0, 16, B)
    assert rho.dtype == np.int64 and rho.shape == (16, 16, 16)
    assert int(rho.sum()) == 5000 * ONE ** 3
    assert rho.min() >= 0


def test_particle_on_node_goes_to_one_cell():
    n = 8
    pos = np.array([[3.0, 5.0, 6.0]])  # L = n, so node g sits at x = g
    rho = O.deposit(pos, float(n), n, B)
    assert rho[6, 5, 3] == ONE ** 3
    assert np.count_nonzero(rho) == 1


def test_particle_at_cube_centre_splits_evenly():
    n = 8
    pos = np.array([[2.5, 4.5, 7.5]])
    rho = O.deposit(pos, float(n), n, B)
    nz = np.argwhere(rho)
    assert len(nz) == 8
    assert np.all(rho[rho != 0] == ONE ** 3 // 8)
    zs, ys, xs = set(nz[:, 0]), set(nz[:, 1]), set(nz[:, 2])
    assert xs == {2, 3} and ys == {4, 5} and zs == {7, 0}  # z wraps periodically


def test_top_edge_wraps_to_node_zero():
    n = 8
    eps_pos = np.nextafter(np.float64(n), 0.0)
    pos = np.array([[eps_pos, 0.0, 0.0]])
    rho = O.deposit(pos, float(n), n, B)
    # q = n 2^B - 1: lower node 7 keeps weight 1, the upper node (0, wrapped) the rest
    assert rho[0, 0, 7] == 1 * ONE * ONE
    assert rho[0, 0, 0] == (ONE - 1) * ONE * ONE


def test_periodic_images_deposit_identically():
    pos = make_box(32.0, 3000, 5, "f64", seed=12).numpy()
    a = O.deposit(pos, 32.0, 16, B)
    b = O.deposit(pos + 32.0, 32.0, 16, B)
    c = O.deposit(pos - 64.0, 32.0, 16, B)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)


def test_order_independent():
    pos = make_box(32.0, 4000, 8, "f32", seed=13).numpy()
    perm = np.random.default_rng(0).permutation(len(pos))
    np.testing.assert_array_equal(O.deposit(pos, 32.0, 16, B), O.deposit(pos[perm], 32.0, 16, B))


def _tent_brute_force(pos, box_len, n, bits):
    """Every node g gets prod_axes max(0, 2^B - periodic |q - g 2^B|), in Python ints."""
    one = 1 << bits
    m = n << bits
    scale = pos.dtype.type(n * one / box_len)
    rho = [[[0] * n for _ in range(n)] for _ in range(n)]
    for p in pos:
        q = [int(np.floor(p[a] * scale)) % m for a in range(3)]
        for gz in range(n):
            for gy in range(n):
                for gx in range(n):
                    w = 1
                    for a, g in zip(range(3), (gx, gy, gz)):
                        d = (q[a] - g * one) % m
                        d = min(d, m - d)
                        w *= max(0, one - d)
                    rho[gz][gy][gx] += w
    return np.array(rho, dtype=object)


@pytest.mark.parametrize("dtype,bits", [(np.float64, 15), (np.float32, 15), (np.float64, 9)])
def test_brute_force_tent_sum(dtype, bits):
    rng = np.random.default_rng(7)
    pos = (rng.random((40, 3)) * 13.0 - 2.0).astype(dtype)  # includes positions outside [0, L)
    got = O.deposit(pos, 9.0, 6, bits)
    ref = _tent_brute_force(pos, 9.0, 6, bits)
    assert np.array_equal(got.astype(object), ref)


def test_overflow_boundary_exact():
    bits = 20  # one full particle is 2^60; eight of them reach 2^63
    pos7 = np.zeros((7, 3))
    rho = O.deposit(pos7, 8.0, 8, bits)
    assert rho[0, 0, 0] == 7 * (1 << 60)
    with pytest.raises(O.DepositOverflow):
        O.deposit(np.zeros((8, 3)), 8.0, 8, bits)


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        O.deposit(np.array([[np.nan, 0.0, 0.0]]), 8.0, 8, B)
    with pytest.raises(ValueError):
        O.deposit(np.zeros((1, 3)), 8.0, 8, 7)


def test_mean_mass_exact_above_int64():
    # total mass beyond 2^63 must still be summed exactly
    rho = np.full((8, 8, 8), (1 << 62) + 3, dtype=np.int64)
    assert O.total_mass(rho) == 512 * ((1 << 62) + 3)
