"""Pins for the oracle's group statistics and filters (steps 5 and 7, Table 1's
dens_th and particle_th).

The brute-force reference walks the labels with dictionaries and decides the
density test in exact integer arithmetic (N_g n^3 >= dens_th V_g N_p with an
integer dens_th), so it shares neither numpy's counting nor the FP64 decision
with the oracle.  A hand-worked example fixes the expected numbers, and a box
that is one group reduces the density ratio to exactly one.
"""
import numpy as np
import pytest

from oracle import cwthf as O


def _brute(cell_label, particle_label, roots, n, np_total, dens_th, particle_th):
    cells, parts = {}, {}
    for v in np.asarray(cell_label).ravel().tolist():
        if v >= 0:
            cells[v] = cells.get(v, 0) + 1
    for v in np.asarray(particle_label).ravel().tolist():
        if v >= 0:
            parts[v] = parts.get(v, 0) + 1
    out_p, out_c, keep = [], [], []
    for r in np.asarray(roots).tolist():
        p, c = parts.get(r, 0), cells.get(r, 0)
        out_p.append(p)
        out_c.append(c)
        keep.append(p * n ** 3 >= dens_th * c * np_total and p >= particle_th)
    kept = {r for r, k in zip(np.asarray(roots).tolist(), keep) if k}
    new_pl = [v if v in kept else -1 for v in np.asarray(particle_label).ravel().tolist()]
    new_cl = [v if v in kept else -1 for v in np.asarray(cell_label).ravel().tolist()]
    return out_p, out_c, keep, new_pl, new_cl


def test_hand_worked_example():
    # n = 4: 64 cells.  Group 5 owns 4 cells and 10 particles, group 40 owns
    # 20 cells and 6 particles; 40 particles in the box, so the mean is 0.625
    # particles per cell.  Group 5: 2.5 per cell = 4.0 x mean (kept at
    # dens_th = 4, the equality case); group 40: 0.3 per cell = 0.48 x mean.
    n = 4
    cl = np.full(64, -1, dtype=np.int32)
    cl[[5, 6, 9, 10]] = 5
    cl[40:60] = 40
    pl = np.array([5] * 10 + [40] * 6 + [-1] * 24, dtype=np.int32)
    r = O.group_stats(cl.reshape(4, 4, 4), pl, [5, 40], n, 40, dens_th=4.0, particle_th=1)
    assert r["particles"].tolist() == [10, 6]
    assert r["cells"].tolist() == [4, 20]
    assert r["keep"].tolist() == [True, False]
    assert (r["particle_label"] == np.array([5] * 10 + [-1] * 30)).all()
    assert set(r["cell_label"].ravel().tolist()) == {-1, 5}
    assert (r["cell_label"].ravel() == 5).sum() == 4
    # Table 1's particle_th = 15 disposes of group 5 (10 particles) as well
    r15 = O.group_stats(cl.reshape(4, 4, 4), pl, [5, 40], n, 40, dens_th=4.0, particle_th=15)
    assert r15["keep"].tolist() == [False, False]
    assert (r15["particle_label"] == -1).all() and (r15["cell_label"] == -1).all()
    # just below the equality: one particle fewer in the box raises the mean
    r_hi = O.group_stats(cl.reshape(4, 4, 4), pl, [5, 40], n, 41, dens_th=4.0, particle_th=1)
    assert r_hi["keep"].tolist() == [False, False]


@pytest.mark.parametrize("dens_th,keep", [(1.0, True), (0.5, True), (1.0000001, False), (4.0, False)])
def test_single_group_box_has_mean_density(dens_th, keep):
    # every cell and particle in one group: its density is the mean, ratio 1
    n, np_ = 8, 1000
    cl = np.full((n, n, n), 17, dtype=np.int32)
    pl = np.full(np_, 17, dtype=np.int32)
    r = O.group_stats(cl, pl, [17], n, np_, dens_th=dens_th, particle_th=15)
    assert r["cells"].tolist() == [n ** 3] and r["particles"].tolist() == [np_]
    assert r["keep"].tolist() == [keep]


@pytest.mark.parametrize("seed,n,ngroups,np_,dens_th,pth", [
    (1, 6, 5, 300, 4, 15), (2, 8, 12, 2000, 4, 15), (3, 8, 3, 50, 1, 0), (4, 10, 40, 5000, 7, 20),
    (5, 4, 1, 0, 4, 15),
])
def test_matches_brute_force(seed, n, ngroups, np_, dens_th, pth):
    rng = np.random.default_rng(seed)
    roots = np.sort(rng.choice(n ** 3, size=ngroups, replace=False))
    # clustered labels: each group gets a random share; some cells and particles unlabelled
    cl = np.where(rng.random(n ** 3) < 0.8, rng.choice(roots, size=n ** 3, p=rng.dirichlet(np.ones(ngroups))), -1)
    cl[roots] = roots  # a root carries its own label
    pl = np.where(rng.random(np_) < 0.9, cl[rng.integers(0, n ** 3, size=np_)], -1) if np_ else np.zeros(0, np.int64)
    r = O.group_stats(cl.reshape(n, n, n).astype(np.int32), pl.astype(np.int32), roots, n, np_, float(dens_th), pth)
    bp, bc, bk, bpl, bcl = _brute(cl, pl, roots, n, np_, dens_th, pth)
    assert r["particles"].tolist() == bp
    assert r["cells"].tolist() == bc
    assert r["keep"].tolist() == bk
    assert r["particle_label"].tolist() == bpl
    assert r["cell_label"].ravel().tolist() == bcl


def test_invariants_and_idempotence_on_a_segmented_box():
    # a real single-scale result: groups partition the labelled cells and particles
    rng = np.random.default_rng(7)
    n, L = 16, 20.0
    pos = np.concatenate([rng.normal(loc=c, scale=0.6, size=(300, 3)) for c in rng.random((6, 3)) * L]
                         + [rng.random((1500, 3)) * L]) % L
    res = O.find_halos(pos, L, n, n / (1000.0 * 2.0))  # a scale of 2 cells
    cl, pl, roots = res["cell_label"], res["particle_label"], res["maxima"]
    # at this scale the box splits into a few broad groups near the mean density
    # (ratios 0.8-1.2), so dens_th = 1 keeps some and disposes of others
    r = O.group_stats(cl, pl, roots, n, len(pos), 1.0, 15)
    assert r["cells"].sum() == (cl >= 0).sum()
    assert r["particles"].sum() == (pl >= 0).sum()
    assert (r["cells"] >= 1).all()  # a root labels its own cell
    kept = set(np.asarray(roots)[r["keep"]].tolist())
    assert set(r["particle_label"][r["particle_label"] >= 0].tolist()) <= kept
    assert r["keep"].any() and not r["keep"].all()
    # filtering again changes nothing: kept groups keep their numbers
    r2 = O.group_stats(r["cell_label"], r["particle_label"], roots, n, len(pos), 1.0, 15)
    assert (r2["keep"] == r["keep"]).all()
    assert (r2["particle_label"] == r["particle_label"]).all()
    assert (r2["cell_label"] == r["cell_label"]).all()


def test_root_mask_disposes_of_groups():
    # step 8: a group whose maximum failed the cross-scale check goes, whatever its density
    n = 4
    cl = np.full(64, -1, dtype=np.int32)
    cl[[5, 6, 9, 10]] = 5
    cl[40:44] = 40
    pl = np.array([5] * 10 + [40] * 10 + [-1] * 20, dtype=np.int32)
    both = O.group_stats(cl.reshape(4, 4, 4), pl, [5, 40], n, 40, dens_th=1.0, particle_th=1)
    assert both["keep"].tolist() == [True, True]
    one = O.group_stats(cl.reshape(4, 4, 4), pl, [5, 40], n, 40, dens_th=1.0, particle_th=1, root_ok=[True, False])
    assert one["keep"].tolist() == [True, False]
    assert one["particles"].tolist() == both["particles"].tolist()
    assert (one["particle_label"] == np.array([5] * 10 + [-1] * 30)).all()
    assert set(one["cell_label"].ravel().tolist()) == {-1, 5}
