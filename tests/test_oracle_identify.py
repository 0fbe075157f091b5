"""Pins for the oracle's identification loop over scales (Sec. 2 steps 2-8 and
the flowchart's pair of grids; unbinding excluded).

- With one scale it reduces to the single-scale path followed by the group
  filters, the cross-scale check made against the all-zero grid.
- A pure-Python recount from each scale's own step-6 labels (computed here by
  the single-scale functions) fixes the bookkeeping: which particles a scale
  may still take, the particle numbers of its groups, the keep decision in
  exact integers, and which scale claims each particle.
- The Gaussian-blob closed form (the centre response of a blob of width s
  peaks at w* = sqrt(6/7)/s) predicts which scale claims a compact and which
  an extended halo.
"""
import math

import numpy as np
import pytest

from oracle import cwthf as O


def _box(seed, L=64.0):
    rng = np.random.default_rng(seed)
    blobs = [rng.normal(loc=c, scale=s, size=(m, 3)) for c, s, m in
             zip(rng.random((8, 3)) * L, rng.uniform(0.5, 4.0, 8), rng.integers(500, 6000, 8))]
    return (np.concatenate(blobs + [rng.random((20000, 3)) * L]) % L).astype(np.float32)


def test_one_scale_is_the_single_scale_path_and_filters():
    pos, L, n = _box(1), 64.0, 32
    kw = n / (1000.0 * 1.5)
    r = O.identify(pos, L, n, [kw], 2.0, 15)
    s = O.find_halos(pos, L, n, kw)
    c = s["cwt"]
    _, val = O.peaks(c, s["maxima"], L)  # against the zero grid: the corrected value must be positive
    ok = val > 0.0
    g = O.group_stats(s["cell_label"], s["particle_label"], s["maxima"], n, len(pos), 2.0, 15, root_ok=ok)
    assert (r["scales"][0]["keep"] == g["keep"]).all()
    assert (r["halo_root"] == g["particle_label"]).all()
    assert ((r["halo_scale"] == 0) == (g["particle_label"] >= 0)).all()


@pytest.mark.parametrize("seed,dens_th,pth", [(2, 1.0, 5), (3, 2.0, 15), (4, 0.5, 30)])
def test_bookkeeping_by_brute_force(seed, dens_th, pth):
    pos, L, n = _box(seed), 64.0, 32
    kws = [n / (1000.0 * a) for a in (3.0, 2.0, 1.5, 1.0)]
    r = O.identify(pos, L, n, kws, dens_th, pth)
    npt = len(pos)
    claimed = [-1] * npt
    root_of = [-1] * npt
    fields = [O.cwt(r["rho"], L, kw) for kw in kws]
    for i, kw in enumerate(kws):
        sc = r["scales"][i]
        cell = O.segment(fields[i])
        raw = O.label(pos, L, n, cell).tolist()
        roots = O.maxima(fields[i]).tolist()
        assert sc["maxima"].tolist() == roots
        cells, parts = {}, {}
        for v in cell.ravel().tolist():
            if v >= 0:
                cells[v] = cells.get(v, 0) + 1
        for p in range(npt):
            if claimed[p] < 0 and raw[p] >= 0:
                parts[raw[p]] = parts.get(raw[p], 0) + 1
        nxt = fields[i + 1] if i + 1 < len(kws) else np.zeros_like(fields[i])
        # step 4's corrected value and position of each maximum (one grid: no cube-size term)
        ppos, pval = O.peaks(fields[i], roots, L) if roots else (np.zeros((0, 3)), np.zeros(0))
        keep = {}
        for k, rt in enumerate(roots):
            x, y, z = (int(math.floor(ppos[k][a] / (L / n) + 0.5)) % n for a in range(3))
            near = max(nxt[(z + a) % n, (y + b) % n, (x + c) % n]
                       for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1))
            p_, c_ = parts.get(rt, 0), cells.get(rt, 0)
            keep[rt] = (pval[k] > near and p_ * n ** 3 >= dens_th * c_ * npt and p_ >= pth)
            assert sc["particles"][k] == p_ and sc["cells"][k] == c_
            assert bool(sc["keep"][k]) == keep[rt]
        for p in range(npt):
            if claimed[p] < 0 and raw[p] >= 0 and keep[raw[p]]:
                claimed[p] = i
                root_of[p] = raw[p]
    assert r["halo_scale"].tolist() == claimed
    assert r["halo_root"].tolist() == root_of
    assert len(set(claimed) - {-1}) >= 2 or seed != 2  # the first case claims at more than one scale


def test_one_grid_per_scale_given_explicitly_is_the_default():
    pos, L, n = _box(6), 64.0, 32
    kws = [n / (1000.0 * a) for a in (3.0, 1.5)]
    a = O.identify(pos, L, n, kws, 2.0, 15)
    b = O.identify(pos, L, n, kws, 2.0, 15, grids=[n, n])
    assert (a["halo_scale"] == b["halo_scale"]).all() and (a["halo_root"] == b["halo_root"]).all()
    assert b["grids"] == [n, n]


@pytest.mark.parametrize("seed,grids,scales,dens_th,pth", [
    (7, (24, 32, 40), (2.5, 2.0, 1.5), 1.0, 5),      # finer grid per smaller scale, as the flowchart's N_g
    (9, (40, 30, 36), (3.0, 2.2, 1.6), 1.0, 5),      # not monotone: the comparison still crosses grids
])
def test_per_scale_grids_by_brute_force(seed, grids, scales, dens_th, pth):
    # scales given in cells of a 32^3 grid; each scale is deposited, transformed,
    # segmented and labelled on its own grid, and step 8 compares across grids
    pos, L = _box(seed), 64.0
    kws = [32 / (1000.0 * a) for a in scales]
    r = O.identify(pos, L, 32, kws, dens_th, pth, grids=list(grids))
    assert r["grids"] == list(grids)
    npt = len(pos)
    claimed = [-1] * npt
    root_of = [-1] * npt
    fields = [O.cwt(O.deposit(pos, L, g), L, kw) for g, kw in zip(grids, kws)]
    for i, (g, kw) in enumerate(zip(grids, kws)):
        sc = r["scales"][i]
        cell = O.segment(fields[i])
        raw = O.label(pos, L, g, cell).tolist()
        roots = O.maxima(fields[i]).tolist()
        assert sc["maxima"].tolist() == roots
        cells, parts = {}, {}
        for v in cell.ravel().tolist():
            if v >= 0:
                cells[v] = cells.get(v, 0) + 1
        for p in range(npt):
            if claimed[p] < 0 and raw[p] >= 0:
                parts[raw[p]] = parts.get(raw[p], 0) + 1
        nxt = fields[i + 1] if i + 1 < len(grids) else np.zeros_like(fields[i])
        gn = nxt.shape[0]
        ppos, pval = O.peaks(fields[i], roots, L) if roots else (np.zeros((0, 3)), np.zeros(0))
        _, _, l1b, l2b = O._peak_fits(fields[i], roots) if roots else (None, None, [], [])
        keep = {}
        for k, rt in enumerate(roots):
            v = pval[k] + 0.3125 * (2 * l2b[k] - l1b[k]) * (1 - (g / gn) ** 2)  # App. B, 3/5 removed
            x, y, z = (int(math.floor(ppos[k][a] / (L / gn) + 0.5)) % gn for a in range(3))
            near = max(nxt[(z + a) % gn, (y + b) % gn, (x + c) % gn]
                       for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1))
            p_, c_ = parts.get(rt, 0), cells.get(rt, 0)
            keep[rt] = (v > near and p_ * g ** 3 >= dens_th * c_ * npt and p_ >= pth)
            assert sc["particles"][k] == p_ and sc["cells"][k] == c_
            assert bool(sc["keep"][k]) == keep[rt]
        for p in range(npt):
            if claimed[p] < 0 and raw[p] >= 0 and keep[raw[p]]:
                claimed[p] = i
                root_of[p] = raw[p]
    assert r["halo_scale"].tolist() == claimed
    assert r["halo_root"].tolist() == root_of
    assert sum(bool(sc["keep"].any()) for sc in r["scales"]) >= 2  # more than one scale keeps groups


def test_paper_grid_schedule():
    # step 1 / the flowchart: N_g = Int(400 k_w + 150)
    for kw, ng in ((0.1, 190), (0.5, 350), (1.0, 550), (2.5, 1150), (0.0123, 154)):
        assert O.paper_grid(kw) == ng


def test_compact_and_extended_halos_claimed_at_their_scales():
    # blob response at its centre peaks at scale length a* = s / sqrt(6/7):
    # extended s = 4 Mpc/h -> a* = 2.2 cells (dx = 2): claimed at a = 2 cells,
    # which beats a = 1 there and loses to nothing coarser it is compared with;
    # compact s = 0.7 -> a* = 0.38 cells: every listed scale is coarser, so the
    # finest (a = 1, compared with the zero grid) claims it
    rng = np.random.default_rng(0)
    L, n = 64.0, 32
    ext, cmp_ = np.array([44.0, 40.0, 30.0]), np.array([20.0, 20.0, 20.0])
    pos = np.concatenate([rng.normal(loc=cmp_, scale=0.7, size=(3000, 3)),
                          rng.normal(loc=ext, scale=4.0, size=(20000, 3)),
                          rng.random((30000, 3)) * L]).astype(np.float32) % L
    scales = (4.0, 2.0, 1.0)
    assert 2.0 < 4.0 / math.sqrt(6.0 / 7.0) / (L / n) < 4.0
    r = O.identify(pos, L, n, [n / (1000.0 * a) for a in scales], 4.0, 15)

    def near(root, p):
        z, y, x = root // (n * n), (root // n) % n, root % n
        d = [min(abs(a - b), n - abs(a - b)) for a, b in zip((x, y, z), np.round(p / 2).astype(int) % n)]
        return max(d) <= 1

    sc, rt = r["halo_scale"], r["halo_root"]
    core_ext = np.linalg.norm(pos[3000:23000] - ext, axis=1) < 2.0
    assert core_ext.any() and (sc[3000:23000][core_ext] == 1).all()
    core_cmp = np.linalg.norm(pos[:3000] - cmp_, axis=1) < 0.5
    assert core_cmp.any() and (sc[:3000][core_cmp] == 2).all()
    assert near(int(rt[3000 + int(np.argmin(np.linalg.norm(pos[3000:23000] - ext, axis=1)))]), ext)
    assert near(int(rt[int(np.argmin(np.linalg.norm(pos[:3000] - cmp_, axis=1)))]), cmp_)


def test_scales_must_increase():
    pos = _box(5)
    with pytest.raises(ValueError):
        O.identify(pos, 64.0, 16, [0.02, 0.01])
    with pytest.raises(ValueError):
        O.identify(pos, 64.0, 16, [])
