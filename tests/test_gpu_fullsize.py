"""Parity at the benchmark's full size: the 1024^3 box of 2^30 FP32 particles
(L = 1000 Mpc/h, 1.2 million NFW halos, a = 2 cells), in the launch
configuration the benchmark times (the one-call pipeline, hf_find_halos).

- Deposit (step 2, Eq. (1)): the whole 1024^3 grid bit for bit against the
  oracle's C deposit of the same particles.
- CWT (step 3, Eqs. (2)-(4)): 256 cells (the 64 largest and 192 seeded random)
  within 1e-5 of the peak of the oracle's transform of the oracle's density,
  evaluated cell by cell as the stencil of half-width 12 scale lengths (equal to
  the sampled periodic transform to 1e-10 of its peak, pinned on the CPU).
- The pipeline's fused maxima, segmentation and kept-order labels equal the
  stand-alone entry points on the pipeline's own field and cell labels.
- Maxima and segmentation (steps 4-5) at 1024^3 against the oracle on a seeded
  smooth field: every listed maximum is one, the list is complete on 8 blocks
  of 32^3 cells, and 20000 sampled cells get the label the oracle's path
  following gives.
- Labels (step 6) at 1024^3 against the oracle on a seeded random cell
  labelling, for 4 million sampled particles.
"""
import math
import os

import numpy as np
import pytest
import torch

from gpu_helpers import CWT_RTOL, O, ensure_built

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def hfm():
    import paper_2501_10622_amd as m
    return m


@pytest.fixture(scope="module")
def m4():
    ensure_built()
    import synth
    from paper_2501_10622_amd import hf
    cfg = synth.CONFIGS["M4"]
    n, L, kw = cfg.n, cfg.box_len, cfg.kw_list[0]
    print(f"full size: generating the {n}^3 box, {cfg.n_particles} particles", flush=True)
    pos = synth.make_config_box(cfg, device="cuda")
    ctx = hf.context(0)
    bufs = hf.job_buffers(n, pos.shape[0], pos.device, True)
    print("full size: one-call pipeline", flush=True)
    hf.find_halos_async(pos, L, n, kw, bufs, ctx=ctx)
    ctx.sync()
    del bufs["ws"]
    torch.cuda.empty_cache()
    state = {"n": n, "L": L, "kw": kw, "a": cfg.scales_cells[0], "pos": pos, "bufs": bufs, "ctx": ctx}
    yield state
    state.clear()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def rho_oracle(m4):
    from oracle import cic
    print(f"full size: oracle deposit on {THREADS} threads", flush=True)
    pos_h = m4["pos"].cpu().numpy()
    rho = cic.deposit_c(pos_h, m4["L"], m4["n"], 15, threads=THREADS)
    del pos_h
    return rho


def test_deposit_whole_grid_bit_exact(m4, rho_oracle):
    got = m4["bufs"]["rho"].cpu().numpy()
    assert np.array_equal(got, rho_oracle)
    assert O.total_mass(rho_oracle) == m4["pos"].shape[0] << 45


def test_cwt_sampled_cells_against_the_oracle(m4, rho_oracle):
    n, L, kw, a = m4["n"], m4["L"], m4["kw"], m4["a"]
    c = m4["bufs"]["cwt"]
    top = torch.topk(c.view(-1), 64).indices.cpu().numpy()
    rnd = np.random.default_rng(1024).integers(0, n ** 3, size=192)
    cells = np.concatenate([top, rnd])
    got = c.view(-1)[torch.as_tensor(cells, device=c.device)].cpu().numpy().astype(np.float64)
    h = int(math.ceil(12 * a))
    print(f"full size: oracle transform at {cells.size} cells (half-width {h})", flush=True)
    want = O.stencil_cwt_at(rho_oracle, L, kw, h, cells)
    peak = np.abs(want[:64]).max()
    err = np.max(np.abs(got - want)) / peak
    print(f"full size: CWT max error / peak = {err:.2e}", flush=True)
    assert err <= CWT_RTOL


def test_pipeline_equals_the_stand_alone_entry_points(m4):
    n, L = m4["n"], m4["L"]
    b = m4["bufs"]
    cnt = int(b["count"].item())
    mx = hfm().maxima(b["cwt"])
    assert cnt > 0 and torch.equal(mx, b["maxima"][:cnt])
    del mx
    cell = hfm().segment(b["cwt"])
    hfm().sync()
    assert torch.equal(cell, b["cell_label"])
    del cell
    lab = hfm().label(m4["pos"], L, n, b["cell_label"])
    hfm().sync()
    assert torch.equal(lab, b["particle_label"][: m4["pos"].shape[0]])


def test_maxima_and_segmentation_on_a_full_size_field():
    ensure_built()
    import synth
    n = 1024
    print("full size: smooth field, stand-alone maxima and segmentation", flush=True)
    f = synth.smooth_field(n, 2024, device="cuda")
    mx = hfm().maxima(f).cpu().numpy().astype(np.int64)
    cell = hfm().segment(f)
    hfm().sync()
    fh = f.cpu().numpy()
    del f
    ch = cell.cpu().numpy().ravel()
    del cell
    torch.cuda.empty_cache()
    assert mx.size > 100000 and np.all(np.diff(mx) > 0)
    assert O.is_maximum_at(fh, mx).all()  # every listed cell is a maximum
    rng = np.random.default_rng(7)
    listed = set(mx.tolist())
    for corner in rng.integers(0, n - 32, size=(8, 3)):  # the list is complete on 8 blocks
        z, y, x = np.meshgrid(*[np.arange(c, c + 32) for c in corner], indexing="ij")
        blk = ((z * n + y) * n + x).ravel()
        want = blk[O.is_maximum_at(fh, blk)]
        got = np.array(sorted(c for c in blk.tolist() if c in listed), dtype=np.int64)
        assert np.array_equal(np.sort(want), got)
    sample = np.concatenate([rng.integers(0, n ** 3, 19000), mx[rng.integers(0, mx.size, 1000)]])
    print(f"full size: path following from {sample.size} cells", flush=True)
    assert np.array_equal(O.follow(fh, sample), ch[sample].astype(np.int64))
    some = ch[rng.integers(0, n ** 3, 10 ** 7)]
    assert np.isin(some[some >= 0], mx).all()  # every label is a listed maximum


def test_labels_on_a_full_size_box(m4):
    n, L = m4["n"], m4["L"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(61)
    cl = torch.randint(-1, n ** 3, (n, n, n), generator=gen, dtype=torch.int32, device="cuda")
    lab = hfm().label(m4["pos"], L, n, cl)
    hfm().sync()
    idx = np.sort(np.random.default_rng(8).choice(m4["pos"].shape[0], 4_000_000, replace=False))
    ti = torch.as_tensor(idx, device="cuda")
    pos_s = m4["pos"][ti].cpu().numpy()
    got = lab[ti].cpu().numpy()
    clh = cl.cpu().numpy()
    del cl, lab
    assert np.array_equal(got, O.label(pos_s, L, n, clh))
