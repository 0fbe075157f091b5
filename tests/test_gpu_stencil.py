"""Step 3 by the truncated real-space stencil (Sec. 2.1; hf_cwt_stencil) against
the FP64 oracle's superposition: max |C32 - C64| <= 1e-5 max |C64|, the CWT
tolerance, on seeded clustered boxes whose grids span several tiles with ragged
edges, at sub-cell scales, with the one-tap stencil and with stencils wider
than the box; at 1024^3 on sampled cells in the benchmark's configuration."""
import numpy as np
import pytest
import torch

from gpu_helpers import CWT_RTOL, LABEL_AGREEMENT, O, cuda, cwt_error, ensure_built, small_box, tie_free

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


def hfm():
    import paper_2501_10622_amd as m
    return m


@pytest.mark.parametrize("n,L,np_,halos,a,h", [
    (32, 32.0, 32 ** 3, 40, 1.0, 4),
    (64, 100.0, 64 ** 3, 200, 2.0, 7),     # one full 64 x 64 tile per pass
    (96, 96.0, 300000, 100, 3.0, 5),       # radix 3: ragged x tiles and line tails
    (48, 60.0, 100000, 50, 0.46, 5),       # sub-cell scale (the paper's k_w = 2.5 regime)
    (24, 30.0, 50000, 20, 1.5, 15),        # 2h + 1 = 31 > 24: the stencil wraps onto itself
    (32, 40.0, 60000, 30, 2.5, 12),
    (8, 10.0, 2000, 3, 1.0, 0),            # one tap: C = 6 P f
    (8, 10.0, 2000, 3, 1.0, 9),            # 19 taps on an 8-cell axis
])
def test_stencil_within_tolerance(n, L, np_, halos, a, h):
    pos = small_box(n, L, np_, halos, "f32", 61)
    kw = n / (1000.0 * a)
    print(f"stencil n={n} a={a} h={h}", flush=True)
    rho = hfm().deposit(cuda(pos), L, n)
    c = hfm().cwt_stencil(rho, L, kw, h)
    hfm().sync()
    c64 = O.stencil_cwt(rho.cpu().numpy(), L, kw, h)
    assert cwt_error(c.cpu().numpy(), c64) <= CWT_RTOL


def test_wide_stencils_match_the_fft_path():
    # h = 64 on a 128 box at a = 1.5 cells: the truncation and the one wrapped
    # line weigh exp(-(64/1.5)^2/4) ~ 1e-198, so both paths compute the sampled
    # periodic convolution; each is within 1e-5 of it
    n, L, a = 128, 128.0, 1.5
    pos = small_box(n, L, 400000, 300, "f32", 62)
    kw = n / (1000.0 * a)
    rho = hfm().deposit(cuda(pos), L, n)
    c_st = hfm().cwt_stencil(rho, L, kw, hfm().STENCIL_MAX_HALF_WIDTH)
    c_32 = hfm().cwt_stencil(rho, L, kw, 32)
    c_fft = hfm().cwt(rho, L, kw, "sampled")
    hfm().sync()
    peak = float(c_fft.abs().max())
    for c in (c_st, c_32):
        assert float((c - c_fft).abs().max()) <= 2 * CWT_RTOL * peak


def test_default_half_width_is_table1_extent():
    # the library's rule equals the oracle's on the paper's grids, the 1024^3
    # box's scales and small test grids
    for kw, n in ((0.1, 190), (2.5, 1150 // 2), (0.512, 1024), (1.024, 1024), (0.256, 1024), (0.5, 64),
                  (0.02, 16), (0.05, 24), (0.3, 192)):
        assert hfm().stencil_half_width(kw, n) == O.stencil_half_width(kw, n), (kw, n)
    n, L = 64, 64.0
    pos = small_box(n, L, 100000, 60, "f32", 63)
    kw = 0.02  # Int(75 + 5) = 80 cells of N_g = 158: ceil(80 * 64 / 158) = 33
    assert hfm().stencil_half_width(kw, n) == 33
    rho = hfm().deposit(cuda(pos), L, n)
    a = hfm().cwt_stencil(rho, L, kw)
    b = hfm().cwt_stencil(rho, L, kw, 33)
    hfm().sync()
    assert torch.equal(a, b)  # fixed summation order: deterministic


def test_errors():
    from paper_2501_10622_amd.hf import HF_ERR_ARG, HF_ERR_INPUT, HFError
    n, L = 16, 16.0
    rho = torch.zeros((n, n, n), dtype=torch.int64, device="cuda")
    for h in (-1, 65):
        with pytest.raises(HFError) as e:
            hfm().cwt_stencil(rho, L, 0.5, h)
        assert e.value.code == HF_ERR_ARG
    for kw in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(HFError) as e:
            hfm().cwt_stencil(rho, L, kw, 2)
        assert e.value.code == HF_ERR_ARG
    hfm().cwt_stencil(rho, L, 0.5, 2)  # all-zero grid: found on the device
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == HF_ERR_INPUT
    rho[3, 4, 5] = 1 << 40
    rho[0, 0, 1] = -7
    hfm().cwt_stencil(rho, L, 0.5, 2)
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == HF_ERR_INPUT
    rho[0, 0, 1] = 0
    c = hfm().cwt_stencil(rho, L, 0.5, 2)
    hfm().sync()
    # a unit point: the stencil itself around it, zero beyond the half-width
    s = O.stencil(n, L, O.scale_w(0.5, L), 2) * n ** 3
    got = c.cpu().numpy()
    np.testing.assert_allclose(got[1:6, 2:7, 3:8], s, rtol=1e-5, atol=1e-5 * np.abs(s).max())
    got[1:6, 2:7, 3:8] = 0.0
    assert not got.any()


def test_full_size_sampled_cells():
    # 1024^3 box of 2^30 particles, a = 2 cells: k_w = 0.512, Table 1's 7 cells
    # of N_g = 354 kept at their extent: half-width 21
    import synth
    cfg = synth.CONFIGS["M4"]
    n, L = cfg.n, cfg.box_len
    kw = cfg.kw_list[0]
    h = hfm().stencil_half_width(kw, n)
    assert h == 21
    print(f"stencil full size n={n} kw={kw} h={h}", flush=True)
    pos = synth.make_config_box(cfg, device="cuda")
    rho = hfm().deposit(pos, L, n)
    del pos
    c = hfm().cwt_stencil(rho, L, kw)
    hfm().sync()
    # the 64 largest values (halo cores) and 192 seeded random cells
    top = torch.topk(c.view(-1), 64).indices.cpu().numpy()
    rnd = np.random.default_rng(64).integers(0, n ** 3, size=192)
    cells = np.concatenate([top, rnd])
    got = c.view(-1)[torch.as_tensor(cells, device="cuda")].cpu().numpy().astype(np.float64)
    rho_h = rho.cpu().numpy()
    del rho, c
    want = O.stencil_cwt_at(rho_h, L, kw, h, cells)
    peak = np.abs(want[:64]).max()
    assert np.max(np.abs(got - want)) <= CWT_RTOL * peak


@pytest.mark.parametrize("h", [33, 64])
def test_wide_stencils_on_sampled_cells(h):
    # half-widths whose y- and z-pass tiles need more than 64 KB of LDS (and the
    # widest one accepted), on a box they wrap around several times
    n, L, kw = 64, 64.0, 0.02
    pos = small_box(n, L, 100000, 60, "f32", 66)
    rho = hfm().deposit(cuda(pos), L, n)
    c = hfm().cwt_stencil(rho, L, kw, h)
    hfm().sync()
    print(f"stencil n={n} h={h}", flush=True)
    top = torch.topk(c.view(-1), 16).indices.cpu().numpy()
    rnd = np.random.default_rng(h).integers(0, n ** 3, size=16)
    cells = np.concatenate([top, rnd])
    got = c.view(-1)[torch.as_tensor(cells, device="cuda")].cpu().numpy().astype(np.float64)
    want = O.stencil_cwt_at(rho.cpu().numpy(), L, kw, h, cells)
    peak = np.abs(want[:16]).max()
    assert peak > 0.0
    assert np.max(np.abs(got - want)) <= CWT_RTOL * peak


def test_stencil_kernel_in_the_transform_and_the_pipeline():
    # HF_KERNEL_STENCIL: hf_cwt and hf_find_halos take the paper's truncated
    # stencil with Table 1's extent (k_w = 0.02: ceil(80 * 32 / 158) = 17, a = 1.6 cells)
    n, L, kw = 32, 40.0, 0.02
    pos = small_box(n, L, 40000, 60, "f32", 65)
    rho = hfm().deposit(cuda(pos), L, n)
    a = hfm().cwt(rho, L, kw, "stencil")
    b = hfm().cwt_stencil(rho, L, kw, 17)
    out = hfm().find_halos(cuda(pos), L, n, kw, kernel="stencil")
    hfm().sync()
    assert torch.equal(a, b) and torch.equal(out["cwt"], b)
    ref = O.find_halos(pos, L, n, kw, mode="stencil")
    c32 = out["cwt"].cpu().numpy()
    assert cwt_error(c32, ref["cwt"]) <= CWT_RTOL
    eps = float(np.max(np.abs(c32.astype(np.float64) - ref["cwt"])))
    got = out["particle_label"].cpu().numpy()
    if tie_free(ref["cwt"], eps):
        np.testing.assert_array_equal(out["maxima"].cpu().numpy(), ref["maxima"])
        np.testing.assert_array_equal(got, ref["particle_label"])
    else:
        assert float(np.mean(got == ref["particle_label"])) >= LABEL_AGREEMENT


def test_stencil_kernel_limits():
    from paper_2501_10622_amd.hf import HF_ERR_ARG, HFError
    n, L = 16, 16.0
    rho = torch.ones((n, n, n), dtype=torch.int64, device="cuda")
    # k_w = 0.0005: Int(3000 + 5) = 3005 cells of N_g = 150 make 321 here, above the widest stencil
    with pytest.raises(HFError) as e:
        hfm().cwt(rho, L, 0.0005, "stencil")
    assert e.value.code == HF_ERR_ARG
    with pytest.raises(HFError):
        hfm().stencil_half_width(0.0005, n)
    # the calls that share FFT passes take no stencil
    with pytest.raises(HFError) as e:
        hfm().cwt_scales(rho, L, [0.3, 0.6], "stencil")
    assert e.value.code == HF_ERR_ARG
    with pytest.raises(HFError) as e:
        hfm().cwt_batch([rho, rho], [L, L], [0.3, 0.3], "stencil")
    assert e.value.code == HF_ERR_ARG


def test_stencil_kernel_in_the_filtered_pipeline():
    # the fused group filter on the stencil transform equals the plain step
    # with the same transform followed by hf_groups (tile-order path at 192^3)
    from paper_2501_10622_amd import hf
    n, L, kw = 192, 187.5, 0.3  # h = ceil(10 * 192 / 270) = 8
    pos = cuda(small_box(n, L, 2_000_000, 7910, "f32", 66))
    np_ = pos.shape[0]
    ctx = hf.context(0)
    fb = hf.job_buffers(n, np_, pos.device, True, with_groups=True, with_stencil=True)
    hf.find_halos_filtered_async(pos, L, n, kw, fb, 2.0, 15, kernel="stencil", ctx=ctx)
    pb = hf.job_buffers(n, np_, pos.device, True, with_stencil=True)
    hf.find_halos_async(pos, L, n, kw, pb, kernel="stencil", ctx=ctx)
    ctx.sync()
    cnt = int(pb["count"].item())
    assert cnt == int(fb["count"].item()) and torch.equal(pb["cwt"], fb["cwt"])
    alone = hf.groups(pb["cell_label"], pb["particle_label"][:np_], pb["maxima"][:cnt], np_, 2.0, 15, ctx=ctx)
    ctx.sync()
    assert torch.equal(alone["keep"], fb["group_keep"][:cnt])
    assert torch.equal(alone["particles"], fb["group_particles"][:cnt])
    assert torch.equal(alone["particle_label"], fb["particle_label"][:np_])
    assert 0 < int(alone["keep"].sum()) < cnt
