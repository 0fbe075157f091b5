"""GPU parity: every stage of libhf against the FP64 oracle, through the C ABI.

Integer stages (deposit, maxima, segment, label) must be bit-exact.  The FP32
CWT must be within 1e-5 of max |C| of the FP64 oracle.  Maxima, segmentation and
labels are checked stage-isolated (both sides decide on the same FP32 field,
which the oracle produces) and end to end (labels bit-exact on inputs certified
tie-free, else >= 99.99% particle agreement).
"""
import numpy as np
import pytest
import torch

from gpu_helpers import CWT_RTOL, LABEL_AGREEMENT, O, cuda, cwt_error, ensure_built, small_box, tie_free

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    import paper_2501_10622_amd as hfm
    return hfm


def hfm():
    import paper_2501_10622_amd as m
    return m


# --------------------------------------------------------------------------- deposit
@pytest.mark.parametrize("n,L,np_,halos,dtype,bits,seed", [
    (8, 8.0, 1000, 3, "f64", 15, 1),
    (16, 40.0, 20000, 20, "f32", 15, 2),
    (24, 30.0, 30000, 10, "f64", 12, 3),
    (64, 100.0, 64 ** 3, 200, "f64", 15, 1),   # the 64^3 FP64 configuration
    (96, 96.0, 300000, 100, "f32", 16, 4),
    (128, 50.0, 500000, 300, "f32", 8, 5),
    # two-level binned path (more than one coarse bucket)
    (144, 144.0, 300000, 200, "f64", 15, 6),      # 27 buckets of 3^3 tiles
    (192, 190.0, 2000000, 3000, "f32", 17, 7),
    (256, 250.0, 256 ** 3, 20000, "f32", 15, 2),   # the 256^3 FP32 configuration
    (512, 500.0, 3000000, 5000, "f32", 15, 8),
    (432, 432.0, 400000, 100, "f32", 15, 9),        # 16-wide tiles, 162 buckets
    # n not a multiple of 16: binned on the next multiple of 16 above n, then
    # the planes at n folded onto the planes at 0
    (9, 9.0, 5000, 4, "f64", 15, 10),               # padded to 16
    (47, 47.0, 100000, 40, "f32", 15, 11),          # padded to 48: the fold plane is the grid's last
    (101, 90.0, 500000, 200, "f32", 16, 12),        # prime, padded to 112
    (270, 250.0, 2000000, 2000, "f32", 15, 13),     # N_g = Int(400 * 0.3 + 150), padded to 272
    (350, 250.0, 1500000, 1500, "f64", 15, 14),     # N_g for k_w = 0.5, padded to 352
])
def test_deposit_bit_exact(n, L, np_, halos, dtype, bits, seed):
    pos = small_box(n, L, np_, halos, dtype, seed)
    print(f"deposit n={n} np={np_} dtype={dtype} bits={bits}", flush=True)
    got = hfm().deposit(cuda(pos), L, n, bits)
    hfm().sync()
    np.testing.assert_array_equal(got.cpu().numpy(), O.deposit(pos, L, n, bits))


@pytest.mark.parametrize("n", [9, 47, 75, 270])
def test_deposit_last_cells_fold_onto_the_first(n):
    # particles in the last cell along one, two and three axes: their upper
    # corners land on plane n of the padded grid and must reach plane 0
    L = float(n)
    rng = np.random.default_rng(n)
    e = L - 0.3 - 0.5 * rng.random((600, 3))          # inside the last cell
    mid = L * rng.random((600, 3))
    pos = np.concatenate([
        np.column_stack([e[:100, 0], mid[:100, 1], mid[:100, 2]]),
        np.column_stack([mid[100:200, 0], e[100:200, 1], e[100:200, 2]]),
        e[200:400],                                    # the far corner cell
        np.column_stack([e[400:, 0], e[400:, 1], mid[400:, 2]]),
    ]).astype(np.float64)
    print(f"deposit last-cell fold n={n}", flush=True)
    got = hfm().deposit(cuda(pos), L, n, 15)
    hfm().sync()
    want = O.deposit(pos, L, n, 15)
    np.testing.assert_array_equal(got.cpu().numpy(), want)
    assert want[0, 0, 0] > 0 and want[:, :, 0].sum() > 0


def test_deposit_wraps_outside_box_and_edge_cases():
    rng = np.random.default_rng(0)
    L, n = 20.0, 16
    pos = (rng.random((5000, 3)) * 3 * L - L).astype(np.float32)  # [-L, 2L)
    pos[:3] = [[0.0, 0.0, 0.0], [np.nextafter(np.float32(L), 0), 0, 0], [-0.0, -0.0, -0.0]]
    got = hfm().deposit(cuda(pos), L, n)
    hfm().sync()
    np.testing.assert_array_equal(got.cpu().numpy(), O.deposit(pos, L, n))


def test_deposit_empty_and_single():
    z = hfm().deposit(torch.zeros((0, 3), dtype=torch.float32, device="cuda"), 10.0, 8)
    hfm().sync()
    assert int(z.abs().sum()) == 0
    one = np.array([[2.5, 4.5, 7.5]])
    got = hfm().deposit(cuda(one), 8.0, 8)
    hfm().sync()
    np.testing.assert_array_equal(got.cpu().numpy(), O.deposit(one, 8.0, 8))


def test_deposit_order_independent_and_deterministic():
    pos = small_box(32, 50.0, 200000, 50, "f32", 9)
    perm = np.random.default_rng(1).permutation(len(pos))
    a = hfm().deposit(cuda(pos), 50.0, 32).clone()
    b = hfm().deposit(cuda(pos[perm]), 50.0, 32).clone()
    c = hfm().deposit(cuda(pos), 50.0, 32).clone()
    hfm().sync()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_deposit_overflow_detected():
    from paper_2501_10622_amd import HFError, hf
    seven = torch.zeros((7, 3), dtype=torch.float64, device="cuda")
    r = hfm().deposit(seven, 8.0, 8, frac_bits=20)
    hfm().sync()
    assert int(r[0, 0, 0]) == 7 * (1 << 60)
    hfm().deposit(torch.zeros((8, 3), dtype=torch.float64, device="cuda"), 8.0, 8, frac_bits=20)
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == hf.HF_ERR_OVERFLOW
    hfm().sync()  # cleared


def test_deposit_rejects_nonfinite_position():
    from paper_2501_10622_amd import HFError, hf
    pos = torch.tensor([[1.0, 2.0, 3.0], [float("nan"), 0.0, 0.0]], dtype=torch.float32, device="cuda")
    r = hfm().deposit(pos, 8.0, 8)
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == hf.HF_ERR_INPUT
    # the finite particle is still deposited
    np.testing.assert_array_equal(r.cpu().numpy(), O.deposit(np.array([[1.0, 2.0, 3.0]], np.float32), 8.0, 8))


# --------------------------------------------------------------------------- CWT
@pytest.mark.parametrize("n,L,a,kernel,seed", [
    (8, 8.0, 1.5, "sampled", 1),
    (12, 24.0, 1.0, "sampled", 2),
    (16, 16.0, 2.0, "analytic", 3),
    (18, 36.0, 1.2, "sampled", 4),
    (24, 30.0, 2.5, "sampled", 5),
    (48, 60.0, 1.0, "analytic", 6),
    (64, 100.0, 2.0, "sampled", 1),
    (96, 96.0, 3.0, "sampled", 7),
    (128, 128.0, 4.0, "analytic", 8),
    (192, 192.0, 1.5, "sampled", 9),
    (256, 250.0, 2.0, "sampled", 2),
])
def test_cwt_within_tolerance(n, L, a, kernel, seed):
    np_ = min(n ** 3, 2_000_000)
    pos = small_box(n, L, np_, max(1, int(1.2e-3 * L ** 3)), "f32", seed)
    kw = n / (1000.0 * a)
    print(f"cwt n={n} a={a} kernel={kernel}", flush=True)
    rho = hfm().deposit(cuda(pos), L, n)
    c = hfm().cwt(rho, L, kw, kernel)
    hfm().sync()
    ref = O.cwt(O.deposit(pos, L, n), L, kw, kernel)
    err = cwt_error(c.cpu().numpy(), ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err <= CWT_RTOL


def test_cwt_single_point_and_uniform():
    n, L = 32, 32.0
    kw = n / (1000 * 3.0)
    pos = np.array([[10.0, 20.0, 5.0]], dtype=np.float32)
    c = hfm().cwt(hfm().deposit(cuda(pos), L, n), L, kw, "sampled")
    hfm().sync()
    ref = O.cwt(O.deposit(pos, L, n), L, kw, "sampled")
    assert cwt_error(c.cpu().numpy(), ref) <= CWT_RTOL
    # uniform lattice: the zero-mean wavelet gives a flat ~0 field
    g = np.arange(n, dtype=np.float32)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    lat = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    cu = hfm().cwt(hfm().deposit(cuda(lat), L, n), L, kw, "sampled")
    hfm().sync()
    peak = float(np.abs(ref).max())
    assert float(cu.abs().max()) < 1e-5 * peak


def test_cwt_rejects_empty_grid():
    from paper_2501_10622_amd import HFError, hf
    rho = torch.zeros((8, 8, 8), dtype=torch.int64, device="cuda")
    hfm().cwt(rho, 8.0, 0.004)
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == hf.HF_ERR_INPUT


# --------------------------------------------------------------------------- maxima / segment / label
def _oracle_field32(n, L, a, seed, quantise=None):
    pos = small_box(n, L, min(n ** 3, 1_000_000), max(1, int(1.2e-3 * L ** 3)), "f32", seed)
    c64 = O.cwt(O.deposit(pos, L, n), L, n / (1000.0 * a))
    c32 = c64.astype(np.float32)
    if quantise:
        c32 = (np.round(c32 / quantise) * quantise).astype(np.float32)
    return pos, c32


@pytest.mark.parametrize("n,L,a,seed,quant,tau", [
    (8, 8.0, 1.0, 1, None, 0.0),
    (16, 20.0, 1.5, 2, None, 0.0),
    (18, 18.0, 1.0, 3, 0.5, 0.0),      # engineered ties
    (32, 40.0, 2.0, 4, None, 5.0),
    (48, 48.0, 1.0, 5, 2.0, -1.0),    # ties, negative threshold
    (64, 100.0, 2.0, 1, None, 0.0),
    (96, 96.0, 1.5, 6, None, 0.0),
    (256, 250.0, 2.0, 2, None, 0.0),
    (128, 128.0, 1.0, 10, 0.5, 0.0),  # engineered ties, most tiles clear of the periodic faces
    # sizes that leave short resolve tiles: one cell wide (33), odd (47), both
    # axes short by different amounts (75)
    (33, 33.0, 1.0, 7, 0.5, 0.0),
    (47, 47.0, 1.5, 8, None, 0.0),
    (75, 70.0, 2.0, 9, None, 0.0),
])
def test_maxima_segment_label_stage_isolated(n, L, a, seed, quant, tau):
    pos, c32 = _oracle_field32(n, L, a, seed, quant)
    print(f"stages n={n} quant={quant} tau={tau}", flush=True)
    cd = cuda(c32)
    mx = hfm().maxima(cd, tau)
    cell = hfm().segment(cd, tau)
    hfm().sync()
    np.testing.assert_array_equal(mx.cpu().numpy(), O.maxima(c32, tau))
    ref_cell = O.segment(c32, tau)
    np.testing.assert_array_equal(cell.cpu().numpy(), ref_cell)
    part = hfm().label(cuda(pos), L, n, cuda(ref_cell.astype(np.int32)))
    hfm().sync()
    np.testing.assert_array_equal(part.cpu().numpy(), O.label(pos, L, n, ref_cell))


def test_signed_zero_field():
    rng = np.random.default_rng(6)
    c = np.where(rng.random((8, 8, 8)) < 0.5, -0.0, 0.0).astype(np.float32)
    mx = hfm().maxima(cuda(c), -1.0)
    cell = hfm().segment(cuda(c), -1.0)
    hfm().sync()
    assert mx.cpu().tolist() == [511]
    assert bool((cell == 511).all())


def test_maxima_capacity_error():
    from paper_2501_10622_amd import HFError, hf
    _, c32 = _oracle_field32(32, 40.0, 1.0, 11)
    expect = O.maxima(c32, 0.0)
    assert len(expect) > 2
    buf, cnt = hfm().maxima(cuda(c32), 0.0, capacity=2, sync=False)
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == hf.HF_ERR_CAPACITY
    assert int(cnt.item()) == len(expect)
    assert buf[:2].cpu().tolist() == expect[:2].tolist()


def test_nan_field_rejected():
    from paper_2501_10622_amd import HFError, hf
    c = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    c[1, 2, 3] = float("nan")
    hfm().segment(c)
    with pytest.raises(HFError) as e:
        hfm().sync()
    assert e.value.code == hf.HF_ERR_INPUT


# --------------------------------------------------------------------------- end to end
@pytest.mark.parametrize("n,L,np_,halos,dtype,a,seed", [
    (64, 100.0, 64 ** 3, 200, "f64", 2.0, 1),   # 64^3 FP64, one scale
    (32, 40.0, 40000, 60, "f32", 1.5, 12),
    (96, 96.0, 96 ** 3, 106, "f32", 2.5, 13),
])
def test_end_to_end(n, L, np_, halos, dtype, a, seed):
    pos = small_box(n, L, np_, halos, dtype, seed)
    kw = n / (1000.0 * a)
    print(f"e2e n={n} np={np_}", flush=True)
    out = hfm().find_halos(cuda(pos), L, n, kw)
    ref = O.find_halos(pos, L, n, kw)
    np.testing.assert_array_equal(out["rho"].cpu().numpy(), ref["rho"])
    c32 = out["cwt"].cpu().numpy()
    err = cwt_error(c32, ref["cwt"])
    assert err <= CWT_RTOL
    eps = float(np.max(np.abs(c32.astype(np.float64) - ref["cwt"])))
    got_lab = out["particle_label"].cpu().numpy()
    if tie_free(ref["cwt"], eps):
        np.testing.assert_array_equal(out["maxima"].cpu().numpy(), ref["maxima"])
        np.testing.assert_array_equal(out["cell_label"].cpu().numpy(), ref["cell_label"])
        np.testing.assert_array_equal(got_lab, ref["particle_label"])
    else:
        agree = float(np.mean(got_lab == ref["particle_label"]))
        print(f"  not tie-free; particle-label agreement {agree:.6f}", flush=True)
        assert agree >= LABEL_AGREEMENT


@pytest.mark.parametrize("n,L,np_,halos,a,seed,bits", [
    (192, 187.5, 192 ** 3, 7910, 2.0, 31, 15),      # several deposit buckets: labels through the kept order
    (256, 250.0, 3_000_000, 18750, 1.5, 32, 15),
    (288, 300.0, 2_000_001, 30000, 3.0, 33, 12),    # radix-3 grid, odd particle count, other fraction bits
])
def test_labels_through_deposit_order(n, L, np_, halos, a, seed, bits):
    """The one-call pipeline labels particles through the deposit's binned order;
    its labels must equal the separate label stage's on the same cell labels,
    bit for bit, including wrapped, edge and rejected positions, and the
    separate label stage must equal the oracle's on a seeded labelling of the
    grid that both sides are given (no oracle input comes from the GPU)."""
    from paper_2501_10622_amd import hf
    from paper_2501_10622_amd.hf import HFError
    pos = small_box(n, L, np_, halos, "f32", seed)
    pos[:7] = np.array([[L, 0.0, 0.0], [-1e-3, L * 0.5, L - 1e-4], [L * 1.5, -L * 0.25, 2 * L],
                        [np.nextafter(np.float32(L), np.float32(0)), 0.0, 0.0], [0.0, 0.0, 0.0],
                        [L * 0.999999, L * 0.999999, L * 0.999999], [1e-7, 1e-7, 1e-7]], dtype=np.float32)
    pos[11] = [np.nan, 1.0, 1.0]
    kw = n / (1000.0 * a)
    print(f"order labels n={n} np={np_} B={bits}", flush=True)
    d = cuda(pos)
    ctx = hf.context(0)
    bufs = hf.job_buffers(n, np_, d.device, True, bits)
    hf.find_halos_async(d, L, n, kw, bufs, frac_bits=bits, ctx=ctx)
    with pytest.raises(HFError) as e:  # the NaN position is reported ...
        ctx.sync()
    assert e.value.code == hf.HF_ERR_INPUT
    got = bufs["particle_label"][:np_].clone()
    cell = bufs["cell_label"]
    alone = torch.empty_like(got)
    hf.label(d, L, n, cell, out=alone, frac_bits=bits, ctx=ctx)
    with pytest.raises(HFError):
        ctx.sync()
    assert torch.equal(got, alone)
    g = got.cpu().numpy()
    assert g[11] == -1  # ... and its particle gets no label
    ok = np.isfinite(pos).all(axis=1)
    synth_cells = np.random.default_rng(seed).integers(-1, n ** 3, size=(n, n, n), dtype=np.int64).astype(np.int32)
    on_synth = hf.label(d, L, n, cuda(synth_cells), frac_bits=bits, ctx=ctx)
    with pytest.raises(HFError):  # the NaN position again
        ctx.sync()
    np.testing.assert_array_equal(on_synth.cpu().numpy()[ok], O.label(pos[ok], L, n, synth_cells, frac_bits=bits))
    assert on_synth.cpu().numpy()[11] == -1
    # the one-call pipeline finds maxima and segments in one pass over the
    # field: same results as the separate stages on its own CWT
    cnt = int(bufs["count"].item())
    mx_alone = hf.maxima(bufs["cwt"], 0.0, ctx=ctx)
    cell_alone = hf.segment(bufs["cwt"], 0.0, ctx=ctx)
    ctx.sync()
    assert torch.equal(bufs["maxima"][:cnt], mx_alone)
    assert torch.equal(cell, cell_alone)


def test_end_to_end_deterministic():
    pos = cuda(small_box(48, 60.0, 200000, 80, "f32", 21))
    a = hfm().find_halos(pos, 60.0, 48, 0.024)
    b = hfm().find_halos(pos, 60.0, 48, 0.024)
    for k in ("rho", "cwt", "maxima", "cell_label", "particle_label"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("n", [32, 64, 96, 160 // 5 * 3])
def test_segment_long_chains_single_basin(n):
    # one periodic bowl: every cell climbs to a single root across many tiles
    g = np.arange(n)
    d = lambda c0: ((g - c0 + n // 2) % n - n // 2).astype(np.float64)
    r2 = d(5)[:, None, None] ** 2 + d(n - 3)[None, :, None] ** 2 + d(n // 2)[None, None, :] ** 2
    c32 = (1000.0 - r2).astype(np.float32)
    print(f"bowl n={n}", flush=True)
    cell = hfm().segment(cuda(c32), 0.0)
    mx = hfm().maxima(cuda(c32), 0.0)
    hfm().sync()
    np.testing.assert_array_equal(mx.cpu().numpy(), O.maxima(c32, 0.0))
    np.testing.assert_array_equal(cell.cpu().numpy(), O.segment(c32, 0.0))
