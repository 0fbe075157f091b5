"""Step 3 at several scales of one grid (hf_cwt_scales): one forward transform
shared by every scale, then a multiplier and inverse transform per scale.
Each scale must give exactly hf_cwt's field (the same arithmetic on the same
spectrum), and be within the FP32 tolerance of the FP64 oracle."""
import numpy as np
import pytest
import torch

from gpu_helpers import CWT_RTOL, O, cuda, cwt_error, ensure_built, small_box

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


def hfm():
    import paper_2501_10622_amd as m
    return m


@pytest.mark.parametrize("n,L,np_,halos,scales,kernel", [
    (64, 100.0, 64 ** 3, 200, (1.0, 2.0, 4.0), "sampled"),
    (96, 96.0, 300000, 100, (1.5, 3.0), "analytic"),      # radix-3 grid
    (256, 250.0, 2_000_000, 20000, (1.0, 2.0, 4.0), "sampled"),
    (48, 60.0, 100000, 50, tuple(1.0 + 0.25 * i for i in range(12)), "sampled"),  # many scales
])
def test_scales_equal_single_scale_transforms(n, L, np_, halos, scales, kernel):
    pos = small_box(n, L, np_, halos, "f32", 51)
    kws = [n / (1000.0 * a) for a in scales]
    print(f"scales n={n} count={len(kws)} kernel={kernel}", flush=True)
    rho = hfm().deposit(cuda(pos), L, n)
    multi = hfm().cwt_scales(rho, L, kws, kernel)
    single = [hfm().cwt(rho, L, kw, kernel).clone() for kw in kws]
    hfm().sync()
    for s, (a, b) in enumerate(zip(multi, single)):
        assert torch.equal(a, b), f"scale {s}"


def test_scales_match_oracle():
    n, L = 32, 40.0
    pos = small_box(n, L, 40000, 60, "f32", 52)
    kws = [n / (1000.0 * a) for a in (1.0, 2.0, 3.0)]
    rho = hfm().deposit(cuda(pos), L, n)
    multi = hfm().cwt_scales(rho, L, kws)
    hfm().sync()
    r64 = O.deposit(pos, L, n)
    for kw, c in zip(kws, multi):
        assert cwt_error(c.cpu().numpy(), O.cwt(r64, L, kw)) <= CWT_RTOL


def test_scales_arguments():
    from paper_2501_10622_amd import HFError, hf
    import ctypes
    rho = hfm().deposit(cuda(small_box(16, 20.0, 2000, 5, "f32", 53)), 20.0, 16)
    hfm().sync()
    b = hf.box(16, 20.0)
    ctx = hfm().context(0)
    k = (ctypes.c_double * 1)(0.01)
    out = torch.empty((16, 16, 16), dtype=torch.float32, device="cuda")
    o = (ctypes.c_void_p * 1)(out.data_ptr())
    ws = torch.empty(hf.cwt_batch_ws_bytes(16, 1), dtype=torch.uint8, device="cuda")
    lib = hf.load_library()
    assert lib.hf_cwt_scales(ctx.handle, ctypes.byref(b), hf._ptr(rho), 0, k, 0, o, hf._ptr(ws), ws.numel()) == hf.HF_ERR_ARG
    assert lib.hf_cwt_scales(ctx.handle, ctypes.byref(b), hf._ptr(rho), 1, k, 0, o, hf._ptr(ws), 16) == hf.HF_ERR_WORKSPACE
    bad = (ctypes.c_double * 1)(-1.0)
    assert lib.hf_cwt_scales(ctx.handle, ctypes.byref(b), hf._ptr(rho), 1, bad, 0, o, hf._ptr(ws), ws.numel()) == hf.HF_ERR_ARG
    assert lib.hf_cwt_scales(ctx.handle, ctypes.byref(b), hf._ptr(rho), 1, k, 0, o, hf._ptr(ws), ws.numel()) == hf.HF_OK
    ctx.sync()
    assert torch.equal(out, hfm().cwt(rho, 20.0, 0.01))


@pytest.mark.parametrize("n,L,np_,halos,scales,bits", [
    (192, 187.5, 2_000_001, 7910, (1.0, 2.0, 4.0), 15),   # binned deposit: labels through the kept order
    (48, 60.0, 200_000, 80, (1.5, 3.0), 12),              # one bucket: labels by gather
])
def test_scales_pipeline_equals_single_scale_pipeline(n, L, np_, halos, scales, bits):
    """hf_find_halos_scales (one deposit, one forward transform) gives every
    scale exactly hf_find_halos's outputs at that scale."""
    from paper_2501_10622_amd import hf
    pos = cuda(small_box(n, L, np_, halos, "f32", 54))
    kws = [n / (1000.0 * a) for a in scales]
    print(f"scales pipeline n={n} count={len(kws)}", flush=True)
    ctx = hf.context(0)
    mb = hf.scales_buffers(n, np_, len(kws), pos.device, bits)
    hf.find_halos_scales_async(pos, L, n, kws, mb, frac_bits=bits, ctx=ctx)
    ctx.sync()
    for j, kw in enumerate(kws):
        sb = hf.job_buffers(n, np_, pos.device, True, bits)
        hf.find_halos_async(pos, L, n, kw, sb, frac_bits=bits, ctx=ctx)
        ctx.sync()
        assert torch.equal(mb["rho"], sb["rho"])
        assert torch.equal(mb["cwt"][j], sb["cwt"]), f"cwt scale {j}"
        cnt = int(sb["count"].item())
        assert int(mb["count"][j].item()) == cnt
        assert torch.equal(mb["maxima"][j][:cnt], sb["maxima"][:cnt])
        assert torch.equal(mb["cell_label"][j], sb["cell_label"]), f"cells scale {j}"
        assert torch.equal(mb["particle_label"][j][:np_], sb["particle_label"][:np_]), f"labels scale {j}"
