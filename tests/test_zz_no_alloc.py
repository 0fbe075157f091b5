"""hf_find_halos_noalloc (the allocation-free entry point, for callers that
cannot allocate device memory) against hf_find_halos through the C ABI: two
calls in a row, the second on a smaller box, each bit-identical to the
entry point that takes a caller workspace; a job beyond the scratch array is
rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

from gpu_helpers import cuda, ensure_built, small_box

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


def _run(hf, pos, L, n, kw, noalloc, kernel="sampled"):
    bufs = hf.job_buffers(n, pos.shape[0], pos.device, True, with_stencil=kernel == "stencil")
    for k in ("rho", "cwt", "maxima", "cell_label", "particle_label"):
        bufs[k].fill_(-7)  # stale values must not survive into the results
    ctx = hf.context(pos.device.index)
    if noalloc:
        hf.find_halos_noalloc_async(pos, L, n, kw, bufs, kernel=kernel, ctx=ctx)
    else:
        hf.find_halos_async(pos, L, n, kw, bufs, kernel=kernel, ctx=ctx)
    ctx.sync()
    cnt = int(bufs["count"].item())
    return {"rho": bufs["rho"], "cwt": bufs["cwt"], "maxima": bufs["maxima"][:cnt],
            "cell_label": bufs["cell_label"], "particle_label": bufs["particle_label"][:pos.shape[0]]}


def test_noalloc_equals_the_workspace_entry_point_twice():
    from paper_2501_10622_amd import hf
    cases = [(128, 128.0, 2 * 128 ** 3, 900, 81, 1.5, "sampled"),   # the largest serving box that fits
             (64, 64.0, 150000, 80, 82, 2.0, "sampled"),            # then a smaller one
             (48, 60.0, 100000, 60, 83, 1.2, "stencil")]            # and the other transform
    for n, L, np_, halos, seed, a, kernel in cases:
        print(f"noalloc n={n} np={np_} kernel={kernel}", flush=True)
        need = hf.workspace_size(n, L, np_, hf.STAGE_ALL | (hf.STAGE_STENCIL if kernel == "stencil" else 0))
        assert need <= hf.NOALLOC_SCRATCH_BYTES
        pos = cuda(small_box(n, L, np_, halos, "f32", seed))
        kw = n / (1000.0 * a)
        want = _run(hf, pos, L, n, kw, False, kernel)
        got = _run(hf, pos, L, n, kw, True, kernel)
        for k in want:
            assert torch.equal(got[k], want[k]), k
        assert got["maxima"].numel() > 0 and int((got["particle_label"] >= 0).sum()) > 0


def test_noalloc_rejects_jobs_beyond_the_scratch_array():
    from paper_2501_10622_amd import hf
    n, np_ = 192, 2 * 192 ** 3
    assert hf.workspace_size(n, 192.0, np_, hf.STAGE_ALL) > hf.NOALLOC_SCRATCH_BYTES
    pos = torch.zeros((np_, 3), dtype=torch.float32, device="cuda")
    bufs = hf.job_buffers(n, np_, pos.device, False)
    with pytest.raises(hf.HFError) as e:
        hf.find_halos_noalloc_async(pos, 192.0, n, 0.1, bufs)
    assert e.value.code == hf.HF_ERR_WORKSPACE
    hf.context(0).sync()  # nothing was enqueued, nothing reported
