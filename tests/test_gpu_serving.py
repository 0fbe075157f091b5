"""Serving parity: batched and served results are bit-identical to stand-alone runs."""
import numpy as np
import pytest
import torch

from gpu_helpers import O, cuda, ensure_built, small_box

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


@pytest.mark.parametrize("n", [64, 192, 256])
def test_cwt_batch_matches_single(n):
    import paper_2501_10622_amd as hfm
    rhos, Ls, kws = [], [], []
    for j, (L, a) in enumerate([(64.0, 1.0), (100.0, 2.5), (80.0, 4.0), (64.0, 1.7)]):
        L = L * n / 64.0
        pos_np = small_box(n, L, 200000 * (n // 64) ** 2, 40 * (n // 64) ** 3, "f32", 30 + j + n)
        pos = cuda(pos_np)
        rhos.append(hfm.deposit(pos, L, n).clone())
        Ls.append(L)
        kws.append(n / (1000.0 * a))
        if j == 1:
            from oracle import cic
            rho_or = cic.deposit_c(pos_np, L, n, threads=8)
    print(f"cwt batch n={n}", flush=True)
    for kernel in ("sampled", "analytic"):
        outs = hfm.cwt_batch(rhos, Ls, kws, kernel)
        singles = [hfm.cwt(r, L, k, kernel).clone() for r, L, k in zip(rhos, Ls, kws)]
        hfm.sync()
        for o, s in zip(outs, singles):
            assert torch.equal(o, s)
        # one member against the oracle (its own density, its own transform)
        assert np.array_equal(rhos[1].cpu().numpy(), rho_or)
        ref = O.cwt(rho_or, Ls[1], kws[1], kernel)
        err = np.max(np.abs(outs[1].cpu().numpy().astype(np.float64) - ref)) / np.max(np.abs(ref))
        assert err <= 1e-5


def test_group_matches_alone_and_oracle():
    import paper_2501_10622_amd as hfm
    n = 96
    entries, alone = [], []
    for j, a in enumerate([1.2, 3.5, 2.0]):
        L = float(n)
        pos_np = small_box(n, L, 400000 + 1000 * j, 106, "f32", 40 + j)
        pos = cuda(pos_np)
        kw = n / (1000.0 * a)
        alone.append(hfm.find_halos(pos, L, n, kw))
        bufs = hfm.job_buffers(n, pos.shape[0], pos.device, with_cwt_ws=False)
        entries.append((pos, L, kw, bufs, pos_np))
    ws = torch.empty(hfm.cwt_batch_ws_bytes(n, len(entries)), dtype=torch.uint8, device="cuda")
    hfm.find_halos_group_async(n, [e[:4] for e in entries], ws)
    hfm.sync()
    for (pos, L, kw, bufs, pos_np), ref in zip(entries, alone):
        cnt = int(bufs["count"].item())
        assert torch.equal(bufs["rho"], ref["rho"])
        assert torch.equal(bufs["cwt"], ref["cwt"])
        assert torch.equal(bufs["maxima"][:cnt], ref["maxima"])
        assert torch.equal(bufs["cell_label"], ref["cell_label"])
        assert torch.equal(bufs["particle_label"][: pos.shape[0]], ref["particle_label"])
    # one member against the oracle: exact density, CWT within tolerance
    pos, L, kw, bufs, pos_np = entries[1]
    np.testing.assert_array_equal(bufs["rho"].cpu().numpy(), O.deposit(pos_np, L, n))
    ref = O.cwt(O.deposit(pos_np, L, n), L, kw)
    err = np.max(np.abs(bufs["cwt"].cpu().numpy().astype(np.float64) - ref)) / np.max(np.abs(ref))
    assert err <= 1e-5


def _requests(n_jobs, rate, sizes=(64, 96, 128), boxes_per_size=2, device="cpu"):
    import synth
    from paper_2501_10622_amd.serve import Request
    jobs = synth.job_stream(n_jobs, seed=11, sizes=sizes, boxes_per_size=boxes_per_size)
    arrivals = synth.poisson_arrivals(n_jobs, rate, seed=11)
    pool = {}
    reqs = []
    for jb, t in zip(jobs, arrivals):
        if jb.box_seed not in pool:
            pool[jb.box_seed] = jb.positions(device).cuda()
        reqs.append(Request(jb.job_id, jb.n, jb.box_len, jb.kw, pool[jb.box_seed], t))
    return reqs


@pytest.mark.parametrize("budget_jobs,max_batch,sizes", [(1000, 8, (64, 96, 128)), (3, 4, (64, 96, 128)),
                                                         (1000, 4, (192, 256)), (2, 2, (192, 256))])
def test_served_equals_plain(budget_jobs, max_batch, sizes):
    from paper_2501_10622_amd.serve import Server, job_footprint, plain_loop, summarize
    large = sizes[0] >= 192
    print(f"served vs plain sizes={sizes} budget={budget_jobs} jobs", flush=True)
    reqs = _requests(10 if large else 24, rate=2000.0, sizes=sizes, boxes_per_size=1 if large else 2,
                     device="cuda" if large else "cpu")
    biggest = max(job_footprint(r.n, r.pos.shape[0]) for r in reqs)
    keep = frozenset(r.job_id for r in reqs)
    plain = {c.job_id: c for c in plain_loop(reqs, keep_outputs=keep)}
    srv = Server(budget_bytes=budget_jobs * biggest, n_streams=4, max_slots=16, max_batch=max_batch)
    served = srv.run(reqs, keep_outputs=keep)
    assert len(served) == len(reqs)
    for c in served:
        p = plain[c.job_id]
        for k in ("maxima", "cell_label", "particle_label"):
            assert torch.equal(c.outputs[k], p.outputs[k]), (c.job_id, k)
        assert c.done >= c.arrival
    s = summarize(served)
    assert s["jobs"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0
    # everything the server held (in-flight and idle buffer sets, transform workspaces) stayed in budget
    assert 0 < srv.stats["peak_resident"] <= srv.budget
    if budget_jobs <= 3:
        assert srv.stats["groups"] >= len(reqs) // max_batch
