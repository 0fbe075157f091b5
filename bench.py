#!/usr/bin/env python
"""Benchmark: the single-scale CWT halo path (deposit -> CWT -> maxima ->
segmentation -> labels) on one MI355X.

One step is one pass of the whole path over one synthetic box that is already
resident in HBM.  Default workload: L = 1000 Mpc/h, 1024^3 grid, 1024^3 FP32
particles (60% in 1.2M NFW halos, 40% uniform, random order), wavelet scale
a = 2 cells (k_w = 0.512), sampled kernel.

Prints ONE JSON line with particles/s, the end-to-end fraction of the HBM
roofline for the model bytes, the dominant kernel's roofline (live HIP-event
timing from the library's kernel timer), and the FP64 oracle timed on a bounded
sample of the same recipe on the host cores.

  python bench.py [--steps K] [--warmup W] [--config M4] [--no-cpu-baseline]
  python bench.py --copy-calibration    # plain copy kernel for HBM counter scaling
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2501_10622_amd", "csrc")

# kernel-timer names of the library -> kernel symbols as rocprofv3 reports them
TIMER_SYMBOLS = {
    "zero_grid": ("fill_u64_kernel",), "deposit": ("tile_accum_kernel",), "label": ("label_kernel",),
    "deposit_atomic": ("deposit_atomic_kernel",),
    "deposit_prep": ("zero_u32_kernel", "l1_scan_kernel", "l1_segs_kernel", "seg_reduce_kernel<0>", "seg_scan_kernel<0>"),
    "deposit_l1_hist": ("l1_hist_kernel",), "deposit_l1_scatter": ("l1_scatter_kernel",),
    "deposit_l2_hist": ("l2_hist_kernel",), "deposit_l2_scatter": ("l2_scatter_kernel",),
    "deposit_fold": ("skirt_fold_kernel",),
    "tables_1": ("tables_stage1",), "tables_2": ("tables_stage2",), "fft_x_fwd": ("fft_x_fwd_kernel",),
    "mass": ("mass_kernel",), "fft_y_fwd": ("fft_y_kernel<false>",), "fft_z_mul": ("fft_z_mul_kernel",),
    "fft_y_inv": ("fft_y_kernel<true>",), "fft_x_inv": ("fft_x_inv_kernel",),
    "maxima_mark": ("max_tile_kernel", "max_direct_kernel"), "maxima_count": ("mask_count_kernel",),
    "maxima_scan": ("seg_reduce_kernel<1>", "seg_scan_kernel<1>"), "maxima_write": ("list_write_kernel",),
    "parent": ("parent_resolve_kernel", "parent_direct_kernel"), "jump_flags": ("fill_flags_kernel",),
    "jump": ("bnd_jump_first_kernel", "bnd_jump_kernel", "jump_direct_kernel"), "finalize": ("seg_finalize_kernel", "finalize_direct_kernel"),
    "label_tiles": ("tile_label_kernel",), "label_level1": ("to_level1_kernel",), "label_input": ("to_input_kernel",),
    "groups_clear": ("groups_clear_kernel",), "groups_cells": ("groups_runs_kernel<false>", "groups_tally_kernel<false>"),
    "groups_particles": ("groups_particles_kernel", "groups_runs_kernel<true>", "groups_tally_kernel<true>"), "groups_decide": ("groups_decide_kernel",),
    "groups_filter": ("groups_filter_kernel",),
    "stencil_x": ("stencil_x_kernel",), "stencil_mass": ("stencil_mass_kernel",),
    "stencil_y": ("stencil_axis_kernel<false>",), "stencil_z": ("stencil_axis_kernel<true>",),
    "claim": ("claim_init_kernel", "claim_filter_kernel"),
}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Stages of one step and the timer names of the launches that make them up.
STAGES = {
    "deposit": ("zero_grid", "deposit_atomic", "deposit_prep", "deposit_l1_hist", "deposit_l1_scatter",
                "deposit_l2_hist", "deposit_l2_scatter", "deposit", "deposit_fold"),
    "cwt_x_fwd": ("tables_1", "tables_2", "fft_x_fwd", "mass"),
    "cwt_y_fwd": ("fft_y_fwd",),
    "cwt_z_mul": ("fft_z_mul",),
    "cwt_y_inv": ("fft_y_inv",),
    "cwt_x_inv": ("fft_x_inv",),
    # the one-call pipeline finds the maxima in the segmentation's parent pass
    "maxima_segment": ("maxima_mark", "maxima_count", "maxima_scan", "maxima_write", "parent",
                       "jump_flags", "jump", "finalize"),
    "label": ("label", "label_tiles", "label_level1", "label_input"),
}


def stage_bytes(n: int, np_: int, pos_bytes: int, scales: int = 1) -> dict:
    """Algorithmic (compulsory) HBM bytes of each stage for one box.

    deposit 12 B/particle (FP32 positions) + 8 B/cell; the transform as five
    pencil sweeps: x forward 8 + 4.01, y 8.02, z*mul*z^-1 8.02, y^-1 8.02, x^-1
    4.01 + 4 (44.06 B/cell); maxima 4 B/cell and segmentation 4 + 4 B/cell,
    one stage since one pass over the field serves both; labels 3 * pos + 4
    (cell label) + 4 (label) B/particle.  Launches that exist only
    because of how a stage is built (histograms, scans, tables, pointer rounds,
    the kept particle order) add no algorithmic bytes.
    """
    cells = n ** 3
    half = n * n * (n // 2 + 1) * 8  # complex64 half spectrum
    # with several scales the deposit and the forward x and y passes run once
    # and everything after them once per scale
    return {
        "deposit": pos_bytes * 3 * np_ + 8 * cells,
        "cwt_x_fwd": 8 * cells + half,
        "cwt_y_fwd": 2 * half,
        "cwt_z_mul": 2 * half * scales,
        "cwt_y_inv": 2 * half * scales,
        "cwt_x_inv": (half + 4 * cells) * scales,
        "maxima_segment": (4 + 8) * cells * scales,
        "label": (pos_bytes * 3 + 4 + 4) * np_ * scales,
    }


def source_digest() -> str:
    """sha256 over the library's HIP sources and its C header: counters taken
    with other sources no longer describe the kernels."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    for f in files + ["../../include/hf.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def short_symbol(name: str) -> str:
    """'void (anonymous namespace)::fft_y_kernel<true>(args...)' -> 'fft_y_kernel<true>'."""
    import re
    m = re.search(r"(?:::|^|\s)([A-Za-z_]\w*)(<[^()]*>)?\(", name)
    if not m:
        return name
    tmpl = m.group(2) or ""
    # keep a template argument only where it names a different pass (fft_y_kernel<INV>, the scans' use)
    return m.group(1) + (tmpl if m.group(1) in ("fft_y_kernel", "seg_reduce_kernel", "seg_scan_kernel",
                                                               "stencil_axis_kernel", "groups_tally_kernel",
                                                               "groups_runs_kernel") else "")


def timer_name(symbol: str):
    for t, syms in TIMER_SYMBOLS.items():
        if symbol in syms:
            return t
    return None


def traffic_file(workload: str) -> str:
    return os.path.join(PROFILES, f"hbm_traffic_{workload}.txt")


def load_traffic(workload: str, digest: str) -> dict:
    """{timer name: [(fetch bytes, write bytes, dispatches per step) per kernel]},
    copy-scaled, from the committed counter summary, or {} if it is missing or
    was taken on other sources."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return {}
    out, ok = {}, False
    for line in open(path):
        if line.startswith("# sources"):
            ok = line.split()[-1] == digest
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "kernel":
            continue
        out.setdefault(f[0], []).append((float(f[3]), float(f[4]), int(f[5])))
    return out if ok else {}


def stage_traffic(counted: dict, stage: str, ran: set):
    """HBM bytes per step of one stage from the counter summary (per-dispatch
    bytes x dispatches per step of the counter run), or None if a launch of the
    stage that ran here has no counters."""
    fetch = write = 0.0
    for t in STAGES[stage]:
        if t not in counted:
            if t in ran:
                return None
            continue
        for f, w, d in counted[t]:
            fetch += f * d
            write += w * d
    return {"fetch_bytes": fetch, "write_bytes": write, "bytes": fetch + write}


def steps_run(bench_line: dict) -> int:
    """Steps a bench run executed: its warmup, the headline steps and as many
    steps with the kernel timer."""
    return bench_line["warmup"] + 2 * bench_line["steps"]


def summarize_profiles(trace_dir: str, pmc_dir: str, workload: str, trace_cmd: str, pmc_cmd: str):
    """Writes the short, committed summaries of a rocprofv3 kernel trace and of
    the FETCH_SIZE / WRITE_SIZE counter runs (copy calibration + one step)."""
    import csv
    import collections
    import glob
    # ---- kernel trace: per-kernel stats of the libhf kernels
    stats = glob.glob(os.path.join(trace_dir, "*_kernel_stats.csv"))[0]
    bench_line = None
    log = os.path.join(os.path.dirname(trace_dir.rstrip("/")), "trace.log")
    if os.path.exists(log):
        for line in open(log):
            if line.startswith("{"):
                bench_line = json.loads(line)
    rows = []
    for r in csv.DictReader(open(stats)):
        sym = short_symbol(r["Name"])
        t = timer_name(sym)
        if t is None:
            continue
        rows.append((t, sym, int(r["Calls"]), float(r["AverageNs"]) / 1e6, float(r["TotalDurationNs"]) / 1e6))
    rows.sort(key=lambda x: -x[4])
    steps = steps_run(bench_line) if bench_line else None
    lines = [f"# rocprofv3 kernel trace, libhf kernels, workload {workload}",
             f"# command: {trace_cmd}",
             f"# bench line of the traced run: ms_per_step={bench_line['ms_per_step'] if bench_line else '?'} "
             f"(steps={bench_line['steps'] if bench_line else '?'}, warmup={bench_line['warmup'] if bench_line else '?'})",
             "# avg_ms = rocprofv3 average duration per dispatch; timer_avg_ms = the library's HIP-event timer in",
             "# the same run (its timer steps); ms/step = total over the run's warmup, headline and timer steps",
             f"{'timer':<20}{'symbol':<26}{'calls':>7}{'avg_ms':>11}{'timer_avg_ms':>14}{'ms/step':>10}"]
    for t, sym, calls, avg, tot in rows:
        tk = (bench_line or {}).get("kernels", {}).get(t)
        tavg = f"{tk['avg_ms']:.4f}" if tk and len(TIMER_SYMBOLS[t]) == 1 else "-"
        per_step = tot / steps if steps else float("nan")
        lines.append(f"{t:<20}{sym:<26}{calls:>7}{avg:>11.4f}{tavg:>14}{per_step:>10.4f}")
    in_step = {t for ts in STAGES.values() for t in ts}
    total = sum(x[4] for x in rows if x[0] in in_step) / steps if steps else float("nan")
    extra = sum(x[4] for x in rows if x[0] not in in_step) / steps if steps else float("nan")
    lines.append(f"# sum of the step's libhf kernels per step (warmup included in the average): {total:.3f} ms")
    lines.append(f"# kernels outside the step (the stencil transform, timed once per step-equivalent): "
                 f"{extra:.3f} ms per call")
    out1 = os.path.join(PROFILES, f"kernel_trace_{workload}.txt")
    with open(out1, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    # ---- counters
    def per_kernel(path):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            agg[short_symbol(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        return agg

    cf = per_kernel(glob.glob(os.path.join(pmc_dir, "copy_FETCH_SIZE_counter_collection.csv"))[0])
    cw = per_kernel(glob.glob(os.path.join(pmc_dir, "copy_WRITE_SIZE_counter_collection.csv"))[0])
    copy_sym = [k for k in cf if "copyBuffer" in k or "copy" in k.lower()][0]
    copy_bytes = 4 << 30
    kib_f = sum(cf[copy_sym]) / len(cf[copy_sym])
    kib_w = sum(cw[copy_sym]) / len(cw[copy_sym])
    ff, fw = copy_bytes / (kib_f * 1024), copy_bytes / (kib_w * 1024)
    mf = per_kernel(glob.glob(os.path.join(pmc_dir, "m4_FETCH_SIZE_counter_collection.csv"))[0])
    mw = per_kernel(glob.glob(os.path.join(pmc_dir, "m4_WRITE_SIZE_counter_collection.csv"))[0])
    digest = None
    runs = 1  # steps the counter run executed
    plog = os.path.join(os.path.dirname(pmc_dir.rstrip("/")), "pmc_m4_FETCH_SIZE.log")
    if os.path.exists(plog):
        for line in open(plog):
            if "libhf sources" in line:
                digest = line.split()[-1]
            if line.startswith("{"):
                runs = steps_run(json.loads(line))
    lines = [f"# HBM traffic per dispatch from rocprofv3 counters, libhf kernels, workload {workload}",
             f"# commands: {pmc_cmd}",
             f"# copy calibration: {copy_sym} of {copy_bytes} B reads FETCH_SIZE {kib_f:.1f} KiB and "
             f"WRITE_SIZE {kib_w:.1f} KiB per dispatch",
             f"# scale factors: fetch x{ff:.4f}, write x{fw:.4f} (bytes = KiB * 1024 * factor)",
             f"# sources {digest or 'unknown'}",
             f"# per dispatch; dispatches = launches per step (the counter run executed {runs} steps)",
             f"{'kernel':<20}{'fetch_KiB':>16}{'write_KiB':>16}{'fetch_B':>18}{'write_B':>18}{'dispatches':>11}"
             "  symbol"]
    for sym in mf:
        t = timer_name(sym)
        if t is None or sym not in mw:
            continue
        f_kib = sum(mf[sym]) / len(mf[sym])
        w_kib = sum(mw[sym]) / len(mw[sym])
        lines.append(f"{t:<20}{f_kib:>16.1f}{w_kib:>16.1f}{f_kib * 1024 * ff:>18.4e}{w_kib * 1024 * fw:>18.4e}"
                     f"{round(len(mf[sym]) / runs):>11}  {sym}")
    with open(traffic_file(workload), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(out1)
    print(traffic_file(workload))


def copy_rate(nbytes: int = 4 << 30, reps: int = 5) -> dict:
    """A plain device-to-device copy of `nbytes`: read + written bytes over the
    average time of `reps` copies, the measured counterpart of the vendor HBM peak."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": ms, "GBps": 2 * nbytes / ms / 1e6}


def copy_calibration():
    """A plain device copy of 4 GiB, for scaling FETCH_SIZE / WRITE_SIZE counters."""
    print(json.dumps(copy_rate()))


def h2d_rate(total_bytes: int, chunk_bytes: int = 1 << 30) -> dict:
    """Host-to-device transfer of `total_bytes` (the positions) from pinned host
    memory, in chunks of `chunk_bytes` into one device buffer."""
    import torch
    chunk = min(chunk_bytes, total_bytes)
    host = torch.empty(chunk, dtype=torch.uint8, pin_memory=True)
    host.fill_(1)
    dev = torch.empty(chunk, dtype=torch.uint8, device="cuda")
    dev.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    left = total_bytes
    while left > 0:
        k = min(chunk, left)
        dev[:k].copy_(host[:k], non_blocking=True)
        left -= k
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e)
    del host, dev
    torch.cuda.empty_cache()
    return {"bytes": total_bytes, "ms": round(ms, 3), "GBps": round(total_bytes / ms / 1e6, 2),
            "method": f"pinned host to device, {chunk >> 20} MiB chunks, one stream"}


def host_info() -> dict:
    model, mem_kb = None, None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    mem_kb = int(line.split()[1])
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cpus": aff,
            "ram_gib": round(mem_kb / 2**20, 1) if mem_kb else None}


def fft_threads() -> int:
    """Worker threads for the multi-threaded CPU FFT: the CPUs this process may
    use, capped by OMP_NUM_THREADS where that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(n, 1)


def cpu_baseline(seed: int) -> dict:
    """The FP64 oracle on a bounded sample of the same recipe: a 256^3 grid box
    with the same cell size, particle density, halo density and scale in cells."""
    import numpy as np
    from oracle import cwthf as O
    import synth
    n, L = 256, 250.0
    np_ = n ** 3
    halos = int(round(1.2e-3 * L ** 3))
    kw = n / (1000.0 * 2.0)
    pos = synth.make_box(L, np_, halos, "f32", seed).numpy()
    t = {}
    t0 = time.perf_counter()
    rho = O.deposit(pos, L, n)
    t["deposit"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    c = O.cwt(rho, L, kw).astype(np.float32)
    t["cwt"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.maxima(c)
    t["maxima"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    cell = O.segment(c)
    t["segment"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.label(pos, L, n, cell)
    t["label"] = time.perf_counter() - t0
    total = sum(t.values())
    # the transform's two 3D FFTs again with scipy's multi-threaded pocketfft (not
    # the oracle: a library timing of the FFT alone, the CWT stage's main cost)
    import scipy.fft as sfft
    workers = fft_threads()
    f = O.normalise(rho)
    t0 = time.perf_counter()
    spec = sfft.rfftn(f, axes=(0, 1, 2), workers=workers)
    sfft.irfftn(spec, s=f.shape, axes=(0, 1, 2), workers=workers)
    fft_mt = time.perf_counter() - t0
    t0 = time.perf_counter()
    spec = np.fft.rfftn(f, axes=(0, 1, 2))
    np.fft.irfftn(spec, s=f.shape, axes=(0, 1, 2))
    fft_1 = time.perf_counter() - t0
    return {"value": np_ / total, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"same recipe at n={n}, L={L:g} Mpc/h, {np_} FP32 particles, {halos} halos, a=2 cells; "
                      f"numpy single-threaded",
            "stage_s": {k: round(v, 3) for k, v in t.items()}, "total_s": round(total, 3),
            "fft_pair_s": {"numpy_1_thread": round(fft_1, 3), "scipy_threads": round(fft_mt, 3),
                           "threads": workers,
                           "what": f"rfftn + irfftn of the normalised {n}^3 FP64 grid"},
            "host": host_info()}


def serving_bench(n_jobs: int, budget_gb: float, n_streams: int, max_batch: int, load: float,
                  sweep: list, big_budget_gb: float) -> dict:
    """Served (continuous batching) against the plain per-request loop on the
    serving workload: grid sizes 64..256, N_p = n^3 U[0.5, 2], scale U[1, 4]
    cells; particles resident (8 pool boxes per size).  Capacity with every
    request waiting at t = 0; latency under Poisson arrivals at `load` times the
    plain loop's capacity, then at each load of `sweep`; capacity and the
    headline load once more with an HBM budget of `big_budget_gb`.  Each budget
    has one server, whose buffer pool a full untimed pass fills first (steady
    state, as a long-running server); it is released before the next budget."""
    import torch
    import synth
    from paper_2501_10622_amd.serve import Request, Server, plain_loop, summarize
    jobs = synth.job_stream(n_jobs, seed=5)
    pool = {}
    for jb in jobs:
        if jb.box_seed not in pool:
            pool[jb.box_seed] = jb.positions("cuda")
    torch.cuda.synchronize()

    def requests(arrivals):
        return [Request(jb.job_id, jb.n, jb.box_len, jb.kw, pool[jb.box_seed], t) for jb, t in zip(jobs, arrivals)]

    def warm_server(gb):
        srv = Server(budget_bytes=int(gb * (1 << 30)), n_streams=n_streams, max_batch=max_batch)
        srv.run(requests([0.0] * len(jobs)))
        return srv

    r = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    plain_loop(requests([0.0] * min(len(jobs), 60)))
    cap_plain = summarize(plain_loop(requests([0.0] * len(jobs))))
    srv = warm_server(budget_gb)
    cap_served = summarize(srv.run(requests([0.0] * len(jobs))))
    groups = dict(srv.stats)
    log(f"serving capacity: plain {cap_plain['jobs_per_s']:.1f} jobs/s, served {cap_served['jobs_per_s']:.1f} jobs/s")

    def at_load(ld, with_plain=True):
        rate = ld * cap_plain["jobs_per_s"]
        arr = synth.poisson_arrivals(len(jobs), rate, seed=5)
        res = {"load": ld, "poisson_rate_per_s": round(rate, 2)}
        if with_plain:
            res["plain"] = r(summarize(plain_loop(requests(arr))))
        res["served"] = r(summarize(srv.run(requests(arr))))
        log(f"serving at load {ld:g} ({rate:.1f} jobs/s, budget {srv.budget / 2**30:g} GB): p50/p99 "
            + (f"plain {res['plain']['p50_ms']:.2f}/{res['plain']['p99_ms']:.2f} ms, " if with_plain else "")
            + f"served {res['served']['p50_ms']:.2f}/{res['served']['p99_ms']:.2f} ms")
        return res

    head = at_load(load)
    out = {"jobs": len(jobs), "pool_boxes": len(pool), "budget_gb": budget_gb, "streams": n_streams,
           "max_batch": max_batch, "capacity": {"plain": r(cap_plain), "served": r(cap_served),
                                                "served_groups": groups},
           "throughput_ratio": round(cap_served["jobs_per_s"] / cap_plain["jobs_per_s"], 3),
           "poisson_rate_per_s": head["poisson_rate_per_s"], "load": load,
           "latency": {"plain": head["plain"], "served": head["served"]}}
    out["load_sweep"] = [at_load(ld) for ld in sweep]
    del srv
    torch.cuda.empty_cache()
    if big_budget_gb > 0:
        srv = warm_server(big_budget_gb)
        cap_big = summarize(srv.run(requests([0.0] * len(jobs))))
        log(f"serving capacity at budget {big_budget_gb:g} GB: {cap_big['jobs_per_s']:.1f} jobs/s")
        out["big_budget"] = {"budget_gb": big_budget_gb, "capacity_served": r(cap_big),
                             "served_groups": dict(srv.stats),
                             "latency_served": at_load(load, with_plain=False)["served"]}
        del srv
        torch.cuda.empty_cache()
    return out


def cwt_summary(stages: dict, cells: int, scales: int = 1) -> dict:
    """The five transform passes together, against the pencil-sweep byte model
    (44.06 B/cell for one scale) and against the strict compulsory bound of
    reading the density once and writing each scale's field (8 + 4 B/cell per
    scale)."""
    parts = [k for k in stages if k.startswith("cwt_")]
    if not parts:
        return {}
    ms = sum(stages[k]["ms_per_step"] for k in parts)
    model = sum(stages[k]["algorithmic_bytes"] for k in parts)
    strict = (8 + 4 * scales) * cells
    return {"ms_per_step": round(ms, 4), "model_bytes": model, "strict_bytes": strict,
            "GBps_model": round(model / ms / 1e6, 1), "frac_model": round(model / ms / 1e6 / HBM_PEAK_GBS, 4),
            "GBps_strict": round(strict / ms / 1e6, 1), "frac_strict": round(strict / ms / 1e6 / HBM_PEAK_GBS, 4)}


def groups_bench(bufs: dict, n: int, np_: int, warmup: int, iters: int, ctx) -> dict:
    """Group statistics and filters (steps 5 and 7, dens_th = 4, particle_th = 15)
    on the step's own outputs: `warmup` untimed calls, then `iters` calls under
    the library's kernel timer (so a trace of the run sees warmup + iters calls,
    as many as the step's launches).  Algorithmic bytes: the cell labels read
    for the volumes and again for the filter, which writes them (12 B/cell), and
    the same for the particle labels (12 B/particle)."""
    import torch
    import paper_2501_10622_amd as hfm
    nmax = int(bufs["count"].item())
    roots, cl, pl = bufs["maxima"][:nmax], bufs["cell_label"], bufs["particle_label"][:np_]
    for _ in range(warmup):
        out = hfm.groups(cl, pl, roots, np_, 4.0, 15, ctx=ctx)
    ctx.sync()
    ctx.profile(True)
    ctx.profile_reset()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(iters):
        out = hfm.groups(cl, pl, roots, np_, 4.0, 15, ctx=ctx)
    stop.record()
    torch.cuda.synchronize()
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    ms = start.elapsed_time(stop) / iters
    kernels = {k: {"ms_per_call": round(v[0] / iters, 4), "launches_per_call": v[1] // iters}
               for k, v in prof.items() if k.startswith("groups_") and v[1]}
    kernel_ms = sum(k["ms_per_call"] for k in kernels.values())
    nbytes = 12 * n ** 3 + 12 * np_
    keep = out["keep"].bool()
    kept = int(keep.sum().item())
    checks = {
        "cells_sum_is_labelled_cells": int(out["cells"].long().sum().item()) == int((cl >= 0).sum().item()),
        "particles_sum_is_labelled_particles": int(out["particles"].long().sum().item()) == int((pl >= 0).sum().item()),
        "kept_particles": int(out["particles"].long()[keep].sum().item()) == int((out["particle_label"] >= 0).sum().item()),
    }
    log(f"groups: {ms:.3f} ms per call, {kept} of {nmax} groups kept")
    return {"what": "group volume, particle number, density >= 4 x mean and >= 15 particles, labels filtered",
            "ms_per_call": round(ms, 4), "kernels": kernels, "groups": nmax, "kept": kept,
            "algorithmic_bytes": nbytes, "GBps": round(nbytes / kernel_ms / 1e6, 1),
            "frac": round(nbytes / kernel_ms / 1e6 / HBM_PEAK_GBS, 4), "checks": checks}


def identify_bench(pos, box_len: float, n: int, ctx, iters: int = 2) -> dict:
    """Sec. 2's identification loop (hf_identify) on the step's box at three
    scales, a = 4, 2 and 1 cells (largest first), dens_th = 4, particle_th = 15:
    one untimed call, then `iters` timed ones; per scale the maxima, the groups
    kept and the particles claimed, with the invariants that every claimed
    particle's root is a kept maximum of its scale and that each scale's kept
    groups hold exactly the particles it claims."""
    import torch
    import paper_2501_10622_amd as hfm
    np_ = pos.shape[0]
    scales = (4.0, 2.0, 1.0)
    kws = [n / (1000.0 * a) for a in scales]
    bufs = hfm.identify_buffers(n, np_, len(kws), pos.device)
    hfm.identify_async(pos, box_len, n, kws, bufs, 4.0, 15, ctx=ctx)
    ctx.sync()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(iters):
        hfm.identify_async(pos, box_len, n, kws, bufs, 4.0, 15, ctx=ctx)
    stop.record()
    torch.cuda.synchronize()
    ctx.sync()
    ms = start.elapsed_time(stop) / iters
    # one more call under the kernel timer: where the time goes
    ctx.profile(True)
    ctx.profile_reset()
    hfm.identify_async(pos, box_len, n, kws, bufs, 4.0, 15, ctx=ctx)
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    kernels = {k: round(v[0], 3) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0]) if v[1]}
    hs = bufs["halo_scale"][:np_]
    per, ok = [], True
    for i in range(len(kws)):
        k = int(bufs["count"][i].item())
        keep = bufs["group_keep"][i][:k].bool()
        mine = hs == i
        claimed = int(mine.sum().item())
        kept_parts = int(bufs["group_particles"][i][:k].long()[keep].sum().item())
        ok = ok and kept_parts == claimed
        ok = ok and bool((bufs["particle_label"][i][:np_][mine] == bufs["halo_root"][:np_][mine]).all().item())
        per.append({"a_cells": scales[i], "kw": kws[i], "maxima": k, "kept": int(keep.sum().item()),
                    "particles_claimed": claimed})
    claimed_all = int((hs >= 0).sum().item())
    del bufs
    torch.cuda.empty_cache()
    log(f"identify (3 scales): {ms:.1f} ms per call, {claimed_all} of {np_} particles claimed")
    return {"what": "identification loop over scales a = 4, 2, 1 cells (steps 2-8, no unbinding), "
                    "dens_th = 4, particle_th = 15", "ms_per_call": round(ms, 3),
            "particles_per_s": np_ / (ms / 1e3), "scales": per, "particles_claimed": claimed_all,
            "kernels_ms_per_call": kernels,
            "checks": {"claimed_equals_kept_group_particles_and_roots": ok}}


def identify_grids_bench(ctx, iters: int = 2) -> dict:
    """The flowchart's own loop (hf_identify_grids): every scale on its own grid
    N_g = Int(400 k_w + 150), the truncated-stencil transform, then steps 5-8,
    and, with velocities, the self-boundness check of steps 9-10.  Workload: a
    phase-space box of L = 250 Mpc/h with 256^3 FP32 particles (20000 NFW halos,
    the M2 recipe plus the synthetic velocity model), k_w = 0.3, 0.5, 0.8
    (N_g = 270, 350, 470), dens_th = 4, particle_th = 15: one untimed call,
    then `iters` timed calls with and without velocities; per scale the maxima,
    the groups steps 7-8 keep, those the check keeps and the particles claimed,
    with the invariant that the particles a scale claims are exactly the bound
    particles of the groups it keeps."""
    import torch
    import paper_2501_10622_amd as hfm
    import synth
    L, npt, halos, seed = 250.0, 256 ** 3, 20000, 2
    kws = [0.3, 0.5, 0.8]
    grids = [hfm.paper_grid(k) for k in kws]
    pos, vel, m_p = synth.make_phase_box(L, npt, halos, "f32", seed, device="cuda")
    gm = synth.G_MPC_KMS2_MSUN * m_p
    bufs = hfm.identify_grids_buffers(grids, npt, pos.device, L, with_velocities=True)
    out = {"what": "the flowchart's loop on per-scale grids N_g = Int(400 k_w + 150) with the stencil transform, "
                   "steps 2-10, dens_th = 4, particle_th = 15",
           "workload": f"L={L:g} Mpc/h, {npt} FP32 particles with velocities, {halos} NFW halos, k_w = "
                       + ", ".join(f"{k:g}" for k in kws), "grids": grids}
    for with_vel in (False, True):
        v = vel if with_vel else None

        def call():
            hfm.identify_grids_async(pos, L, kws, bufs, 4.0, 15, vel=v, grav_mass=gm, ctx=ctx)

        call()
        ctx.sync()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(iters):
            call()
        stop.record()
        torch.cuda.synchronize()
        ctx.sync()
        ms = start.elapsed_time(stop) / iters
        ctx.profile(True)
        ctx.profile_reset()
        call()
        ctx.sync()
        prof = ctx.profile_read()
        ctx.profile(False)
        hs = bufs["halo_scale"][:npt]
        per, ok = [], True
        for i in range(len(kws)):
            k = int(bufs["count"][i].item())
            keep = bufs["group_keep"][i][:k].bool()
            bound = bufs["bound_keep"][i][:k].bool() if with_vel else keep
            mine = hs == i
            claimed = int(mine.sum().item())
            lab = bufs["particle_label"][i][:npt]
            ok = ok and bool((lab[mine] == bufs["halo_root"][:npt][mine]).all().item())
            ok = ok and int((lab >= 0).sum().item()) == claimed
            ok = ok and not bool((bound & ~keep).any().item())
            per.append({"grid": grids[i], "kw": kws[i], "maxima": k, "kept_steps_7_8": int(keep.sum().item()),
                        "kept_steps_9_10": int(bound.sum().item()) if with_vel else None,
                        "particles_claimed": claimed})
        key = "with_velocities" if with_vel else "without_velocities"
        out[key] = {"ms_per_call": round(ms, 3), "scales": per,
                    "particles_claimed": int((hs >= 0).sum().item()),
                    "kernels_ms_per_call": {kk: round(vv[0], 3) for kk, vv in
                                            sorted(prof.items(), key=lambda kv: -kv[1][0]) if vv[1]},
                    "checks": {"claims_are_the_kept_groups_bound_particles": ok}}
        log(f"identify on per-scale grids {grids} ({key}): {ms:.1f} ms per call, "
            f"{out[key]['particles_claimed']} of {npt} claimed")
    del bufs, pos, vel
    torch.cuda.empty_cache()
    return out


def stencil_bench(rho, c_fft, box_len: float, n: int, kw: float, warmup: int, iters: int, ctx) -> dict:
    """Step 3 by the paper's truncated real-space stencil (hf_cwt_stencil with
    Table 1's half-width) on the step's density: `warmup` untimed calls, then
    `iters` under the library's kernel timer (a trace sees warmup + iters calls,
    as many as the step's launches).  Algorithmic bytes: the x pass reads rho
    and writes two FP32 fields (16 B/cell), the y pass reads two and writes two
    (16 B/cell), the z pass reads two and writes C (12 B/cell): 44 B/cell; the
    strict bound reads rho and writes C (12 B/cell).  Also reported: the largest
    difference from the step's FFT field relative to its peak, which is what the
    stencil's truncation changes."""
    import torch
    import paper_2501_10622_amd as hfm
    from paper_2501_10622_amd import hf
    h = hfm.stencil_half_width(kw, n)
    out = torch.empty_like(c_fft)
    ws = torch.empty(hf.workspace_size(n, box_len, 0, hf.STAGE_STENCIL), dtype=torch.uint8, device=rho.device)
    for _ in range(warmup):
        hfm.cwt_stencil(rho, box_len, kw, h, out=out, ctx=ctx, ws=ws)
    ctx.sync()
    ctx.profile(True)
    ctx.profile_reset()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(iters):
        hfm.cwt_stencil(rho, box_len, kw, h, out=out, ctx=ctx, ws=ws)
    stop.record()
    torch.cuda.synchronize()
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    ms = start.elapsed_time(stop) / iters
    kernels = {k: {"ms_per_call": round(v[0] / iters, 4), "launches_per_call": v[1] // iters}
               for k, v in prof.items() if k.startswith("stencil_") and v[1]}
    kernel_ms = sum(k["ms_per_call"] for k in kernels.values())
    cells = n ** 3
    model, strict = 44 * cells, 12 * cells
    per_pass = {"stencil_x": 16 * cells, "stencil_y": 16 * cells, "stencil_z": 12 * cells}
    for k, b in per_pass.items():
        if k in kernels:
            kernels[k]["GBps"] = round(b / kernels[k]["ms_per_call"] / 1e6, 1)
    peak = float(c_fft.abs().max())
    diff = float((out - c_fft).abs().max()) / peak
    del ws, out
    torch.cuda.empty_cache()
    log(f"stencil CWT (half-width {h}): {ms:.3f} ms per call, {model / kernel_ms / 1e6:.0f} GB/s on "
        f"{model // cells} B/cell; "
        f"max |C_stencil - C_fft| = {diff:.3e} of the peak")
    return {"what": "grid CWT by the truncated real-space stencil of Sec. 2.1, seven separable convolutions "
                    "in x, y and z passes",
            "half_width": h, "ms_per_call": round(ms, 4), "kernels": kernels,
            "model_bytes": model, "GBps_model": round(model / kernel_ms / 1e6, 1),
            "frac_model": round(model / kernel_ms / 1e6 / HBM_PEAK_GBS, 4),
            "strict_bytes": strict, "GBps_strict": round(strict / kernel_ms / 1e6, 1),
            "frac_strict": round(strict / kernel_ms / 1e6 / HBM_PEAK_GBS, 4),
            "max_abs_diff_from_fft_rel_peak": diff}


def scales_bench(rho, box_len: float, n: int, kernel: str, iters: int, ctx) -> dict:
    """The transform of the step's density at three scales (a = 1, 2 and 4 cells),
    once with one forward transform for all of them (hf_cwt_scales) and once as
    three separate hf_cwt calls; `iters` timed repetitions of each after one
    untimed one.  The shared form skips two of the three forward x and y passes."""
    import torch
    import paper_2501_10622_amd as hfm
    kws = [n / (1000.0 * a) for a in (1.0, 2.0, 4.0)]
    outs = [torch.empty_like(rho, dtype=torch.float32) for _ in kws]
    ws_multi = torch.empty(hfm.cwt_batch_ws_bytes(n, len(kws)), dtype=torch.uint8, device=rho.device)

    def timed(fn):
        fn()
        ctx.sync()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(iters):
            fn()
        e.record()
        torch.cuda.synchronize()
        ctx.sync()
        return s.elapsed_time(e) / iters

    ms_multi = timed(lambda: hfm.cwt_scales(rho, box_len, kws, kernel, outs=outs, ws=ws_multi, ctx=ctx))
    first = [o.clone() for o in outs]
    ms_sep = timed(lambda: [hfm.cwt(rho, box_len, kw, kernel, out=o, ctx=ctx) for kw, o in zip(kws, outs)])
    same = all(bool(torch.equal(a, b)) for a, b in zip(first, outs))
    del ws_multi, outs, first
    torch.cuda.empty_cache()
    log(f"three scales: {ms_multi:.3f} ms with one forward transform, {ms_sep:.3f} ms as three transforms")
    return {"scales_cells": [1.0, 2.0, 4.0], "ms_shared_forward": round(ms_multi, 4), "ms_separate": round(ms_sep, 4),
            "saved_ms": round(ms_sep - ms_multi, 4), "identical_fields": same}


def filtered_bench(pos, box_len: float, n: int, kw: float, bufs: dict, warmup: int, steps: int, kernel: str, ctx,
                   ms_plain: float) -> dict:
    """The whole step with the group statistics and filters fused in
    (hf_find_halos_filtered: particles counted in the deposit's tile order, the
    filter applied on the way back to input order), timed like the headline,
    and its cost over the plain step.  Its extra algorithmic bytes are the cell
    labels read for the group volumes and read and written by the cell-label
    filter (12 B/cell); the particle counts and filter ride on passes the step
    makes anyway."""
    import torch
    import paper_2501_10622_amd as hfm
    from paper_2501_10622_amd import hf
    np_ = pos.shape[0]
    cap = bufs["maxima"].numel()
    dev = pos.device
    bufs.pop("ws")  # the plain step's workspace makes room for the larger one
    torch.cuda.empty_cache()
    need = hf.workspace_size(n, 1.0, np_, hf.STAGE_ALL | hf.STAGE_GROUPS)
    fb = dict(bufs)
    fb.update(ws=torch.empty(need, dtype=torch.uint8, device=dev),
              group_particles=torch.empty(cap, dtype=torch.int32, device=dev),
              group_cells=torch.empty(cap, dtype=torch.int32, device=dev),
              group_keep=torch.empty(cap, dtype=torch.uint8, device=dev),
              cell_label_kept=torch.empty_like(bufs["cell_label"]))

    def step():
        hfm.find_halos_filtered_async(pos, box_len, n, kw, fb, 4.0, 15, kernel=kernel, ctx=ctx)

    for _ in range(warmup):
        step()
    ctx.sync()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ctx.sync()
    ms = start.elapsed_time(stop) / steps
    ctx.profile(True)
    ctx.profile_reset()
    for _ in range(steps):
        step()
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    kernels = {k: round(v[0] / steps, 4) for k, v in prof.items()
               if v[1] and (k.startswith("groups_") or k.startswith("label_"))}
    cnt = int(fb["count"].item())
    keep = fb["group_keep"][:cnt].bool()
    parts = fb["group_particles"][:cnt].long()
    checks = {
        "kept_particles_are_labelled": int(parts[keep].sum().item()) == int((fb["particle_label"][:np_] >= 0).sum().item()),
        "cells_sum_is_labelled_cells": int(fb["group_cells"][:cnt].long().sum().item())
        == int((fb["cell_label"] >= 0).sum().item()),
    }
    log(f"filtered step: {ms:.3f} ms ({ms - ms_plain:+.3f} over the plain step), {int(keep.sum())} of {cnt} groups kept")
    return {"what": "steps 2-6 with the group statistics and filters of steps 5 and 7 fused in "
                    "(dens_th = 4, particle_th = 15)",
            "ms_per_step": round(ms, 4), "over_plain_ms": round(ms - ms_plain, 4),
            "particles_per_s": np_ / (ms / 1e3), "extra_algorithmic_bytes": 12 * n ** 3,
            "kernels_ms_per_step": kernels, "groups": cnt, "kept": int(keep.sum()), "checks": checks}


def synth_n(config: str) -> int:
    import synth
    return synth.CONFIGS[config].n


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="M4", choices=["M1", "M2", "M3", "M4"])
    ap.add_argument("--kernel", default="sampled", choices=["sampled", "analytic"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-groups", action="store_true", help="skip the group statistics measurement")
    ap.add_argument("--no-stencil", action="store_true", help="skip the real-space stencil CWT measurement")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--summarize-profiles", nargs=2, metavar=("TRACE_DIR", "PMC_DIR"),
                    help="write the committed summaries of a kernel trace and of the counter runs")
    ap.add_argument("--trace-cmd", default="")
    ap.add_argument("--pmc-cmd", default="")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="serving requests (0 skips serving)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-sweep", default="0.5,1.0,1.5", help="further loads for the latency sweep ('' skips)")
    ap.add_argument("--serve-big-budget-gb", type=float, default=250.0, help="second HBM budget (0 skips)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(jobs and boxes are sharded one per GPU by the caller).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    tag = f"{args.config.lower()}_{synth_n(args.config)}"
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles[0], args.summarize_profiles[1], tag, args.trace_cmd,
                           args.pmc_cmd)
        return
    digest = source_digest()
    log(f"libhf sources {digest}")

    import torch
    import paper_2501_10622_amd as hfm
    import synth

    if not os.path.exists(hfm.LIB_PATH):
        from paper_2501_10622_amd import build as _b
        _b.build(verbose=False)
    cfg = synth.CONFIGS[args.config]
    n, L = cfg.n, cfg.box_len
    kws = list(cfg.kw_list)
    kw = kws[0]
    multi = len(kws) > 1  # several scales: one deposit and forward transform, the rest per scale
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"generating {args.config}: n={n} np={cfg.n_particles} on the GPU")
    t0 = time.perf_counter()
    pos = synth.make_config_box(cfg, device=dev)
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    ctx = hfm.context(0)
    if multi:
        bufs = hfm.scales_buffers(n, cfg.n_particles, len(kws), dev)
    else:
        bufs = hfm.job_buffers(n, cfg.n_particles, dev, True)
    log(f"workspace {bufs['ws'].numel() / 2**30:.2f} GiB")

    def step():
        if multi:
            hfm.find_halos_scales_async(pos, L, n, kws, bufs, kernel=args.kernel, ctx=ctx)
        else:
            hfm.find_halos_async(pos, L, n, kw, bufs, kernel=args.kernel, ctx=ctx)

    for i in range(args.warmup):
        step()
        ctx.sync()
        log(f"warmup {i + 1}/{args.warmup} done")

    # the headline: K steps as a caller runs them, the library's kernel timer off
    torch.cuda.synchronize()
    # (an event between steps, on the library's stream, gives each step's time)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    start, stop = evs[0], evs[-1]
    w0 = time.perf_counter()
    start.record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.sync()
    ms_step = start.elapsed_time(stop) / args.steps
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    ms_median = per_step[len(per_step) // 2] if len(per_step) % 2 else \
        0.5 * (per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2])
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, median {ms_median:.3f} "
        f"(wall {1e3 * wall / args.steps:.3f})")
    # the breakdown: K more steps with the kernel timer (HIP events around every
    # launch, on the library's stream); its markers add a little to each step
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    start.record()
    for i in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ctx.sync()
    ms_step_timer = start.elapsed_time(stop) / args.steps
    prof = ctx.profile_read()
    ctx.profile(False)
    log(f"{args.steps} steps with the kernel timer: {ms_step_timer:.3f} ms/step")

    # properties that hold at any size: exact mass, labelled roots are the maxima
    rho = bufs["rho"]
    lo = int((rho & 0xFFFFFFFF).sum().item())
    hi = int((rho >> 32).sum().item())
    mass_ok = (hi << 32) + lo == cfg.n_particles << (3 * 15)
    per_scale = [(bufs["cell_label"][j], bufs["count"][j], bufs["maxima"][j]) for j in range(len(kws))] if multi \
        else [(bufs["cell_label"], bufs["count"], bufs["maxima"])]
    roots_ok, nmaxs = True, []
    for cell, cnt_t, buf in per_scale:
        nmax = int(cnt_t.item())
        nmaxs.append(nmax)
        if nmax:
            roots_ok &= bool((cell.view(-1)[buf[:nmax].long()] == buf[:nmax]).all().item())
    nmax = nmaxs[0] if not multi else nmaxs
    cell, buf = per_scale[0][0], per_scale[0][2]

    pos_bytes = 4 if cfg.dtype == "f32" else 8
    sb = stage_bytes(n, cfg.n_particles, pos_bytes, len(kws))
    kernels = {}
    for name, (ms, launches) in prof.items():
        if launches == 0:
            continue
        kernels[name] = {"ms_per_step": round(ms / args.steps, 4), "launches_per_step": launches // args.steps,
                         "avg_ms": round(ms / launches, 4)}
    counted = load_traffic(tag, digest)
    stages = {}
    for st, timers in STAGES.items():
        ran = [t for t in timers if t in kernels]
        if not ran:
            continue
        ms = sum(kernels[t]["ms_per_step"] for t in ran)
        gbs = sb[st] / ms / 1e6
        stages[st] = {"ms_per_step": round(ms, 4), "launches": {t: kernels[t]["launches_per_step"] for t in ran},
                      "algorithmic_bytes": sb[st], "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                      "traffic": stage_traffic(counted, st, set(ran)) if counted else None}
    dom = max(stages, key=lambda k: stages[k]["ms_per_step"])
    d = stages[dom]
    traffic = d["traffic"]
    model_bytes = sum(sb.values())
    e2e_gbs = model_bytes / ms_step / 1e6
    cells = n ** 3
    out = {
        "metric": "particles/s end-to-end (deposit+CWT+maxima+segmentation+labels) and % of HBM roofline",
        "value": cfg.n_particles / (ms_step / 1e3),
        "unit": "particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(ms_median, 4),
        "ms_per_step_min_max": [round(per_step[0], 4), round(per_step[-1], 4)],
        "ms_per_step_with_kernel_timer": round(ms_step_timer, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: periodic box L={L:g} Mpc/h, {n}^3 grid, {cfg.n_particles} "
                               f"{'FP32' if pos_bytes == 4 else 'FP64'} particles, {cfg.n_halos} NFW halos (60%) + "
                               f"uniform, random order, "
                               + (f"{len(kws)} scales a={'/'.join(f'{a:g}' for a in cfg.scales_cells)} cells "
                                  f"(k_w={'/'.join(f'{k:g}' for k in kws)}; one deposit and forward transform)"
                                  if multi else f"one scale a={cfg.scales_cells[0]:g} cells (k_w={kw:g})")
                               + f", {args.kernel} kernel",
                   "grid": n, "particles": cfg.n_particles, "kw": kws if multi else kw, "kernel": args.kernel,
                   "seed": cfg.seed},
        "cells_per_s": cells / (ms_step / 1e3),
        "e2e_model_bytes": model_bytes,
        "e2e_hbm_roofline_frac": round(e2e_gbs / HBM_PEAK_GBS, 4),
        "roofline": {"kernel": f"{dom} stage", "launches": d["launches"], "bound": "hbm",
                     "achieved": d["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["frac"],
                     "bytes_per_step": sb[dom], "ms_per_step": d["ms_per_step"],
                     "traffic": traffic["bytes"] if traffic else None, "traffic_detail": traffic,
                     "traffic_source": os.path.relpath(traffic_file(tag), ROOT) if traffic else None},
        "stages": stages,
        "cwt": cwt_summary(stages, cells, len(kws)),
        "kernels": kernels,
        "checks": {"mass_exact": mass_ok, "labelled_roots_are_maxima": roots_ok, "maxima": nmax},
    }
    if not multi and not args.no_stencil:
        out["stencil"] = stencil_bench(bufs["rho"], bufs["cwt"], L, n, kw, args.warmup, 2 * args.steps, ctx)
    if not args.no_groups and not multi:
        out["cwt_scales"] = scales_bench(bufs["rho"], L, n, args.kernel, 3, ctx)
        out["groups"] = groups_bench(bufs, n, cfg.n_particles, args.warmup, 2 * args.steps, ctx)
        out["filtered_pipeline"] = filtered_bench(pos, L, n, kw, bufs, args.warmup, args.steps, args.kernel, ctx,
                                                  ms_step)
    del bufs, rho, cell, buf
    torch.cuda.empty_cache()
    if not args.no_groups and not multi:
        out["identify"] = identify_bench(pos, L, n, ctx)
    del pos
    torch.cuda.empty_cache()
    if not args.no_groups and not multi:
        out["identify_grids"] = identify_grids_bench(ctx)
    cp = copy_rate()
    out["hbm_copy_measured"] = {"GBps": round(cp["GBps"], 1), "frac_of_peak": round(cp["GBps"] / HBM_PEAK_GBS, 4),
                                "what": "device copy of 4 GiB (read + write bytes / time), torch copy_"}
    out["roofline"]["frac_of_measured_copy"] = round(d["GBps"] / cp["GBps"], 4)
    out["e2e_frac_of_measured_copy"] = round(e2e_gbs / cp["GBps"], 4)
    log(f"device copy {cp['GBps']:.0f} GB/s")
    h2d = h2d_rate(pos_bytes * 3 * cfg.n_particles)
    h2d["particles_per_s_including_h2d"] = cfg.n_particles / ((ms_step + h2d["ms"]) / 1e3)
    out["h2d_positions"] = h2d
    log(f"positions host to device: {h2d['ms']:.1f} ms ({h2d['GBps']:.1f} GB/s)")
    if args.serve_jobs > 0:
        log(f"serving: {args.serve_jobs} requests")
        sweep = [float(x) for x in args.serve_sweep.split(",") if x.strip()]
        out["serving"] = serving_bench(args.serve_jobs, args.serve_budget_gb, args.serve_streams, args.serve_batch,
                                       args.serve_load, sweep, args.serve_big_budget_gb)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
