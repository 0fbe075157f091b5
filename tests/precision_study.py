#!/usr/bin/env python
"""Precision study: the FP32 GPU path against the FP64 oracle, per stage and per scale.

Workload (default): periodic box L = 500 Mpc/h, 512^3 grid, 512^3 FP32 particles
(150000 NFW halos + uniform), three wavelet scales a = 1, 2, 4 cells.  The GPU
computes the CWT with FP32 arithmetic and FP32 accumulation (FP64 only for the
mean density and the twiddle/multiplier tables); the oracle computes
everything in FP64.  For each scale the report gives:

  deposit   cells that differ (must be 0: both are exact integers)
  cwt       max |C32 - C64| / max |C64| and the RMS error relative to RMS(C64)
  maxima    counts, common maxima, and maxima differing
  segment   fraction of cells with the same label
  labels    fraction of particles with the same label
  tie_free  whether C64 is certified tie-free for the FP32 error measured, in
            which case maxima and labels must agree exactly

Run on a GPU host:  python tests/precision_study.py --out precision_m3.json
The oracle work for the scales runs in threads before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cwthf as O  # noqa: E402
import synth  # noqa: E402


def log(msg):
    print(f"[precision] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def tie_free(c64, eps, tau=0.0):
    for (dz, dy, dx) in O.neighbour_offsets()[:13]:
        if np.any(np.abs(c64 - np.roll(c64, (-dz, -dy, -dx), axis=(0, 1, 2))) <= 2 * eps):
            return False
    mx = O.maxima(c64, -np.inf)
    return not np.any(np.abs(c64.ravel()[mx] - tau) <= 2 * eps)


def oracle_scale(rho, pos, L, n, kw):
    t0 = time.perf_counter()
    c = O.cwt(rho, L, kw)
    log(f"kw={kw:g}: oracle cwt done")
    mx = O.maxima(c)
    log(f"kw={kw:g}: oracle maxima done ({mx.size})")
    cell = O.segment(c)
    log(f"kw={kw:g}: oracle segmentation done")
    lab = O.label(pos, L, n, cell)
    return {"cwt": c, "maxima": mx, "cell": cell.astype(np.int32), "label": lab.astype(np.int32),
            "seconds": time.perf_counter() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="M3", choices=list(synth.CONFIGS))
    ap.add_argument("--out", default="precision.json", help="where the JSON report goes")
    ap.add_argument("--skip-tie-check", action="store_true")
    args = ap.parse_args()
    cfg = synth.CONFIGS[args.config]
    n, L = cfg.n, cfg.box_len
    log(f"{args.config}: n={n} np={cfg.n_particles} scales(cells)={cfg.scales_cells}")
    import torch
    pos = synth.make_config_box(cfg, device="cuda" if torch.cuda.is_available() else "cpu").cpu().numpy()
    log("positions generated")
    t0 = time.perf_counter()
    from oracle import cic
    rho64 = cic.deposit_c(pos, L, n, 15, threads=max(1, min(16, len(os.sched_getaffinity(0)))))
    t_dep = time.perf_counter() - t0
    log(f"oracle deposit (C, exact integers) {t_dep:.1f} s")
    with ThreadPoolExecutor(max_workers=len(cfg.kw_list)) as ex:
        futs = [ex.submit(oracle_scale, rho64, pos, L, n, kw) for kw in cfg.kw_list]
        ref = [f.result() for f in futs]
    log("oracle scales done: " + ", ".join(f"{r['seconds']:.0f} s" for r in ref))

    import paper_2501_10622_amd as hfm
    dev = torch.device("cuda", 0)
    pos_d = torch.as_tensor(pos, device=dev)
    report = {"config": args.config, "n": n, "box_len": L, "particles": cfg.n_particles, "halos": cfg.n_halos,
              "gpu_precision": "FP32 FFT/CWT with FP32 accumulation; FP64 mean density and tables",
              "oracle_precision": "FP64 throughout", "oracle_deposit_s": round(t_dep, 1), "scales": []}
    for a, kw, r in zip(cfg.scales_cells, cfg.kw_list, ref):
        out = hfm.find_halos(pos_d, L, n, kw)
        rho = out["rho"].cpu().numpy()
        c32 = out["cwt"].cpu().numpy()
        mx = out["maxima"].cpu().numpy()
        cell = out["cell_label"].cpu().numpy()
        lab = out["particle_label"].cpu().numpy()
        c64 = r["cwt"]
        err = np.abs(c32.astype(np.float64) - c64)
        eps = float(err.max())
        common = np.intersect1d(mx, r["maxima"]).size
        entry = {
            "scale_cells": a, "kw": kw,
            "deposit_cells_differing": int(np.count_nonzero(rho != rho64)),
            "cwt_max_abs_err_rel": eps / float(np.abs(c64).max()),
            "cwt_rms_err_rel": float(np.sqrt(np.mean(err ** 2)) / np.sqrt(np.mean(c64 ** 2))),
            "cwt_max_abs": float(np.abs(c64).max()),
            "maxima_gpu": int(mx.size), "maxima_oracle": int(r["maxima"].size), "maxima_common": int(common),
            "maxima_differing": int(mx.size + r["maxima"].size - 2 * common),
            "cell_label_agreement": float(np.mean(cell.ravel() == r["cell"].ravel())),
            "particle_label_agreement": float(np.mean(lab == r["label"])),
            "oracle_scale_s": round(r["seconds"], 1),
        }
        if not args.skip_tie_check:
            entry["tie_free"] = bool(tie_free(c64, eps))
        report["scales"].append(entry)
        log(json.dumps(entry))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(report, f, indent=1)
    log(f"wrote {args.out}")
    ok = all(e["deposit_cells_differing"] == 0 and e["cwt_max_abs_err_rel"] <= 1e-5 and
             (e.get("tie_free") is False or e["particle_label_agreement"] == 1.0) and
             e["particle_label_agreement"] >= 0.9999 for e in report["scales"])
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
