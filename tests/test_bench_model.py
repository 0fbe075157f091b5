"""The benchmark's algorithmic-byte model (the denominator of every roofline
fraction it reports), checked against totals worked out by hand from the
per-stage compulsory traffic: deposit 12 B per FP32 particle (24 for FP64) plus
8 B per cell; the transform as five half-spectrum sweeps (x forward 8 + 4.01,
y 8.02, z with the multiplier 8.02, y inverse 8.02, x inverse 4.01 + 4 B per
cell); maxima and segmentation 4 + 8 B per cell; labels 12 + 4 + 4 B per
particle.  With several scales the deposit and the forward x and y passes
count once and everything after them once per scale."""
import pytest

import bench


@pytest.mark.parametrize("n,np_,pos_bytes,scales,total_gb", [
    (64, 64 ** 3, 8, 1, 0.032),        # 64^3, FP64 positions
    (256, 256 ** 3, 4, 1, 1.615),      # 256^3
    (512, 512 ** 3, 4, 3, 27.96),      # 512^3 at three scales
    (1024, 1024 ** 3, 4, 1, 103.15),   # 1024^3
])
def test_model_totals(n, np_, pos_bytes, scales, total_gb):
    tot = sum(bench.stage_bytes(n, np_, pos_bytes, scales).values()) / 1e9
    assert abs(tot - total_gb) <= 0.006 * max(total_gb, 1.0)


def test_model_per_cell_and_particle():
    # 64.06 B per cell and 32 B per FP32 particle at one scale, for large n
    n = 1024
    sb = bench.stage_bytes(n, 0, 4)
    per_cell = sum(sb.values()) / n ** 3
    assert abs(per_cell - 64.06) < 0.01
    sp = bench.stage_bytes(n, 1000, 4)
    assert sum(sp.values()) - sum(sb.values()) == 32 * 1000


def test_cwt_summary_strict_bound():
    stages = {k: {"ms_per_step": 1.0, "algorithmic_bytes": v}
              for k, v in bench.stage_bytes(512, 0, 4, 3).items() if k.startswith("cwt_")}
    s = bench.cwt_summary(stages, 512 ** 3, 3)
    assert s["strict_bytes"] == (8 + 4 * 3) * 512 ** 3  # read rho once, write three fields
    assert s["model_bytes"] == sum(v["algorithmic_bytes"] for v in stages.values())
