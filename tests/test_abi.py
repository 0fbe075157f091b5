"""Host-only checks of the C ABI: the library loads, exports every function that
include/hf.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2501_10622_amd as hfm
from paper_2501_10622_amd import hf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hf.LIB_PATH):
        from paper_2501_10622_amd import build
        build.build(verbose=False)
    return hf.load_library()


def _declared():
    text = open(os.path.join(ROOT, "include", "hf.h")).read()
    return sorted(set(re.findall(r"\b(hf_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert set(declared) == set(hf.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(8):
        assert lib.hf_status_str(code)
    assert b"overflow" in lib.hf_status_str(hf.HF_ERR_OVERFLOW).lower()


@pytest.mark.parametrize("n,ok", [(8, True), (12, True), (96, True), (1024, True), (6, False), (10, False),
                                  (9, False), (2048, False), (100, False), (1536, False)])
def test_supported_sizes(lib, n, ok):
    out = ctypes.c_size_t()
    b = hf.Box(n, 15, 10.0)
    code = lib.hf_workspace_size(ctypes.byref(b), 0, hf.STAGE_CWT, ctypes.byref(out))
    assert (code == hf.HF_OK) == ok
    if not ok:
        assert code == hf.HF_ERR_SIZE


def test_frac_bits_and_box_checks(lib):
    out = ctypes.c_size_t()
    for bits, code in ((7, hf.HF_ERR_SIZE), (8, hf.HF_OK), (20, hf.HF_OK), (21, hf.HF_ERR_SIZE)):
        b = hf.Box(16, bits, 10.0)
        assert lib.hf_workspace_size(ctypes.byref(b), 0, hf.STAGE_DEPOSIT, ctypes.byref(out)) == code
    for L in (0.0, -1.0, float("nan"), float("inf")):
        b = hf.Box(16, 15, L)
        assert lib.hf_workspace_size(ctypes.byref(b), 0, hf.STAGE_DEPOSIT, ctypes.byref(out)) == hf.HF_ERR_ARG
    b = hf.Box(16, 15, 10.0)
    assert lib.hf_workspace_size(ctypes.byref(b), -1, hf.STAGE_DEPOSIT, ctypes.byref(out)) == hf.HF_ERR_ARG
    assert lib.hf_workspace_size(ctypes.byref(b), 0, 128, ctypes.byref(out)) == hf.HF_ERR_ARG
    # the stencil stage: three FP32 grids and a few partial sums
    assert lib.hf_workspace_size(ctypes.byref(b), 0, hf.STAGE_STENCIL, ctypes.byref(out)) == hf.HF_OK
    assert 3 * 4 * 16 ** 3 <= out.value <= 3 * 4 * 16 ** 3 + 64 * 1024


def test_workspace_grows_with_n(lib):
    sizes = [hfm.workspace_size(n, 10.0, 0, hf.STAGE_CWT | hf.STAGE_MAXIMA | hf.STAGE_SEGMENT)
             for n in (8, 64, 256)]
    assert sizes == sorted(sizes) and sizes[0] > 0
    # the half spectrum dominates: n * n * (n/2 + 1) complex64
    assert sizes[-1] >= 256 * 256 * 129 * 8


def test_label_stage_keeps_deposit_order_only_where_binned(lib):
    dep_seg = hf.STAGE_DEPOSIT | hf.STAGE_CWT | hf.STAGE_MAXIMA | hf.STAGE_SEGMENT
    assert hf.STAGE_ALL == dep_seg | hf.STAGE_LABEL
    np_ = 1_000_003
    # 192^3 and 256^3 bin the particles into several buckets: the order region
    # (16 B per particle) sits in front of the shared part
    for n in (192, 256):
        plain = hfm.workspace_size(n, 10.0, np_, dep_seg)
        full = hfm.workspace_size(n, 10.0, np_, hf.STAGE_ALL)
        assert full >= plain + 16 * np_ - 12 * np_  # level-1 records move out of the deposit's own part
        assert full > plain
    # a single bucket (64^3) or an unbinned size (B = 18) keeps no order
    assert hfm.workspace_size(64, 10.0, np_, hf.STAGE_ALL) == hfm.workspace_size(64, 10.0, np_, dep_seg)
    assert (hfm.workspace_size(256, 10.0, np_, hf.STAGE_ALL, frac_bits=18) ==
            hfm.workspace_size(256, 10.0, np_, dep_seg, frac_bits=18))
    # the label bit alone needs nothing
    assert hfm.workspace_size(256, 10.0, np_, hf.STAGE_LABEL) == 0


def test_null_context_rejected_before_any_device_call(lib):
    b = hf.Box(16, 15, 10.0)
    vp = ctypes.c_void_p
    assert lib.hf_deposit(None, ctypes.byref(b), vp(0), 0, 0, vp(0), vp(0), 0) == hf.HF_ERR_ARG
    assert lib.hf_cwt(None, ctypes.byref(b), vp(0), 0.1, 0, vp(0), vp(0), 0) == hf.HF_ERR_ARG
    assert lib.hf_maxima(None, ctypes.byref(b), vp(0), 0.0, vp(0), 0, vp(0), vp(0), 0) == hf.HF_ERR_ARG
    assert lib.hf_segment(None, ctypes.byref(b), vp(0), 0.0, vp(0), vp(0), 0) == hf.HF_ERR_ARG
    assert lib.hf_label(None, ctypes.byref(b), vp(0), 0, 0, vp(0), vp(0)) == hf.HF_ERR_ARG
    assert lib.hf_sync(None) == hf.HF_ERR_ARG
    assert lib.hf_destroy(None) == hf.HF_ERR_ARG
    assert lib.hf_cwt_stencil(None, ctypes.byref(b), vp(0), 0.1, 3, vp(0), vp(0), 0) == hf.HF_ERR_ARG
    jobs = (hf.ScaleJob * 1)(hf.ScaleJob(0.1, 0, 0, 0, 0, 0, 0))
    groups = (hf.IdentifyGroups * 1)(hf.IdentifyGroups(0, 0, 0))
    assert lib.hf_identify(None, ctypes.byref(b), vp(0), 0, 0, 0, 0.0, vp(0), 1, jobs, groups, 4.0, 15, vp(0),
                           vp(0), vp(0), 0) == hf.HF_ERR_ARG


def test_identify_workspace(lib):
    # that of the multi-scale step, the group counters (8 B a cell) and one
    # byte per maximum of the largest list; more with more particles
    b = hf.Box(64, 15, 100.0)
    out, base = ctypes.c_size_t(), ctypes.c_size_t()

    def jobs(*caps):
        return (hf.ScaleJob * len(caps))(*[hf.ScaleJob(0.1 * (j + 1), 0, 0, c, 0, 0, 0) for j, c in enumerate(caps)])

    assert lib.hf_find_halos_scales_ws_size(ctypes.byref(b), 100000, 2, ctypes.byref(base)) == hf.HF_OK
    assert lib.hf_identify_ws_size(ctypes.byref(b), 100000, 2, jobs(1000, 5000), ctypes.byref(out)) == hf.HF_OK
    assert out.value >= base.value + 8 * 64 ** 3 + 5000
    small = out.value
    assert lib.hf_identify_ws_size(ctypes.byref(b), 100000, 2, jobs(1000, 50000), ctypes.byref(out)) == hf.HF_OK
    assert out.value >= small + 45000 - 256
    assert lib.hf_identify_ws_size(ctypes.byref(b), 100000, 2, jobs(1000, -1), ctypes.byref(out)) == hf.HF_ERR_ARG
    assert lib.hf_identify_ws_size(ctypes.byref(b), 100000, 0, jobs(1000), ctypes.byref(out)) == hf.HF_ERR_ARG
    assert lib.hf_identify_ws_size(ctypes.byref(b), 100000, 1, None, ctypes.byref(out)) == hf.HF_ERR_ARG


def test_create_out_pointer_checked(lib):
    assert lib.hf_create(0, None, None) == hf.HF_ERR_ARG


def test_serving_footprint_and_summary(lib):
    from paper_2501_10622_amd.serve import Completion, job_footprint, summarize
    small, big = job_footprint(64, 200000), job_footprint(256, 30_000_000)
    assert 0 < small < big
    # outputs alone: 16 B per cell + 4 B per particle, plus workspaces
    assert big > 256 ** 3 * 16 + 30_000_000 * 4
    done = [Completion(i, 64, 1000, 0.01 * i, 0.01 * i + 0.001 * (1 + i % 5)) for i in range(100)]
    s = summarize(done)
    assert s["jobs"] == 100 and s["p50_ms"] <= s["p99_ms"] <= 5.0 + 1e-9
    assert abs(s["particles_per_s"] - 100 * 1000 / s["makespan_s"]) < 1e-6


def test_header_is_plain_c99(tmp_path):
    """include/hf.h is a C header: it compiles as strict C99 (no C++ in the
    ABI), and every struct the entry points take is complete."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_hf.c"
    src.write_text('#include "hf.h"\n'
                   "int main(void) {\n"
                   "    return (int)(sizeof(hf_box) + sizeof(hf_job) + sizeof(hf_cwt_item) + sizeof(hf_group_item)\n"
                   "                 + sizeof(hf_group_filter) + sizeof(hf_scale_job)) == 0;\n"
                   "}\n")
    include = os.path.join(ROOT, "include")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-I", include,
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_stencil_half_width_rule_matches_the_oracle(lib):
    """hf_stencil_half_width (host only) gives the oracle's reading of Table 1's
    gdw_resolution on any grid, and rejects what the stencil kernels cannot take."""
    from oracle import cwthf as O
    h = ctypes.c_int32()
    for kw in (0.0123, 0.05, 0.1, 0.128, 0.256, 0.3, 0.512, 0.75, 1.024, 1.7, 2.5, 4.0):
        for n in (8, 16, 24, 64, 96, 190, 256, 354, 512, 559, 1024):
            want = O.stencil_half_width(kw, n)
            code = lib.hf_stencil_half_width(ctypes.c_double(kw), n, ctypes.byref(h))
            if want <= 64:
                assert code == hf.HF_OK and h.value == want, (kw, n)
            else:
                assert code == hf.HF_ERR_ARG, (kw, n)
    for kw, n in ((0.0, 64), (-1.0, 64), (float("nan"), 64), (float("inf"), 64), (0.5, 0), (0.5, 1025)):
        assert lib.hf_stencil_half_width(ctypes.c_double(kw), n, ctypes.byref(h)) == hf.HF_ERR_ARG
    assert lib.hf_stencil_half_width(ctypes.c_double(0.5), 64, None) == hf.HF_ERR_ARG


def test_cross_scale_rejects_before_any_device_call(lib):
    b = hf.Box(16, 15, 10.0)
    vp = ctypes.c_void_p
    assert lib.hf_cross_scale(None, ctypes.byref(b), vp(0), 0, vp(0), 16, vp(0), vp(0)) == hf.HF_ERR_ARG
