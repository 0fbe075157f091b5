"""ctypes binding of libhf (include/hf.h): argument marshalling only.

Every stage runs in the HIP kernels of libhf.so.  There is no CPU fallback:
if the library is missing or no GPU is visible, the calls raise.
PyTorch provides device memory and the stream the kernels are enqueued on.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhf.so")

HF_OK, HF_ERR_ARG, HF_ERR_SIZE, HF_ERR_WORKSPACE = 0, 1, 2, 3
HF_ERR_OVERFLOW, HF_ERR_CAPACITY, HF_ERR_DEVICE, HF_ERR_INPUT = 4, 5, 6, 7
HF_F32, HF_F64 = 0, 1
KERNELS = {"sampled": 0, "analytic": 1, "stencil": 2}
STAGE_DEPOSIT, STAGE_CWT, STAGE_MAXIMA, STAGE_SEGMENT, STAGE_LABEL = 1, 2, 4, 8, 16

EXPORTS = ("hf_create", "hf_destroy", "hf_status_str", "hf_sync", "hf_workspace_size",
           "hf_deposit", "hf_cwt", "hf_maxima", "hf_segment", "hf_label",
           "hf_profile_enable", "hf_profile_reset", "hf_profile_read",
           "hf_cwt_batch_ws_size", "hf_cwt_batch", "hf_find_halos", "hf_find_halos_group", "hf_groups",
           "hf_find_halos_filtered", "hf_cwt_scales",
           "hf_find_halos_scales_ws_size", "hf_find_halos_scales", "hf_cross_scale", "hf_peaks",
           "hf_cwt_stencil", "hf_stencil_half_width", "hf_identify_ws_size", "hf_identify",
           "hf_find_halos_noalloc", "hf_identify_grids_ws_size", "hf_identify_grids", "hf_unbind_ws_size",
           "hf_unbind")
CWT_BATCH_MAX = 32
STAGE_ALL = 31
STAGE_GROUPS = 32
STAGE_STENCIL = 64
STENCIL_MAX_HALF_WIDTH = 64


class HFError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_str(code)} (hf_status {code})")


class Box(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("frac_bits", ctypes.c_int32), ("box_len", ctypes.c_double)]


class CwtItem(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("cwt", ctypes.c_void_p), ("box_len", ctypes.c_double),
                ("kw", ctypes.c_double)]


class Job(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("np", ctypes.c_int64), ("dtype", ctypes.c_int),
                ("kw", ctypes.c_double), ("kernel", ctypes.c_int), ("tau", ctypes.c_float),
                ("rho", ctypes.c_void_p), ("cwt", ctypes.c_void_p), ("max_idx", ctypes.c_void_p),
                ("max_cap", ctypes.c_int64), ("d_count", ctypes.c_void_p), ("cell_label", ctypes.c_void_p),
                ("particle_label", ctypes.c_void_p)]


class ScaleJob(ctypes.Structure):
    _fields_ = [("kw", ctypes.c_double), ("cwt", ctypes.c_void_p), ("max_idx", ctypes.c_void_p),
                ("max_cap", ctypes.c_int64), ("d_count", ctypes.c_void_p), ("cell_label", ctypes.c_void_p),
                ("particle_label", ctypes.c_void_p)]


class IdentifyGroups(ctypes.Structure):
    _fields_ = [("group_particles", ctypes.c_void_p), ("group_cells", ctypes.c_void_p),
                ("group_keep", ctypes.c_void_p)]


class GridScale(ctypes.Structure):
    _fields_ = [("kw", ctypes.c_double), ("n", ctypes.c_int32), ("rho", ctypes.c_void_p), ("cwt", ctypes.c_void_p),
                ("max_idx", ctypes.c_void_p), ("max_cap", ctypes.c_int64), ("d_count", ctypes.c_void_p),
                ("cell_label", ctypes.c_void_p), ("particle_label", ctypes.c_void_p),
                ("group_particles", ctypes.c_void_p), ("group_cells", ctypes.c_void_p),
                ("group_keep", ctypes.c_void_p), ("bound_keep", ctypes.c_void_p)]


class GroupFilter(ctypes.Structure):
    _fields_ = [("dens_th", ctypes.c_double), ("particle_th", ctypes.c_int64), ("group_particles", ctypes.c_void_p),
                ("group_cells", ctypes.c_void_p), ("group_keep", ctypes.c_void_p),
                ("cell_label_kept", ctypes.c_void_p)]


class GroupItem(ctypes.Structure):
    _fields_ = [("job", Job), ("box_len", ctypes.c_double), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhf.so and declare its signatures (no GPU needed to load)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run __graft_entry__.build() "
                               "(python -m paper_2501_10622_amd.build)")
        lib = ctypes.CDLL(path)
        vp, i32, i64, sz, dbl, flt = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                                      ctypes.c_double, ctypes.c_float)
        bp = ctypes.POINTER(Box)
        sig = {
            "hf_create": (ctypes.c_int, [ctypes.c_int, vp, ctypes.POINTER(vp)]),
            "hf_destroy": (ctypes.c_int, [vp]),
            "hf_status_str": (ctypes.c_char_p, [ctypes.c_int]),
            "hf_sync": (ctypes.c_int, [vp]),
            "hf_workspace_size": (ctypes.c_int, [bp, i64, ctypes.c_int, ctypes.POINTER(sz)]),
            "hf_deposit": (ctypes.c_int, [vp, bp, vp, ctypes.c_int, i64, vp, vp, sz]),
            "hf_cwt": (ctypes.c_int, [vp, bp, vp, dbl, ctypes.c_int, vp, vp, sz]),
            "hf_cwt_stencil": (ctypes.c_int, [vp, bp, vp, dbl, i32, vp, vp, sz]),
            "hf_stencil_half_width": (ctypes.c_int, [dbl, i32, ctypes.POINTER(i32)]),
            "hf_maxima": (ctypes.c_int, [vp, bp, vp, flt, vp, i64, vp, vp, sz]),
            "hf_segment": (ctypes.c_int, [vp, bp, vp, flt, vp, vp, sz]),
            "hf_label": (ctypes.c_int, [vp, bp, vp, ctypes.c_int, i64, vp, vp]),
            "hf_profile_enable": (ctypes.c_int, [vp, ctypes.c_int]),
            "hf_profile_reset": (ctypes.c_int, [vp]),
            "hf_profile_read": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
            "hf_cwt_batch_ws_size": (ctypes.c_int, [i32, i32, ctypes.POINTER(sz)]),
            "hf_cwt_batch": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(CwtItem), ctypes.c_int, vp, sz]),
            "hf_cwt_scales": (ctypes.c_int, [vp, bp, vp, i32, ctypes.POINTER(dbl), ctypes.c_int,
                                             ctypes.POINTER(vp), vp, sz]),
            "hf_find_halos_scales_ws_size": (ctypes.c_int, [bp, i64, i32, ctypes.POINTER(sz)]),
            "hf_find_halos_scales": (ctypes.c_int, [vp, bp, vp, ctypes.c_int, i64, ctypes.c_int, flt, vp, i32,
                                                    ctypes.POINTER(ScaleJob), vp, sz]),
            "hf_find_halos": (ctypes.c_int, [vp, bp, ctypes.POINTER(Job), vp, sz]),
            "hf_find_halos_noalloc": (ctypes.c_int, [vp, bp, ctypes.POINTER(Job)]),
            "hf_identify_grids_ws_size": (ctypes.c_int, [dbl, i32, i64, i32, ctypes.POINTER(GridScale), i32,
                                                         ctypes.POINTER(sz)]),
            "hf_identify_grids": (ctypes.c_int, [vp, dbl, i32, vp, vp, i32, i64, flt, i32, ctypes.POINTER(GridScale),
                                                 dbl, i64, dbl, vp, vp, vp, sz]),
            "hf_unbind_ws_size": (ctypes.c_int, [bp, i64, i64, ctypes.POINTER(sz)]),
            "hf_unbind": (ctypes.c_int, [vp, bp, vp, vp, i32, i64, vp, i64, vp, vp, dbl, i64, vp, vp, sz]),
            "hf_identify_ws_size": (ctypes.c_int, [bp, i64, i32, ctypes.POINTER(ScaleJob), ctypes.POINTER(sz)]),
            "hf_identify": (ctypes.c_int, [vp, bp, vp, ctypes.c_int, i64, ctypes.c_int, flt, vp, i32,
                                           ctypes.POINTER(ScaleJob), ctypes.POINTER(IdentifyGroups), dbl, i64, vp,
                                           vp, vp, sz]),
            "hf_find_halos_group": (ctypes.c_int, [vp, i32, i32, i32, ctypes.POINTER(GroupItem), ctypes.c_int,
                                                   vp, sz]),
            "hf_groups": (ctypes.c_int, [vp, bp, i64, vp, i64, vp, vp, dbl, i64, vp, vp, vp, vp, vp, vp, vp, sz]),
            "hf_cross_scale": (ctypes.c_int, [vp, bp, vp, i64, vp, i32, vp, vp]),
            "hf_peaks": (ctypes.c_int, [vp, bp, vp, vp, i64, vp, vp]),
            "hf_find_halos_filtered": (ctypes.c_int, [vp, bp, ctypes.POINTER(Job), ctypes.POINTER(GroupFilter), vp,
                                                      sz]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def status_str(code: int) -> str:
    try:
        return load_library().hf_status_str(int(code)).decode()
    except RuntimeError:
        return f"status {code}"


def _check(code: int, where: str):
    if code != HF_OK:
        raise HFError(code, where)


# ---------------------------------------------------------------------------
# contexts and workspaces
# ---------------------------------------------------------------------------
class Context:
    """An hf_ctx bound to one device and one HIP stream."""

    def __init__(self, device: int, stream: torch.cuda.Stream):
        lib = load_library()
        self.device = int(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.hf_create(self.device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), "hf_create")
        self.handle = h

    def sync(self):
        _check(load_library().hf_sync(self.handle), "hf_sync")

    def profile(self, enable: bool = True):
        """Turn the library's per-kernel event timer on or off."""
        _check(load_library().hf_profile_enable(self.handle, int(bool(enable))), "hf_profile_enable")

    def profile_reset(self):
        _check(load_library().hf_profile_reset(self.handle), "hf_profile_reset")

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} accumulated since the last reset."""
        lib = load_library()
        out = {}
        i = 0
        while True:
            name, ms, cnt = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_int64()
            code = lib.hf_profile_read(self.handle, i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt))
            if code == HF_ERR_ARG:
                break
            _check(code, "hf_profile_read")
            out[name.value.decode()] = (ms.value, cnt.value)
            i += 1
        return out

    def close(self):
        if self.handle:
            load_library().hf_destroy(self.handle)
            self.handle = None


_ctxs: dict = {}
_ws: dict = {}


def _require_cuda(t: torch.Tensor, name: str):
    if not torch.cuda.is_available():
        raise RuntimeError("libhf needs a ROCm GPU; none is visible")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def context(device=None, stream=None) -> Context:
    dev = torch.cuda.current_device() if device is None else torch.device("cuda", device).index
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    key = (dev, st.cuda_stream)
    ctx = _ctxs.get(key)
    if ctx is None:
        with torch.cuda.device(dev):
            ctx = Context(dev, st)
        _ctxs[key] = ctx
    return ctx


def workspace(nbytes: int, ctx: Context) -> torch.Tensor:
    """A reusable device workspace of at least nbytes, one per (device, stream).

    It is allocated on the context's own stream, the only stream its kernels
    run on, so when a larger one replaces it the caching allocator cannot hand
    the old memory to work still queued on another stream; two contexts on
    different streams never share one."""
    key = (ctx.device, ctx.stream.cuda_stream)
    cur = _ws.get(key)
    if cur is None or cur.numel() < nbytes:
        with torch.cuda.stream(ctx.stream):
            cur = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=torch.device("cuda", ctx.device))
        _ws[key] = cur
    return cur


def box(n: int, box_len: float, frac_bits: int = 15) -> Box:
    return Box(int(n), int(frac_bits), float(box_len))


def workspace_size(n: int, box_len: float, np_: int, stages: int, frac_bits: int = 15) -> int:
    out = ctypes.c_size_t()
    b = box(n, box_len, frac_bits)
    _check(load_library().hf_workspace_size(ctypes.byref(b), int(np_), int(stages), ctypes.byref(out)),
           "hf_workspace_size")
    return out.value


def _dtype_code(pos: torch.Tensor) -> int:
    if pos.dtype == torch.float32:
        return HF_F32
    if pos.dtype == torch.float64:
        return HF_F64
    raise ValueError("positions must be float32 or float64")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


# ---------------------------------------------------------------------------
# stages
# ---------------------------------------------------------------------------
def deposit(pos: torch.Tensor, box_len: float, n: int, frac_bits: int = 15, out=None, ctx=None) -> torch.Tensor:
    """Step 2: CIC deposit -> int64 grid [n, n, n] (units of 2^-3B particle)."""
    _require_cuda(pos, "pos")
    if pos.ndim != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be [np, 3]")
    ctx = ctx or context(pos.device.index)
    if out is None:
        out = torch.empty((n, n, n), dtype=torch.int64, device=pos.device)
    b = box(n, box_len, frac_bits)
    need = workspace_size(n, box_len, pos.shape[0], STAGE_DEPOSIT, frac_bits)
    ws = workspace(need, ctx) if need else None
    _check(load_library().hf_deposit(ctx.handle, ctypes.byref(b), _ptr(pos), _dtype_code(pos), pos.shape[0],
                                     _ptr(out), _ptr(ws), need), "hf_deposit")
    return out


def cwt(rho: torch.Tensor, box_len: float, kw: float, kernel: str = "sampled", out=None, ctx=None,
        frac_bits: int = 15) -> torch.Tensor:
    """Step 3: grid CWT (FP32) of an int64 CIC grid at scale k_w."""
    _require_cuda(rho, "rho")
    if rho.dtype != torch.int64 or rho.ndim != 3:
        raise ValueError("rho must be an int64 [n, n, n] grid")
    n = rho.shape[0]
    ctx = ctx or context(rho.device.index)
    if out is None:
        out = torch.empty((n, n, n), dtype=torch.float32, device=rho.device)
    b = box(n, box_len, frac_bits)
    need = workspace_size(n, box_len, 0, STAGE_STENCIL if kernel == "stencil" else STAGE_CWT, frac_bits)
    ws = workspace(need, ctx)
    _check(load_library().hf_cwt(ctx.handle, ctypes.byref(b), _ptr(rho), float(kw), KERNELS[kernel], _ptr(out),
                                 _ptr(ws), need), "hf_cwt")
    return out


def stencil_half_width(kw: float, n: int) -> int:
    """The library's default stencil half-width on an n^3 grid (hf_stencil_half_width:
    Table 1's count Int(1.5/k_w + 5) kept at its extent on the grid N_g = Int(400 k_w + 150))."""
    h = ctypes.c_int32()
    _check(load_library().hf_stencil_half_width(float(kw), int(n), ctypes.byref(h)), "hf_stencil_half_width")
    return int(h.value)


def cwt_stencil(rho: torch.Tensor, box_len: float, kw: float, half_width: int | None = None, out=None, ctx=None,
                frac_bits: int = 15, ws=None) -> torch.Tensor:
    """Step 3 by the truncated real-space stencil of Sec. 2.1 (FP32), half-width
    stencil_half_width(kw, n) unless given.  Enqueued on the context's stream."""
    _require_cuda(rho, "rho")
    if rho.dtype != torch.int64 or rho.ndim != 3:
        raise ValueError("rho must be an int64 [n, n, n] grid")
    n = rho.shape[0]
    h = stencil_half_width(kw, n) if half_width is None else int(half_width)
    ctx = ctx or context(rho.device.index)
    if out is None:
        out = torch.empty((n, n, n), dtype=torch.float32, device=rho.device)
    b = box(n, box_len, frac_bits)
    need = workspace_size(n, box_len, 0, STAGE_STENCIL, frac_bits)
    if ws is None:
        ws = workspace(need, ctx)
    elif ws.numel() * ws.element_size() < need:
        raise ValueError("workspace too small for hf_cwt_stencil")
    _check(load_library().hf_cwt_stencil(ctx.handle, ctypes.byref(b), _ptr(rho), float(kw), h, _ptr(out), _ptr(ws),
                                         ws.numel() * ws.element_size()), "hf_cwt_stencil")
    return out


def maxima(c: torch.Tensor, tau: float = 0.0, capacity: int | None = None, ctx=None, sync: bool = True):
    """Step 4: sorted int32 linear indices of the local maxima above tau.

    With sync=True the list is trimmed to the count (one stream sync);
    otherwise (buffer, device_count) is returned."""
    _require_cuda(c, "cwt")
    if c.dtype != torch.float32 or c.ndim != 3:
        raise ValueError("cwt must be a float32 [n, n, n] grid")
    n = c.shape[0]
    ctx = ctx or context(c.device.index)
    if capacity is None:
        capacity = ((n + 1) // 2) ** 3  # two maxima are never neighbours
    buf = torch.empty(max(int(capacity), 1), dtype=torch.int32, device=c.device)
    cnt = torch.empty(1, dtype=torch.int64, device=c.device)
    b = box(n, 1.0)
    need = workspace_size(n, 1.0, 0, STAGE_MAXIMA)
    ws = workspace(need, ctx)
    _check(load_library().hf_maxima(ctx.handle, ctypes.byref(b), _ptr(c), float(tau), _ptr(buf), int(capacity),
                                    _ptr(cnt), _ptr(ws), need), "hf_maxima")
    if not sync:
        return buf, cnt
    ctx.sync()
    return buf[: int(cnt.item())]


def segment(c: torch.Tensor, tau: float = 0.0, out=None, ctx=None) -> torch.Tensor:
    """Step 5: int32 cell labels (root index or -1)."""
    _require_cuda(c, "cwt")
    if c.dtype != torch.float32 or c.ndim != 3:
        raise ValueError("cwt must be a float32 [n, n, n] grid")
    n = c.shape[0]
    ctx = ctx or context(c.device.index)
    if out is None:
        out = torch.empty((n, n, n), dtype=torch.int32, device=c.device)
    b = box(n, 1.0)
    need = workspace_size(n, 1.0, 0, STAGE_SEGMENT)
    ws = workspace(need, ctx)
    _check(load_library().hf_segment(ctx.handle, ctypes.byref(b), _ptr(c), float(tau), _ptr(out), _ptr(ws), need),
           "hf_segment")
    return out


def label(pos: torch.Tensor, box_len: float, n: int, cell_label: torch.Tensor, frac_bits: int = 15, out=None,
          ctx=None) -> torch.Tensor:
    """Step 6: int32 particle labels from the nearest node's cell label."""
    _require_cuda(pos, "pos")
    _require_cuda(cell_label, "cell_label")
    if cell_label.dtype != torch.int32 or cell_label.numel() != n ** 3:
        raise ValueError("cell_label must be int32 with n^3 cells")
    ctx = ctx or context(pos.device.index)
    if out is None:
        out = torch.empty(pos.shape[0], dtype=torch.int32, device=pos.device)
    b = box(n, box_len, frac_bits)
    _check(load_library().hf_label(ctx.handle, ctypes.byref(b), _ptr(pos), _dtype_code(pos), pos.shape[0],
                                   _ptr(cell_label), _ptr(out)), "hf_label")
    return out


def peaks(c: torch.Tensor, roots: torch.Tensor, box_len: float, ctx=None):
    """Step 4's correction of the maxima roots of c (App. B): FP64 positions
    [k, 3] (x, y, z) in box units and corrected values [k]."""
    _require_cuda(c, "cwt")
    if c.dtype != torch.float32 or c.ndim != 3:
        raise ValueError("cwt must be a float32 [n, n, n] grid")
    if roots.dtype != torch.int32:
        raise ValueError("roots must be int32")
    n = c.shape[0]
    ctx = ctx or context(c.device.index)
    k = roots.numel()
    pos = torch.empty((max(k, 1), 3), dtype=torch.float64, device=c.device)[:k]
    val = torch.empty(max(k, 1), dtype=torch.float64, device=c.device)[:k]
    b = box(n, box_len)
    _check(load_library().hf_peaks(ctx.handle, ctypes.byref(b), _ptr(c), _ptr(roots), k, _ptr(pos), _ptr(val)),
           "hf_peaks")
    return pos, val


def cross_scale(c_scale: torch.Tensor, c_smaller: torch.Tensor, roots: torch.Tensor, ctx=None) -> torch.Tensor:
    """Step 8: uint8 flags, 1 where the maximum roots[i] of c_scale, corrected
    for the grid (step 4, App. B), exceeds c_smaller (the adjacent smaller
    scale over the same box, on a grid of its own size) near its corrected
    position."""
    _require_cuda(c_scale, "cwt")
    if c_scale.dtype != torch.float32 or c_smaller.dtype != torch.float32:
        raise ValueError("both fields must be float32")
    for c in (c_scale, c_smaller):
        if c.dim() != 3 or not (c.shape[0] == c.shape[1] == c.shape[2]) or not c.is_contiguous():
            raise ValueError("fields must be contiguous [n, n, n]")
    if roots.dtype != torch.int32:
        raise ValueError("roots must be int32")
    n = c_scale.shape[0]
    ctx = ctx or context(c_scale.device.index)
    out = torch.empty(max(roots.numel(), 1), dtype=torch.uint8, device=c_scale.device)[: roots.numel()]
    b = box(n, 1.0)
    _check(load_library().hf_cross_scale(ctx.handle, ctypes.byref(b), _ptr(roots), roots.numel(), _ptr(c_scale),
                                         c_smaller.shape[0], _ptr(c_smaller), _ptr(out)), "hf_cross_scale")
    return out


def groups(cell_label: torch.Tensor, particle_label: torch.Tensor, roots: torch.Tensor, n_particles: int,
           dens_th: float = 4.0, particle_th: int = 15, filter_cells: bool = True, filter_particles: bool = True,
           ctx=None, root_ok: torch.Tensor | None = None) -> dict:
    """Steps 5 and 7 (Table 1's dens_th, particle_th): per-group cell and
    particle numbers and keep flags for the sorted maxima list ``roots``, and
    the labels with disposed groups set to -1 (new tensors).  The counts are
    the library's uint32 values held in int32 tensors (below 2^31 for any box
    of fewer than 2^31 particles)."""
    _require_cuda(cell_label, "cell_label")
    if cell_label.dtype != torch.int32 or cell_label.ndim != 3:
        raise ValueError("cell_label must be an int32 [n, n, n] grid")
    if particle_label.dtype != torch.int32 or roots.dtype != torch.int32:
        raise ValueError("particle_label and roots must be int32")
    n = cell_label.shape[0]
    dev = cell_label.device
    ctx = ctx or context(dev.index)
    nroots = roots.numel()
    out = {
        "particles": torch.empty(max(nroots, 1), dtype=torch.int32, device=dev)[:nroots],
        "cells": torch.empty(max(nroots, 1), dtype=torch.int32, device=dev)[:nroots],
        "keep": torch.empty(max(nroots, 1), dtype=torch.uint8, device=dev)[:nroots],
        "cell_label": torch.empty_like(cell_label) if filter_cells else None,
        "particle_label": torch.empty_like(particle_label) if filter_particles else None,
    }
    b = box(n, 1.0)
    need = workspace_size(n, 1.0, int(particle_label.numel()), STAGE_GROUPS)  # with the partitioned count's room
    ws = workspace(need, ctx)
    if root_ok is not None and (root_ok.dtype != torch.uint8 or root_ok.numel() != nroots):
        raise ValueError("root_ok must be uint8 with one flag per root")
    _check(load_library().hf_groups(ctx.handle, ctypes.byref(b), int(n_particles), _ptr(roots), int(nroots),
                                    _ptr(cell_label), _ptr(particle_label), float(dens_th), int(particle_th),
                                    _ptr(root_ok), _ptr(out["particles"]), _ptr(out["cells"]), _ptr(out["keep"]),
                                    _ptr(out["cell_label"]), _ptr(out["particle_label"]), _ptr(ws), need),
           "hf_groups")
    return out


def sync(device=None):
    """Wait for the current stream and raise on a device-detected error."""
    context(device).sync()


def cwt_batch(rhos, box_lens, kws, kernel: str = "sampled", outs=None, ws=None, ctx=None) -> list:
    """Step 3 for several same-n grids in one launch per FFT pass (at most CWT_BATCH_MAX)."""
    count = len(rhos)
    if count < 1 or count > CWT_BATCH_MAX:
        raise ValueError(f"batch size must be 1..{CWT_BATCH_MAX}")
    n = rhos[0].shape[0]
    for r in rhos:
        _require_cuda(r, "rho")
        if r.dtype != torch.int64 or r.shape != (n, n, n):
            raise ValueError("all grids must be int64 [n, n, n] of the same n")
    ctx = ctx or context(rhos[0].device.index)
    if outs is None:
        outs = [torch.empty((n, n, n), dtype=torch.float32, device=r.device) for r in rhos]
    need = ctypes.c_size_t()
    lib = load_library()
    _check(lib.hf_cwt_batch_ws_size(n, count, ctypes.byref(need)), "hf_cwt_batch_ws_size")
    if ws is None:
        ws = torch.empty(need.value, dtype=torch.uint8, device=rhos[0].device)
    items = (CwtItem * count)(*[CwtItem(r.data_ptr(), o.data_ptr(), float(L), float(k))
                                 for r, o, L, k in zip(rhos, outs, box_lens, kws)])
    _check(lib.hf_cwt_batch(ctx.handle, n, count, items, KERNELS[kernel], _ptr(ws), ws.numel()), "hf_cwt_batch")
    return outs


def cwt_scales(rho: torch.Tensor, box_len: float, kws, kernel: str = "sampled", outs=None, ws=None, ctx=None,
               frac_bits: int = 15) -> list:
    """Step 3 of one int64 grid at several scales (at most CWT_BATCH_MAX): one
    forward transform, then a multiplier and inverse transform per scale."""
    _require_cuda(rho, "rho")
    if rho.dtype != torch.int64 or rho.ndim != 3:
        raise ValueError("rho must be an int64 [n, n, n] grid")
    count = len(kws)
    if count < 1 or count > CWT_BATCH_MAX:
        raise ValueError(f"number of scales must be 1..{CWT_BATCH_MAX}")
    n = rho.shape[0]
    ctx = ctx or context(rho.device.index)
    if outs is None:
        outs = [torch.empty((n, n, n), dtype=torch.float32, device=rho.device) for _ in range(count)]
    need = cwt_batch_ws_bytes(n, count)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=rho.device)
    b = box(n, box_len, frac_bits)
    k = (ctypes.c_double * count)(*[float(x) for x in kws])
    o = (ctypes.c_void_p * count)(*[t.data_ptr() for t in outs])
    _check(load_library().hf_cwt_scales(ctx.handle, ctypes.byref(b), _ptr(rho), count, k, KERNELS[kernel], o,
                                        _ptr(ws), ws.numel()), "hf_cwt_scales")
    return outs


def job_buffers(n: int, np_: int, device, with_cwt_ws: bool = True, frac_bits: int = 15,
                with_groups: bool = False, with_stencil: bool = False) -> dict:
    """Output and workspace tensors for one box (allocated on the current stream);
    with_groups adds the group outputs and workspace of find_halos_filtered_async,
    with_stencil the workspace of the "stencil" transform."""
    stages = STAGE_ALL if with_cwt_ws else (STAGE_DEPOSIT | STAGE_MAXIMA | STAGE_SEGMENT)
    if with_groups:
        stages |= STAGE_GROUPS
    if with_stencil:  # the stencil transform's workspace instead of the FFT's (any n)
        stages = (stages & ~STAGE_CWT) | STAGE_STENCIL
    need = workspace_size(n, 1.0, np_, stages, frac_bits)
    cap = ((n + 1) // 2) ** 3
    extra = {}
    if with_groups:
        extra = {
            "group_particles": torch.empty(cap, dtype=torch.int32, device=device),
            "group_cells": torch.empty(cap, dtype=torch.int32, device=device),
            "group_keep": torch.empty(cap, dtype=torch.uint8, device=device),
            "cell_label_kept": torch.empty((n, n, n), dtype=torch.int32, device=device),
        }
    return extra | {
        "rho": torch.empty((n, n, n), dtype=torch.int64, device=device),
        "cwt": torch.empty((n, n, n), dtype=torch.float32, device=device),
        "maxima": torch.empty(cap, dtype=torch.int32, device=device),
        "count": torch.empty(1, dtype=torch.int64, device=device),
        "cell_label": torch.empty((n, n, n), dtype=torch.int32, device=device),
        "particle_label": torch.empty(max(np_, 1), dtype=torch.int32, device=device),
        "ws": torch.empty(max(need, 256), dtype=torch.uint8, device=device),
    }


def find_halos_async(pos: torch.Tensor, box_len: float, n: int, kw: float, bufs: dict, frac_bits: int = 15,
                     tau: float = 0.0, kernel: str = "sampled", ctx=None):
    """Enqueue steps 2-6 with the native single-call driver (no synchronisation)."""
    _require_cuda(pos, "pos")
    ctx = ctx or context(pos.device.index)
    b = box(n, box_len, frac_bits)
    job = _job_struct(pos, kw, bufs, tau, kernel)
    _check(load_library().hf_find_halos(ctx.handle, ctypes.byref(b), ctypes.byref(job), _ptr(bufs["ws"]),
                                        bufs["ws"].numel()), "hf_find_halos")


NOALLOC_SCRATCH_BYTES = 64 << 20


def find_halos_noalloc_async(pos: torch.Tensor, box_len: float, n: int, kw: float, bufs: dict, frac_bits: int = 15,
                             tau: float = 0.0, kernel: str = "sampled", ctx=None):
    """Enqueue steps 2-6 through hf_find_halos_noalloc: outputs in bufs (as from
    job_buffers; its "ws" entry is not used), the workspace the library's own
    per-device scratch array.  Calls that overlap on one device race."""
    _require_cuda(pos, "pos")
    ctx = ctx or context(pos.device.index)
    b = box(n, box_len, frac_bits)
    job = _job_struct(pos, kw, bufs, tau, kernel)
    _check(load_library().hf_find_halos_noalloc(ctx.handle, ctypes.byref(b), ctypes.byref(job)),
           "hf_find_halos_noalloc")


def scales_buffers(n: int, np_: int, count: int, device, frac_bits: int = 15) -> dict:
    """Outputs (one list entry per scale) and workspace for find_halos_scales_async."""
    out = ctypes.c_size_t()
    b = box(n, 1.0, frac_bits)
    _check(load_library().hf_find_halos_scales_ws_size(ctypes.byref(b), int(np_), int(count), ctypes.byref(out)),
           "hf_find_halos_scales_ws_size")
    cap = ((n + 1) // 2) ** 3
    return {
        "rho": torch.empty((n, n, n), dtype=torch.int64, device=device),
        "cwt": [torch.empty((n, n, n), dtype=torch.float32, device=device) for _ in range(count)],
        "maxima": [torch.empty(cap, dtype=torch.int32, device=device) for _ in range(count)],
        "count": [torch.empty(1, dtype=torch.int64, device=device) for _ in range(count)],
        "cell_label": [torch.empty((n, n, n), dtype=torch.int32, device=device) for _ in range(count)],
        "particle_label": [torch.empty(max(np_, 1), dtype=torch.int32, device=device) for _ in range(count)],
        "ws": torch.empty(max(out.value, 256), dtype=torch.uint8, device=device),
    }


def find_halos_scales_async(pos: torch.Tensor, box_len: float, n: int, kws, bufs: dict, frac_bits: int = 15,
                            tau: float = 0.0, kernel: str = "sampled", ctx=None):
    """Enqueue steps 2-6 at several scales of one box: one deposit and one
    forward transform, then per scale the rest (bufs from scales_buffers)."""
    _require_cuda(pos, "pos")
    ctx = ctx or context(pos.device.index)
    count = len(kws)
    if count != len(bufs["cwt"]):
        raise ValueError("one buffer set per scale")
    jobs = (ScaleJob * count)(*[ScaleJob(float(kw), bufs["cwt"][j].data_ptr(), bufs["maxima"][j].data_ptr(),
                                         bufs["maxima"][j].numel(), bufs["count"][j].data_ptr(),
                                         bufs["cell_label"][j].data_ptr(), bufs["particle_label"][j].data_ptr())
                                for j, kw in enumerate(kws)])
    b = box(n, box_len, frac_bits)
    _check(load_library().hf_find_halos_scales(ctx.handle, ctypes.byref(b), _ptr(pos), _dtype_code(pos),
                                               pos.shape[0], KERNELS[kernel], float(tau), _ptr(bufs["rho"]), count,
                                               jobs, _ptr(bufs["ws"]), bufs["ws"].numel()), "hf_find_halos_scales")


def _scale_jobs(kws, bufs):
    return (ScaleJob * len(kws))(*[ScaleJob(float(kw), bufs["cwt"][j].data_ptr(), bufs["maxima"][j].data_ptr(),
                                            bufs["maxima"][j].numel(), bufs["count"][j].data_ptr(),
                                            bufs["cell_label"][j].data_ptr(), bufs["particle_label"][j].data_ptr())
                                   for j, kw in enumerate(kws)])


def identify_buffers(n: int, np_: int, count: int, device, frac_bits: int = 15) -> dict:
    """Outputs and workspace for identify_async: those of scales_buffers, the
    per-maximum group outputs of every scale and the per-particle halo_scale
    and halo_root."""
    bufs = scales_buffers(n, np_, count, device, frac_bits)
    cap = bufs["maxima"][0].numel()
    bufs["group_particles"] = [torch.empty(cap, dtype=torch.int32, device=device) for _ in range(count)]
    bufs["group_cells"] = [torch.empty(cap, dtype=torch.int32, device=device) for _ in range(count)]
    bufs["group_keep"] = [torch.empty(cap, dtype=torch.uint8, device=device) for _ in range(count)]
    bufs["halo_scale"] = torch.empty(max(np_, 1), dtype=torch.int32, device=device)
    bufs["halo_root"] = torch.empty(max(np_, 1), dtype=torch.int32, device=device)
    out = ctypes.c_size_t()
    b = box(n, 1.0, frac_bits)
    jobs = _scale_jobs([1.0 + j for j in range(count)], bufs)
    _check(load_library().hf_identify_ws_size(ctypes.byref(b), int(np_), int(count), jobs, ctypes.byref(out)),
           "hf_identify_ws_size")
    bufs["ws"] = torch.empty(max(out.value, 256), dtype=torch.uint8, device=device)
    return bufs


def identify_async(pos: torch.Tensor, box_len: float, n: int, kws, bufs: dict, dens_th: float = 4.0,
                   particle_th: int = 15, frac_bits: int = 15, tau: float = 0.0, kernel: str = "sampled", ctx=None):
    """Enqueue Sec. 2's identification loop over the scales kws (increasing k_w),
    steps 2-8 without unbinding (bufs from identify_buffers)."""
    _require_cuda(pos, "pos")
    ctx = ctx or context(pos.device.index)
    count = len(kws)
    if count != len(bufs["cwt"]):
        raise ValueError("one buffer set per scale")
    jobs = _scale_jobs(kws, bufs)
    groups = (IdentifyGroups * count)(*[IdentifyGroups(bufs["group_particles"][j].data_ptr(),
                                                       bufs["group_cells"][j].data_ptr(),
                                                       bufs["group_keep"][j].data_ptr()) for j in range(count)])
    b = box(n, box_len, frac_bits)
    _check(load_library().hf_identify(ctx.handle, ctypes.byref(b), _ptr(pos), _dtype_code(pos), pos.shape[0],
                                      KERNELS[kernel], float(tau), _ptr(bufs["rho"]), count, jobs, groups,
                                      float(dens_th), int(particle_th), _ptr(bufs["halo_scale"]),
                                      _ptr(bufs["halo_root"]), _ptr(bufs["ws"]), bufs["ws"].numel()), "hf_identify")


def paper_grid(kw: float) -> int:
    """The flowchart's grid size for a scale, N_g = Int(400 k_w + 150)."""
    return int(400.0 * kw + 150.0)


def _grid_scales(kws, bufs):
    return (GridScale * len(kws))(*[GridScale(float(kw), int(bufs["grids"][j]), bufs["rho"][j].data_ptr(),
                                              bufs["cwt"][j].data_ptr(), bufs["maxima"][j].data_ptr(),
                                              bufs["maxima"][j].numel(), bufs["count"][j].data_ptr(),
                                              bufs["cell_label"][j].data_ptr(), bufs["particle_label"][j].data_ptr(),
                                              bufs["group_particles"][j].data_ptr(),
                                              bufs["group_cells"][j].data_ptr(), bufs["group_keep"][j].data_ptr(),
                                              bufs["bound_keep"][j].data_ptr())
                                    for j, kw in enumerate(kws)])


def identify_grids_buffers(grids, np_: int, device, box_len: float = 1.0, frac_bits: int = 15,
                           with_velocities: bool = False) -> dict:
    """Outputs (one entry per scale, each on its own grid size in ``grids``) and
    workspace for identify_grids_async (with_velocities: room for steps 9-10)."""
    count = len(grids)
    caps = [((g + 1) // 2) ** 3 for g in grids]
    bufs = {
        "grids": [int(g) for g in grids],
        "rho": [torch.empty((g, g, g), dtype=torch.int64, device=device) for g in grids],
        "cwt": [torch.empty((g, g, g), dtype=torch.float32, device=device) for g in grids],
        "maxima": [torch.empty(c, dtype=torch.int32, device=device) for c in caps],
        "count": [torch.empty(1, dtype=torch.int64, device=device) for _ in grids],
        "cell_label": [torch.empty((g, g, g), dtype=torch.int32, device=device) for g in grids],
        "particle_label": [torch.empty(max(np_, 1), dtype=torch.int32, device=device) for _ in grids],
        "group_particles": [torch.empty(c, dtype=torch.int32, device=device) for c in caps],
        "group_cells": [torch.empty(c, dtype=torch.int32, device=device) for c in caps],
        "group_keep": [torch.empty(c, dtype=torch.uint8, device=device) for c in caps],
        "bound_keep": [torch.empty(c, dtype=torch.uint8, device=device) for c in caps],
        "halo_scale": torch.empty(max(np_, 1), dtype=torch.int32, device=device),
        "halo_root": torch.empty(max(np_, 1), dtype=torch.int32, device=device),
    }
    out = ctypes.c_size_t()
    jobs = _grid_scales([0.1 * (j + 1) for j in range(count)], bufs)
    _check(load_library().hf_identify_grids_ws_size(float(box_len), int(frac_bits), int(np_), count, jobs,
                                                    int(bool(with_velocities)), ctypes.byref(out)),
           "hf_identify_grids_ws_size")
    bufs["ws"] = torch.empty(max(out.value, 256), dtype=torch.uint8, device=device)
    return bufs


def identify_grids_async(pos: torch.Tensor, box_len: float, kws, bufs: dict, dens_th: float = 4.0,
                         particle_th: int = 15, frac_bits: int = 15, tau: float = 0.0, vel=None,
                         grav_mass: float = 0.0, ctx=None):
    """Enqueue Sec. 2's identification loop with every scale on its own grid
    (bufs from identify_grids_buffers, e.g. with grids [paper_grid(kw) ...]);
    with velocities vel [np, 3] (km/s) and grav_mass = G m_p, steps 9-10 too."""
    _require_cuda(pos, "pos")
    if vel is not None:
        _require_cuda(vel, "vel")
        if vel.dtype != pos.dtype or vel.shape != pos.shape:
            raise ValueError("vel must match pos in dtype and shape")
    ctx = ctx or context(pos.device.index)
    count = len(kws)
    if count != len(bufs["grids"]):
        raise ValueError("one grid per scale")
    jobs = _grid_scales(kws, bufs)
    _check(load_library().hf_identify_grids(ctx.handle, float(box_len), int(frac_bits), _ptr(pos), _ptr(vel),
                                            _dtype_code(pos), pos.shape[0], float(tau), count, jobs, float(dens_th),
                                            int(particle_th), float(grav_mass), _ptr(bufs["halo_scale"]),
                                            _ptr(bufs["halo_root"]), _ptr(bufs["ws"]), bufs["ws"].numel()),
           "hf_identify_grids")


def unbind(pos: torch.Tensor, vel: torch.Tensor, box_len: float, n: int, roots: torch.Tensor,
           group_keep: torch.Tensor, particle_label: torch.Tensor, grav_mass: float, particle_th: int = 15,
           frac_bits: int = 15, ctx=None) -> torch.Tensor:
    """Steps 9-10 on one scale's groups (hf_unbind): particle_label is changed in
    place to the bound particles' labels; returns the uint8 bound_keep flags."""
    _require_cuda(pos, "pos")
    _require_cuda(vel, "vel")
    if vel.dtype != pos.dtype or vel.shape != pos.shape:
        raise ValueError("vel must match pos in dtype and shape")
    if roots.dtype != torch.int32 or particle_label.dtype != torch.int32 or group_keep.dtype != torch.uint8:
        raise ValueError("roots and particle_label must be int32, group_keep uint8")
    ctx = ctx or context(pos.device.index)
    b = box(n, box_len, frac_bits)
    out = ctypes.c_size_t()
    _check(load_library().hf_unbind_ws_size(ctypes.byref(b), pos.shape[0], roots.numel(), ctypes.byref(out)),
           "hf_unbind_ws_size")
    ws = workspace(out.value, ctx)
    bound = torch.empty(max(roots.numel(), 1), dtype=torch.uint8, device=pos.device)[: roots.numel()]
    _check(load_library().hf_unbind(ctx.handle, ctypes.byref(b), _ptr(pos), _ptr(vel), _dtype_code(pos),
                                    pos.shape[0], _ptr(roots), roots.numel(), _ptr(group_keep),
                                    _ptr(particle_label), float(grav_mass), int(particle_th), _ptr(bound),
                                    _ptr(ws), out.value), "hf_unbind")
    return bound


def find_halos_filtered_async(pos: torch.Tensor, box_len: float, n: int, kw: float, bufs: dict,
                              dens_th: float = 4.0, particle_th: int = 15, frac_bits: int = 15, tau: float = 0.0,
                              kernel: str = "sampled", ctx=None):
    """Enqueue steps 2-6 and the group statistics and filters of steps 5 and 7
    (bufs from job_buffers(..., with_groups=True)); bufs["particle_label"]
    receives the labels after the filter, bufs["cell_label"] the segmentation
    and bufs["cell_label_kept"] the filtered cell labels."""
    _require_cuda(pos, "pos")
    ctx = ctx or context(pos.device.index)
    b = box(n, box_len, frac_bits)
    job = _job_struct(pos, kw, bufs, tau, kernel)
    gf = GroupFilter(float(dens_th), int(particle_th), bufs["group_particles"].data_ptr(),
                     bufs["group_cells"].data_ptr(), bufs["group_keep"].data_ptr(),
                     bufs["cell_label_kept"].data_ptr())
    _check(load_library().hf_find_halos_filtered(ctx.handle, ctypes.byref(b), ctypes.byref(job), ctypes.byref(gf),
                                                 _ptr(bufs["ws"]), bufs["ws"].numel()), "hf_find_halos_filtered")


def cwt_batch_ws_bytes(n: int, count: int) -> int:
    out = ctypes.c_size_t()
    _check(load_library().hf_cwt_batch_ws_size(int(n), int(count), ctypes.byref(out)), "hf_cwt_batch_ws_size")
    return out.value


def _job_struct(pos, kw, bufs, tau, kernel):
    return Job(pos.data_ptr(), pos.shape[0], _dtype_code(pos), float(kw), KERNELS[kernel], float(tau),
               bufs["rho"].data_ptr(), bufs["cwt"].data_ptr(), bufs["maxima"].data_ptr(), bufs["maxima"].numel(),
               bufs["count"].data_ptr(), bufs["cell_label"].data_ptr(), bufs["particle_label"].data_ptr())


def find_halos_group_async(n: int, entries, cwt_ws: torch.Tensor, frac_bits: int = 15, tau: float = 0.0,
                           kernel: str = "sampled", ctx=None):
    """Enqueue steps 2-6 for same-n boxes with one batched transform.

    entries: list of (pos, box_len, kw, bufs) with bufs from job_buffers(..., with_cwt_ws=False)."""
    count = len(entries)
    if count < 1 or count > CWT_BATCH_MAX:
        raise ValueError(f"group size must be 1..{CWT_BATCH_MAX}")
    ctx = ctx or context(entries[0][0].device.index)
    items = (GroupItem * count)(*[
        GroupItem(_job_struct(pos, kw, bufs, tau, kernel), float(L), bufs["ws"].data_ptr(), bufs["ws"].numel())
        for pos, L, kw, bufs in entries])
    _check(load_library().hf_find_halos_group(ctx.handle, int(n), int(frac_bits), count, items, KERNELS[kernel],
                                              _ptr(cwt_ws), cwt_ws.numel()), "hf_find_halos_group")


def find_halos(pos: torch.Tensor, box_len: float, n: int, kw: float, frac_bits: int = 15, tau: float = 0.0,
               kernel: str = "sampled") -> dict:
    """Steps 2-6 at one scale, all on the GPU through one native call; one sync at the end."""
    ctx = context(pos.device.index)
    bufs = job_buffers(n, pos.shape[0], pos.device, True, frac_bits, with_stencil=kernel == "stencil")
    find_halos_async(pos, box_len, n, kw, bufs, frac_bits, tau, kernel, ctx)
    ctx.sync()
    cnt = int(bufs["count"].item())
    return {"rho": bufs["rho"], "cwt": bufs["cwt"], "maxima": bufs["maxima"][:cnt], "cell_label": bufs["cell_label"],
            "particle_label": bufs["particle_label"][: pos.shape[0]]}
