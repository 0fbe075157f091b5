"""Plain CPU FP64 oracle of the CWTHF single-scale hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the GPU library.

It follows the paper's identification steps 1-6 (Sec. 2, enumerated list) for
one scale:

  step 1  k_w = w L / 1000                          -> ``scale_w``
  step 2  CIC assignment, Eq. (1)                   -> ``deposit``
  step 3  grid CWT, Eqs. (2)-(4)                    -> ``cwt``
          or with the truncated stencil (Sec. 2.1)  -> ``stencil_cwt``
  step 4  local maxima of the grid CWT              -> ``maxima``
          and their correction for the grid (App. B) -> ``peaks``
  step 5  segmentation by the maxima (Sec. 2.3)     -> ``segment``
  step 6  particles take their cell's label         -> ``label``

and, after them, the group statistics of steps 5 and 7 with Table 1's
thresholds dens_th and particle_th                  -> ``group_stats``
and the cross-scale maximum check of step 8         -> ``cross_scale``
and the loop over scales of the flowchart           -> ``identify``

Readings taken where the paper is silent are listed in the design notes and
repeated at each function.  Everything here is deliberately unblocked and
unfused; numpy's FFT is used as a library primitive for the periodic
convolution, in FP64.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "scale_w", "fixed_point", "deposit", "total_mass", "mean_mass", "normalise",
    "wavelet", "wavelet_hat", "sampled_kernel", "kernel_hat", "cwt_field", "cwt",
    "gdw_resolution", "paper_grid", "stencil_half_width", "stencil", "stencil_cwt_field", "stencil_cwt", "stencil_cwt_at",
    "neighbour_offsets", "maxima", "is_maximum_at", "parents", "segment", "follow", "ngp_nodes", "label",
    "find_halos", "group_stats", "cross_scale", "peaks", "cube_size_term", "identify", "DepositOverflow",
    "GRAV", "self_bound",
]


class DepositOverflow(ArithmeticError):
    """A CIC cell sum does not fit a signed 64-bit integer."""


# --------------------------------------------------------------------------
# step 1: scale parameter
# --------------------------------------------------------------------------
def scale_w(kw: float, box_len: float) -> float:
    """w (h/Mpc) from the dimensionless k_w = w L_box / 1000 (Sec. 2, step 1 footnote)."""
    return 1000.0 * kw / box_len


# --------------------------------------------------------------------------
# step 2: cloud-in-cell deposit, Eq. (1)
# --------------------------------------------------------------------------
def fixed_point(pos: np.ndarray, box_len: float, n: int, frac_bits: int) -> np.ndarray:
    """Per-axis fixed-point coordinate q in [0, n 2^B), in units of 2^-B cell.

    Reading: the node g sits at g dx and the particle's CIC weights are taken
    from its position in cell units with B fraction bits.  The scale factor
    s = n 2^B / L is rounded once to the position dtype and t = x s is one
    correctly rounded multiply in that dtype; q = floor(t) mod n 2^B, so
    positions outside [0, L) wrap periodically.
    """
    pos = np.asarray(pos)
    if pos.dtype not in (np.float32, np.float64):
        raise TypeError("positions must be float32 or float64")
    if pos.ndim != 2 or pos.shape[1] != 3:
        raise ValueError("positions must have shape [np, 3]")
    ft = pos.dtype.type
    s = ft(float(n) * float(1 << frac_bits) / float(box_len))
    t = pos * s  # elementwise, in the position dtype
    if not np.all(np.isfinite(t)) or np.any(np.abs(t) >= 2.0 ** 62):
        raise ValueError("non-finite or out-of-range particle position")
    m = n << frac_bits
    return np.mod(np.floor(t).astype(np.int64), m)


def deposit(pos: np.ndarray, box_len: float, n: int, frac_bits: int = 15) -> np.ndarray:
    """CIC mass on the periodic n^3 grid, int64 in units of 2^-3B particle.

    Eq. (1): each particle becomes (at most) eight pseudo-particles on the grid
    nodes around it, with the usual tri-linear cloud-in-cell weights.  A node's
    weight along one axis is 2^B - f for the lower node and f for the upper,
    f being the fractional part of q; the eight products are summed exactly.
    Grid layout is [z][y][x].
    """
    if not 8 <= frac_bits <= 20:
        raise ValueError("frac_bits must be in [8, 20]")
    q = fixed_point(pos, box_len, n, frac_bits)
    one = 1 << frac_bits
    cell = q >> frac_bits
    f = q & (one - 1)
    w = (one - f, f)  # lower / upper node weight per axis
    # Exact sums: split each product (< 2^61) into 32-bit halves so that no
    # partial sum wraps, then recombine with Python integers for the check.
    lo = np.zeros(n ** 3, dtype=np.int64)
    hi = np.zeros(n ** 3, dtype=np.int64)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                iz = (cell[:, 2] + cz) % n
                iy = (cell[:, 1] + cy) % n
                ix = (cell[:, 0] + cx) % n
                idx = (iz * n + iy) * n + ix
                wt = w[cz][:, 2] * w[cy][:, 1] * w[cx][:, 0]
                np.add.at(lo, idx, wt & 0xFFFFFFFF)
                np.add.at(hi, idx, wt >> 32)
    # true cell value = hi * 2^32 + lo; it must be <= 2^63 - 1
    if np.any(hi + (lo >> 32) >= (1 << 31)):
        raise DepositOverflow("a CIC cell exceeds 2^63 - 1")
    rho = (hi << 32) + lo
    return rho.reshape(n, n, n)


def total_mass(rho: np.ndarray) -> int:
    """Exact integer sum of a non-negative int64 grid (may exceed 2^63)."""
    r = np.asarray(rho, dtype=np.int64).ravel()
    if np.any(r < 0):
        raise ValueError("negative cell mass")
    lo = int(np.sum(r & 0xFFFFFFFF, dtype=np.uint64))
    hi = int(np.sum(r >> 32, dtype=np.uint64))
    return (hi << 32) + lo


def mean_mass(rho: np.ndarray) -> float:
    """Mean cell mass: exact integer total rounded once to FP64, then / n^3."""
    return float(total_mass(rho)) / float(rho.size)


def normalise(rho: np.ndarray) -> np.ndarray:
    """f = rho / mean, so densities are in units of the mean density (step 7 unit)."""
    mbar = mean_mass(rho)
    if mbar == 0.0:
        raise ValueError("empty grid: the mean density is zero")
    return rho.astype(np.float64) / mbar


# --------------------------------------------------------------------------
# step 3: the grid CWT, Eqs. (2)-(4)
# --------------------------------------------------------------------------
def wavelet(w: float, r2) -> np.ndarray:
    """Isotropic Mexican-hat wavelet of Eq. (4) as a function of r^2."""
    u = (w * w) * np.asarray(r2, dtype=np.float64)
    return w ** 1.5 * (6.0 - u) * np.exp(-u / 4.0)


def wavelet_hat(w: float, k) -> np.ndarray:
    """Continuum Fourier transform of Eq. (4): 32 pi^1.5 w^-1.5 (k/w)^2 exp(-(k/w)^2).

    Derived from Eq. (4) with F(k) = int Psi(x) exp(-i k.x) d^3x.  It vanishes
    at k = 0 (zero-mean wavelet) and peaks at k = w.
    """
    s = (np.asarray(k, dtype=np.float64) / w) ** 2
    return 32.0 * math.pi ** 1.5 * w ** -1.5 * s * np.exp(-s)


def _image_count(w: float, box_len: float) -> int:
    # Images beyond |m| = I lie at distance >= (I + 1/2) L from every node
    # (offsets are minimum-image); choose the least I >= 0 with
    # w (I + 1/2) L >= 16, where |Psi| / Psi(0) < 1e-25: the images left out
    # sum to below 1e-24 of the peak, far under the FP64 rounding of the rest.
    return max(0, int(math.ceil(16.0 / (w * box_len) - 0.5)))


def sampled_kernel(n: int, box_len: float, w: float) -> np.ndarray:
    """dx^3 * sum over periodic images of Psi(w, x_j + m L), sampled on the grid.

    This is the paper's discretised convolution (Eq. (2) last line, Sec. 2.1):
    the wavelet sampled on the CIC grid spacing, here periodic and untruncated.
    Offsets are minimum-image node offsets.
    """
    dx = box_len / n
    j = np.arange(n)
    off = ((j + n // 2) % n - n // 2) * dx
    images = _image_count(w, box_len)
    k = np.zeros((n, n, n), dtype=np.float64)
    for mz in range(-images, images + 1):
        z = (off + mz * box_len)[:, None, None]
        for my in range(-images, images + 1):
            y = (off + my * box_len)[None, :, None]
            for mx in range(-images, images + 1):
                x = (off + mx * box_len)[None, None, :]
                k += wavelet(w, x * x + y * y + z * z)
    return k * dx ** 3


def kernel_hat(n: int, box_len: float, w: float, mode: str = "sampled") -> np.ndarray:
    """DFT-domain multiplier on the rfftn half-spectrum [n][n][n/2+1].

    ``sampled``: rfftn of the sampled kernel (real, since the kernel is even).
    ``analytic``: the continuum transform at the DFT wavenumbers 2 pi m / L.
    """
    if mode == "sampled":
        return np.fft.rfftn(sampled_kernel(n, box_len, w), axes=(0, 1, 2)).real
    if mode == "analytic":
        kf = 2.0 * math.pi * np.fft.fftfreq(n, d=box_len / n)
        kh = 2.0 * math.pi * np.fft.rfftfreq(n, d=box_len / n)
        k2 = kf[:, None, None] ** 2 + kf[None, :, None] ** 2 + kh[None, None, :] ** 2
        return wavelet_hat(w, np.sqrt(k2))
    raise ValueError("mode must be 'sampled' or 'analytic'")


def cwt_field(f: np.ndarray, box_len: float, w: float, mode: str = "sampled") -> np.ndarray:
    """C_j = sum_g f_g K(x_j - x_g): the periodic discrete convolution of Eq. (2)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    spec = np.fft.rfftn(f, axes=(0, 1, 2))
    spec *= kernel_hat(n, box_len, w, mode)
    return np.fft.irfftn(spec, s=f.shape, axes=(0, 1, 2))


def cwt(rho: np.ndarray, box_len: float, kw: float, mode: str = "sampled") -> np.ndarray:
    """Step 3 on a CIC grid: normalise to the mean density, then Eq. (2).
    ``stencil`` is the truncated real-space stencil of Sec. 2.1 with Table 1's
    extent (``stencil_cwt``)."""
    if mode == "stencil":
        return stencil_cwt(rho, box_len, kw)
    return cwt_field(normalise(rho), box_len, scale_w(kw, box_len), mode)


# --------------------------------------------------------------------------
# step 3 by the paper's own discretisation: the truncated real-space stencil
# --------------------------------------------------------------------------
def gdw_resolution(kw: float) -> int:
    """Table 1's wavelet grid resolution Int(1.5 / k_w + 5).

    Read as the stencil's half-width in cells of the paper's grid for that
    scale: offsets -h..h on every axis, 2h + 1 points per axis (the paper does
    not say whether the count is the half or the full width)."""
    return int(1.5 / kw + 5.0)


def paper_grid(kw: float) -> int:
    """The flowchart's grid size for a scale, N_g = Int(400 k_w + 150)."""
    return int(400.0 * kw + 150.0)


def stencil_half_width(kw: float, n: int) -> int:
    """Half-width in cells of an n^3 grid covering the physical extent of
    Table 1's count on the paper's own grid: ceil(gdw_resolution(k_w) n / N_g).

    Reading: the flowchart deposits each scale on N_g = Int(400 k_w + 150)
    cells, where the scale length is 0.4 + 0.15 / k_w cells and Table 1's
    count spans 10-12 scale lengths, far enough that the truncated Mexican hat
    keeps its zero mean.  On another grid the same count of cells would cover
    a different extent (3.5 scale lengths at n = 1024, k_w = 0.512), so the
    extent is kept instead; on the paper's grid this is the count itself."""
    c, ng = gdw_resolution(kw), paper_grid(kw)
    return (c * int(n) + ng - 1) // ng


def stencil(n: int, box_len: float, w: float, half_width: int) -> np.ndarray:
    """dx^3 Psi(w, d dx) on the cube of node offsets |d_i| <= h, [2h+1]^3.

    Sec. 2.1: the wavelet sampled on the CIC grid spacing, truncated to the
    stencil, with no periodic images (the stencil itself wraps on the box)."""
    dx = box_len / n
    d = np.arange(-half_width, half_width + 1, dtype=np.float64) * dx
    r2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    return wavelet(w, r2) * dx ** 3


def stencil_cwt_field(f: np.ndarray, box_len: float, w: float, half_width: int) -> np.ndarray:
    """Sec. 2.1's superposition: every grid point g adds f_g times the stencil
    centred on g, periodically, C_j = sum_{|d_i| <= h} S_d f_{j - d}.

    Points with f_g = 0 add nothing, so the sum runs over all of them at once:
    one shifted copy of the grid per stencil offset, weighted and added (the
    array additions the paper describes).  A stencil wider than the box
    (2h + 1 > n) adds a point's wrapped offsets onto the same cells."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    h = int(half_width)
    s = stencil(n, box_len, w, h)
    c = np.zeros_like(f)
    for iz, dz in enumerate(range(-h, h + 1)):
        fz = np.roll(f, dz, axis=0)
        for iy, dy in enumerate(range(-h, h + 1)):
            fzy = np.roll(fz, dy, axis=1)
            for ix, dxo in enumerate(range(-h, h + 1)):
                c += s[iz, iy, ix] * np.roll(fzy, dxo, axis=2)
    return c


def stencil_cwt_at(rho: np.ndarray, box_len: float, kw: float, half_width: int, cells) -> np.ndarray:
    """stencil_cwt at the given linear cell indices only, each a sum over its
    own (2h+1)^3 window of f = rho / mean, for grids too large to superpose
    whole.  The mean is that of the whole grid."""
    rho = np.asarray(rho)
    n = rho.shape[0]
    h = int(half_width)
    mbar = mean_mass(rho)
    if mbar == 0.0:
        raise ValueError("empty grid: the mean density is zero")
    s = stencil(n, box_len, scale_w(kw, box_len), h)
    out = np.empty(len(cells), dtype=np.float64)
    for k, j in enumerate(np.asarray(cells, dtype=np.int64).tolist()):
        z, y, x = j // (n * n), (j // n) % n, j % n
        # window[a, b, c] = f at (z, y, x) - d for d = (a, b, c) - h, matching S_d
        iz = [(z - d) % n for d in range(-h, h + 1)]
        iy = [(y - d) % n for d in range(-h, h + 1)]
        ix = [(x - d) % n for d in range(-h, h + 1)]
        win = rho[np.ix_(iz, iy, ix)].astype(np.float64) / mbar
        out[k] = float(np.sum(s * win))
    return out


def stencil_cwt(rho: np.ndarray, box_len: float, kw: float, half_width: int | None = None) -> np.ndarray:
    """Step 3 with the truncated stencil: normalise to the mean density, then
    superpose; the half-width defaults to Table 1's extent on this grid
    (``stencil_half_width``)."""
    h = stencil_half_width(kw, np.asarray(rho).shape[0]) if half_width is None else int(half_width)
    if h < 0:
        raise ValueError("half_width must be >= 0")
    return stencil_cwt_field(normalise(rho), box_len, scale_w(kw, box_len), h)


# --------------------------------------------------------------------------
# step 4: local maxima
# --------------------------------------------------------------------------
def neighbour_offsets():
    """The 26 (dz, dy, dx) offsets of the 3x3x3 neighbourhood without the centre."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if (dz, dy, dx) != (0, 0, 0)]


def _check_field(c: np.ndarray) -> np.ndarray:
    c = np.asarray(c)
    if c.ndim != 3 or not (c.shape[0] == c.shape[1] == c.shape[2]):
        raise ValueError("field must be n^3")
    if np.any(np.isnan(c)):
        raise ValueError("NaN in the CWT field")
    return c


def _beats(c_a, i_a, c_b, i_b):
    """Strict total order on (value, linear index): a beats b.

    Equal values (with -0 equal to +0) are broken by the larger linear index.
    """
    return (c_a > c_b) | ((c_a == c_b) & (i_a > i_b))


def maxima(c: np.ndarray, tau: float = 0.0) -> np.ndarray:
    """Sorted linear indices of cells that beat all 26 periodic neighbours and exceed tau.

    Step 4 and Sec. 2.3: a halo is a positive CWT peak; tau = 0 by default.
    Comparisons are made in the dtype of ``c``.
    """
    c = _check_field(c)
    n = c.shape[0]
    idx = np.arange(n ** 3, dtype=np.int64).reshape(n, n, n)
    is_max = c > c.dtype.type(tau)
    for (dz, dy, dx) in neighbour_offsets():
        nb_c = np.roll(c, (-dz, -dy, -dx), axis=(0, 1, 2))
        nb_i = np.roll(idx, (-dz, -dy, -dx), axis=(0, 1, 2))
        is_max &= _beats(c, idx, nb_c, nb_i)
    return np.flatnonzero(is_max.ravel()).astype(np.int64)


def is_maximum_at(c: np.ndarray, cells, tau: float = 0.0) -> np.ndarray:
    """``maxima``'s test evaluated at the given linear cells only: the cell beats
    each of its 26 periodic neighbours in the (value, index) order and exceeds
    tau.  For fields too large to test whole."""
    c = np.asarray(c)
    n = c.shape[0]
    cells = np.asarray(cells, dtype=np.int64).ravel()
    z, y, x = cells // (n * n), (cells // n) % n, cells % n
    v = c[z, y, x]
    if np.any(np.isnan(v)):
        raise ValueError("NaN in the CWT field")
    ok = v > c.dtype.type(tau)
    for (dz, dy, dx) in neighbour_offsets():
        k = (((z + dz) % n) * n + (y + dy) % n) * n + (x + dx) % n
        u = c.ravel()[k]
        if np.any(np.isnan(u)):
            raise ValueError("NaN in the CWT field")
        ok &= _beats(v, cells, u, k)
    return ok


# --------------------------------------------------------------------------
# step 5: segmentation
# --------------------------------------------------------------------------
def _peak_fits(c: np.ndarray, roots):
    """Step 4's per-axis quadratic through each grid maximum (App. B), FP64.

    For the maximum B and its two neighbours along an axis, A the larger and
    C the smaller one, take l1 = A - C and l2 = B - C (App. B puts A, B, C at
    heights l1, l2, 0, one cell apart).  The parabola through the three points
    tops out l1^2 / (16 l2 - 8 l1) above B, and its vertex lies
    l1 / (2 (2 l2 - l1)) cells from B towards A.  A flat axis (l2 = 0, hence
    A = B = C) contributes nothing.

    Returns the shift of every root in cells [k][3] (x, y, z), the grid value
    plus the three axes' corrections added in the order x, y, z [k], and the
    means of l1 and of l2 over the three axes [k] (used by the cube-size term).
    """
    c = _check_field(c).astype(np.float64)
    n = c.shape[0]
    roots = np.asarray(roots, dtype=np.int64).ravel()
    z, y, x = roots // (n * n), (roots // n) % n, roots % n
    centre = c[z, y, x]
    value = centre.copy()
    shift = np.zeros((roots.size, 3), dtype=np.float64)
    l1s, l2s = [], []
    for ax, (ex, ey, ez) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        up = c[(z + ez) % n, (y + ey) % n, (x + ex) % n]
        down = c[(z - ez) % n, (y - ey) % n, (x - ex) % n]
        a = np.maximum(up, down)
        low = np.minimum(up, down)
        l1, l2 = a - low, centre - low
        flat = l2 == 0.0
        den = np.where(flat, 1.0, 16.0 * l2 - 8.0 * l1)
        corr = np.where(flat, 0.0, l1 * l1 / den)
        toward = np.where(up >= down, 1.0, -1.0)
        shift[:, ax] = np.where(flat, 0.0, toward * l1 / np.where(flat, 1.0, 2.0 * (2.0 * l2 - l1)))
        value = value + corr
        l1s.append(l1)
        l2s.append(l2)
    l1bar = (l1s[0] + l1s[1] + l1s[2]) / 3.0
    l2bar = (l2s[0] + l2s[1] + l2s[2]) / 3.0
    return shift, value, l1bar, l2bar


def peaks(c: np.ndarray, roots, box_len: float):
    """Step 4's correction of grid maxima for the finite grid (App. B, first
    part): each maximum moves to the vertex of its per-axis quadratics and its
    value rises by their corrections (``_peak_fits``).

    Returns positions [k][3] (x, y, z) in box units, wrapped into [0, L), and
    the corrected values [k].
    """
    c = _check_field(c)
    n = c.shape[0]
    dx = box_len / n
    roots = np.asarray(roots, dtype=np.int64).ravel()
    z, y, x = roots // (n * n), (roots // n) % n, roots % n
    shift, value, _, _ = _peak_fits(c, roots)
    pos = np.stack([x, y, z], axis=1).astype(np.float64) + shift
    return np.mod(pos * dx, box_len), value


def cube_size_term(l1bar, l2bar, n_scale: int, n_smaller: int):
    """App. B's second correction, made to a maximum of the larger scale before
    it is compared with a smaller scale on a finer grid: the grid value of a
    peak is the average over its cube, and the average over the smaller cube of
    the finer grid is higher.  With the peak taken as the average of the three
    per-axis quadratics, the difference is (3/16)(2 l2bar - l1bar)
    [1 - (r1/r2)^2], r2 and r1 the two grid spacings; the paper removes the
    factor 3/5 from it, leaving (5/16)(2 l2bar - l1bar)[1 - (r1/r2)^2].

    r1 / r2 = (L / n_smaller) / (L / n_scale) = n_scale / n_smaller, so the
    term vanishes when both scales share one grid.  Evaluated in FP64 as
    (0.3125 (2 l2bar - l1bar)) (1 - r r) with r = n_scale / n_smaller.
    """
    r = float(n_scale) / float(n_smaller)
    return (0.3125 * (2.0 * np.asarray(l2bar) - np.asarray(l1bar))) * (1.0 - r * r)


def parents(c: np.ndarray) -> np.ndarray:
    """parent(j) = the cell of {j} + N26(j) that is largest in the (value, index) order."""
    c = _check_field(c)
    n = c.shape[0]
    idx = np.arange(n ** 3, dtype=np.int64).reshape(n, n, n)
    best_c = c.copy()
    best_i = idx.copy()
    for (dz, dy, dx) in neighbour_offsets():
        nb_c = np.roll(c, (-dz, -dy, -dx), axis=(0, 1, 2))
        nb_i = np.roll(idx, (-dz, -dy, -dx), axis=(0, 1, 2))
        take = _beats(nb_c, nb_i, best_c, best_i)
        best_c = np.where(take, nb_c, best_c)
        best_i = np.where(take, nb_i, best_i)
    return best_i.ravel()


def segment(c: np.ndarray, tau: float = 0.0) -> np.ndarray:
    """Cell labels: the root reached by steepest ascent, or -1.

    Sec. 2.3 extends each halo from its positive peak out to the CWT valley
    with no threshold.  Reading: every cell climbs to its largest neighbour
    until it reaches a local maximum (its root); the basins meet at the
    valleys.  Cells whose root is not above tau get -1.
    """
    c = _check_field(c)
    par = parents(c)
    root = par.copy()
    active = np.flatnonzero(par[root] != root)
    while active.size:  # follow the parent chain one step at a time
        root[active] = par[root[active]]
        active = active[par[root[active]] != root[active]]
    flat = c.ravel()
    return np.where(flat[root] > flat.dtype.type(tau), root, -1).astype(np.int64).reshape(c.shape)


def follow(c: np.ndarray, cells, tau: float = 0.0) -> np.ndarray:
    """``segment``'s label of the given linear cells only, by walking the
    steepest-ascent path from each: step to the largest of the cell and its 26
    periodic neighbours in the (value, index) order until the cell is its own
    largest.  For fields too large to segment whole."""
    c = np.asarray(c)
    n = c.shape[0]
    flat = c.ravel()
    offs = np.array(neighbour_offsets() + [(0, 0, 0)], dtype=np.int64)
    cur = np.asarray(cells, dtype=np.int64).ravel().copy()
    active = np.arange(cur.size)
    while active.size:
        j = cur[active]
        z, y, x = j // (n * n), (j // n) % n, j % n
        cand = (((z[:, None] + offs[:, 0]) % n) * n + (y[:, None] + offs[:, 1]) % n) * n + (x[:, None] + offs[:, 2]) % n
        vals = flat[cand]
        if np.any(np.isnan(vals)):
            raise ValueError("NaN in the CWT field")
        best_v, best_i = vals[:, 0].copy(), cand[:, 0].copy()
        for k in range(1, cand.shape[1]):
            take = _beats(vals[:, k], cand[:, k], best_v, best_i)
            best_v = np.where(take, vals[:, k], best_v)
            best_i = np.where(take, cand[:, k], best_i)
        moved = best_i != j
        cur[active] = best_i
        active = active[moved]
    return np.where(flat[cur] > flat.dtype.type(tau), cur, -1).astype(np.int64)


# --------------------------------------------------------------------------
# step 6: particle labels
# --------------------------------------------------------------------------
def ngp_nodes(pos: np.ndarray, box_len: float, n: int, frac_bits: int = 15) -> np.ndarray:
    """Linear index of each particle's nearest node (the largest CIC weight).

    Reading: a particle belongs to the node carrying its largest CIC weight;
    at exactly half a cell it goes to the upper node.
    """
    q = fixed_point(pos, box_len, n, frac_bits)
    node = ((q + (1 << (frac_bits - 1))) >> frac_bits) % n
    return (node[:, 2] * n + node[:, 1]) * n + node[:, 0]


def label(pos: np.ndarray, box_len: float, n: int, cell_label: np.ndarray,
          frac_bits: int = 15) -> np.ndarray:
    """Step 6: a particle gets the label (temporary ID) of its segmented cell."""
    return np.asarray(cell_label).ravel()[ngp_nodes(pos, box_len, n, frac_bits)]


# --------------------------------------------------------------------------
# steps 5 and 7: group volume, mass and density; Table 1 thresholds
# --------------------------------------------------------------------------
def group_stats(cell_label, particle_label, roots, n: int, np_total: int, dens_th: float = 4.0,
                particle_th: int = 15, root_ok=None) -> dict:
    """Grid volume, particle number and density filter of every group.

    Step 5 gives each segmented structure its grid volume: the cells that carry
    its label, each of volume (L/n)^3.  Step 6 makes the particles of one label
    a group; the particles have equal mass, so a group's mass is its particle
    number.  Step 7 disposes of groups whose density is below dens_th times the
    mean density of the whole box, N_p / L^3 (Table 1: dens_th = 4), and
    Table 1's particle_th (15) is the minimum particle number.

    Reading: the density test N_g / (V_g (L/n)^3) >= dens_th N_p / L^3 is,
    with V_g counted in cells, N_g n^3 >= dens_th V_g N_p; it is decided in FP64
    as float(N_g) * float(n^3) >= (dens_th * float(V_g)) * float(N_p).  A group
    is kept if it passes that test and has at least particle_th particles.

    ``roots`` is the sorted maxima list (the labels in use); the per-group
    arrays are indexed like it.  ``root_ok`` (optional, one flag per root)
    disposes of the groups whose maximum failed another test, such as the
    cross-scale check of step 8.  Returns the particle number, the cell count and
    the keep flag of every group, and both label arrays with the labels of
    disposed groups replaced by -1.
    """
    roots = np.asarray(roots, dtype=np.int64).ravel()
    cl = np.asarray(cell_label).ravel().astype(np.int64)
    pl = np.asarray(particle_label).ravel().astype(np.int64)
    ncell = n ** 3
    # per root cell: cells and particles carrying that label
    cells_at = np.bincount(cl[cl >= 0], minlength=ncell)
    parts_at = np.bincount(pl[pl >= 0], minlength=ncell)
    g_cells = cells_at[roots]
    g_parts = parts_at[roots]
    dense = g_parts.astype(np.float64) * float(ncell) >= (float(dens_th) * g_cells.astype(np.float64)) * float(np_total)
    keep = dense & (g_parts >= particle_th)
    if root_ok is not None:
        keep &= np.asarray(root_ok, dtype=bool).ravel()
    keep_at = np.zeros(ncell, dtype=bool)
    keep_at[roots[keep]] = True
    new_pl = np.where(pl >= 0, np.where(keep_at[np.maximum(pl, 0)], pl, -1), -1)
    new_cl = np.where(cl >= 0, np.where(keep_at[np.maximum(cl, 0)], cl, -1), -1)
    return {
        "particles": g_parts.astype(np.int64),
        "cells": g_cells.astype(np.int64),
        "keep": keep,
        "particle_label": new_pl.astype(np.int32),
        "cell_label": new_cl.astype(np.int32).reshape(np.shape(cell_label)),
    }


# --------------------------------------------------------------------------
# step 8: cross-scale maxima
# --------------------------------------------------------------------------
def cross_scale(c_scale: np.ndarray, c_smaller: np.ndarray, roots) -> np.ndarray:
    """Which maxima of one scale are also maxima across scale (step 8, with
    the comparison of the flowchart's two grids described in Sec. 2).

    Each maximum is first corrected for the grid (step 4, App. B): its value
    becomes the top of its per-axis quadratics plus the cube-size term for the
    smaller scale's grid spacing, and its position the vertex of those
    quadratics.  It is kept if that value strictly exceeds the smaller scale's
    CWT at every grid point near the same physical position.

    Readings: "near" is the smaller scale's grid node nearest the corrected
    position (half a cell rounds up) and its 26 periodic neighbours; the
    smaller scale's values are its raw grid values (App. B adjusts the larger
    scale's maxima only).  The two fields may be on grids of different size
    n_scale and n_smaller over the same box; on one grid the cube-size term is
    zero.  The position in the smaller grid's cells is
    ((g + shift) n_smaller) / n_scale, FP64 throughout.

    Returns one flag per root of ``roots`` (linear cell indices of c_scale).
    """
    cs = _check_field(c_scale)
    cm = _check_field(c_smaller).astype(np.float64)
    n2, n1 = cs.shape[0], cm.shape[0]
    roots = np.asarray(roots, dtype=np.int64).ravel()
    shift, value, l1bar, l2bar = _peak_fits(cs, roots)
    value = value + cube_size_term(l1bar, l2bar, n2, n1)
    g = np.stack([roots % n2, (roots // n2) % n2, roots // (n2 * n2)], axis=1).astype(np.float64)
    u = ((g + shift) * float(n1)) / float(n2)
    node = np.mod(np.floor(u + 0.5).astype(np.int64), n1)  # (x, y, z) on the smaller grid
    near = np.full(roots.size, -np.inf)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                v = cm[(node[:, 2] + dz) % n1, (node[:, 1] + dy) % n1, (node[:, 0] + dx) % n1]
                near = np.maximum(near, v)
    return value > near


# --------------------------------------------------------------------------
# steps 9-10: the self-boundness check (Sec. 2.3)
# --------------------------------------------------------------------------
# Newton's constant in (Mpc/h) (km/s)^2 / (M_sun/h): G M_sun / Mpc from
# G = 6.67430e-11 m^3 kg^-1 s^-2, M_sun = 1.98841e30 kg, Mpc = 3.0856775814913673e22 m
# (the factors of h cancel in G M / r with masses in M_sun/h and lengths in Mpc/h).
GRAV = 6.67430e-11 * 1.98841e30 / 3.0856775814913673e22 / 1.0e6


def self_bound(pos, vel, box_len: float, members, ref, grav_mass: float, margins: bool = False):
    """The self-boundness check of one group (Sec. 2.3, steps 9-10), FP64.

    ``members`` are the group's particle indices (ascending), ``ref`` a point
    of the group (its root node) about which positions are unwrapped
    periodically (minimum image), ``grav_mass`` = G m_p for the equal particle
    mass m_p, in (Mpc/h) (km/s)^2.  Each round:

      centre c = mean of the remaining members' unwrapped positions (the
      centre of mass, equal masses), bulk velocity u = mean of their velocities;
      r_i = |x_i - c|; in the order of increasing (r_i, member position) the
      shells inside and at r_i act as a point mass at the centre, the shells
      outside as shells: Phi_i = -G m [(rank_i + 1) / r_i + sum over later j
      of 1 / r_j] (spherical symmetry); the local escape speed is
      sqrt(-2 Phi_i), and particle i escapes if |v_i - u|^2 > -2 Phi_i.

    Escaping particles are removed and the round repeats until none escapes.
    The group is kept unless more than 40% of its particles were removed
    (decided exactly: 5 removed > 2 N).  Readings: peculiar velocities relative to the remaining
    members' mean, no Hubble flow; the potential of the remaining members only;
    a member exactly at the centre (r = 0) is bound.

    Returns the bound flags of the members, the kept flag and the rounds made
    (with ``margins``, also the smallest |(|v - u|^2 + 2 Phi)| / |2 Phi| of
    any decision made, a diagnostic of how far each one was from a tie).
    """
    members = np.asarray(members, dtype=np.int64).ravel()
    n0 = members.size
    x = np.asarray(pos, dtype=np.float64)[members]
    v = np.asarray(vel, dtype=np.float64)[members]
    d = x - np.asarray(ref, dtype=np.float64)
    half = 0.5 * box_len
    d = np.where(d >= half, d - box_len, np.where(d < -half, d + box_len, d))  # minimum image
    alive = np.ones(n0, dtype=bool)
    rounds = 0
    margin = np.inf
    while alive.any():
        rounds += 1
        idx = np.flatnonzero(alive)
        c = d[idx].sum(axis=0) / idx.size
        u = v[idx].sum(axis=0) / idx.size
        r = np.sqrt(((d[idx] - c) ** 2).sum(axis=1))
        order = np.lexsort((idx, r))  # by radius, ties by member position
        rs = r[order]
        with np.errstate(divide="ignore"):
            inv = 1.0 / rs
        outer = np.concatenate([np.cumsum(inv[::-1])[::-1][1:], [0.0]])  # sum over later shells
        with np.errstate(divide="ignore", invalid="ignore"):
            phi = -grav_mass * (np.arange(1, idx.size + 1) / rs + outer)
        speed2 = ((v[idx[order]] - u) ** 2).sum(axis=1)
        escape = speed2 > -2.0 * phi  # r = 0: -2 phi = inf, bound
        if margins:
            with np.errstate(invalid="ignore", divide="ignore"):
                rel = np.abs(speed2 + 2.0 * phi) / np.abs(2.0 * phi)
            margin = min(margin, float(np.nanmin(rel)) if rel.size else np.inf)
        if not escape.any():
            break
        alive[idx[order][escape]] = False
    removed = n0 - int(alive.sum())
    kept = bool(5 * removed <= 2 * n0 and alive.any())
    return (alive, kept, rounds, margin) if margins else (alive, kept, rounds)


# --------------------------------------------------------------------------
# the identification loop over scales (Sec. 2 and its flowchart)
# --------------------------------------------------------------------------
def identify(pos, box_len: float, n: int, kws, dens_th: float = 4.0, particle_th: int = 15,
             frac_bits: int = 15, tau: float = 0.0, mode: str = "sampled", decide_dtype=np.float64,
             grids=None, vel=None, grav_mass: float | None = None) -> dict:
    """Steps 2-8 over the scales ``kws`` (increasing k_w: from the largest
    scale length down), without the self-boundness check of steps 9-10.

    The flowchart keeps two grids: the one being identified and the next
    (smaller) scale's.  Each scale in turn: its maxima and segmentation; the
    particles that no earlier scale has claimed take their cell's label (a
    temporary ID); groups are formed from those particles and a group is
    discarded unless it passes the density and particle-number thresholds
    (step 7) and its maximum, corrected for the grid as step 4 asks (App. B),
    exceeds the next scale's field near its corrected position (step 8; after
    the last scale the next grid is all zeros, of the last scale's size).  The
    particles of a kept group are claimed at this scale with the group's root
    as their ID.

    Grids: by default every scale uses the box's n^3 grid.  ``grids`` gives
    each scale its own grid size instead; ``grids="paper"`` is the flowchart's
    N_g = Int(400 k_w + 150) per scale (step 1), where each scale deposits the
    particles afresh (step 2) and the cross-scale check compares grids of
    different spacing with App. B's cube-size term.  A group's grid volume and
    the density test count cells of its own scale's grid.  Reading: the density
    of a group counts the particles it takes at its scale against the mean of
    all particles.

    With velocities ``vel`` [np][3] (km/s) and ``grav_mass`` = G m_p, steps 9
    and 10 follow: every group kept by steps 7-8 takes the self-boundness check
    (``self_bound``) on its particles, and only its bound particles are
    claimed; a group that fails the check, or whose bound particles number
    fewer than particle_th (Table 1's minimum particle number of a halo), is
    discarded and claims none.  Particles it leaves stay free for the next
    scales.
    """
    kws = [float(k) for k in kws]
    if not kws or any(b <= a for a, b in zip(kws, kws[1:])):
        raise ValueError("scales must be given in increasing k_w")
    if grids is None:
        sizes = [int(n)] * len(kws)
    elif isinstance(grids, str):
        if grids != "paper":
            raise ValueError("grids must be None, 'paper' or one size per scale")
        sizes = [paper_grid(kw) for kw in kws]
    else:
        sizes = [int(g) for g in grids]
        if len(sizes) != len(kws):
            raise ValueError("one grid size per scale")
    np_total = len(pos)
    rhos = {}
    for size in sizes:
        if size not in rhos:
            rhos[size] = deposit(pos, box_len, size, frac_bits)
    fields = [cwt(rhos[size], box_len, kw, mode).astype(decide_dtype) for size, kw in zip(sizes, kws)]
    halo_scale = np.full(np_total, -1, dtype=np.int64)
    halo_root = np.full(np_total, -1, dtype=np.int64)
    per_scale = []
    for i, c in enumerate(fields):
        ni = sizes[i]
        nxt = fields[i + 1] if i + 1 < len(fields) else np.zeros_like(c)  # the flowchart's zero current_grid
        roots = maxima(c, tau)
        cell = segment(c, tau)
        pl = label(pos, box_len, ni, cell, frac_bits)
        pl = np.where(halo_scale >= 0, -1, pl)  # only particles with no label yet
        ok = cross_scale(c, nxt, roots)
        g = group_stats(cell, pl, roots, ni, np_total, dens_th, particle_th, root_ok=ok)
        plab = g["particle_label"].astype(np.int64)
        bound_keep = g["keep"].copy()
        if vel is not None:
            dxi = box_len / ni
            for k in np.flatnonzero(g["keep"]):
                rt = int(roots[k])
                members = np.flatnonzero(plab == rt)
                ref = np.array([rt % ni, (rt // ni) % ni, rt // (ni * ni)], dtype=np.float64) * dxi
                bound, kept, _ = self_bound(pos, vel, box_len, members, ref, grav_mass)
                if not kept or int(bound.sum()) < particle_th:
                    bound_keep[k] = False
                    bound[:] = False
                plab[members[~bound]] = -1
        take = plab >= 0
        halo_scale[take] = i
        halo_root[take] = plab[take]
        per_scale.append({"grid": ni, "cwt": c, "maxima": roots, "cell_label": cell, "cross_scale": ok,
                          "particles": g["particles"], "cells": g["cells"], "keep": g["keep"],
                          "bound_keep": bound_keep, "particle_label": plab.astype(np.int32)})
    return {"rho": rhos[sizes[0]], "rhos": [rhos[size] for size in sizes], "grids": sizes, "scales": per_scale,
            "halo_scale": halo_scale, "halo_root": halo_root}


# --------------------------------------------------------------------------
# the whole single-scale path
# --------------------------------------------------------------------------
def find_halos(pos, box_len: float, n: int, kw: float, frac_bits: int = 15,
               tau: float = 0.0, mode: str = "sampled", decide_dtype=np.float64) -> dict:
    """Steps 2-6 at one scale.  ``decide_dtype`` is the precision the maxima and
    segmentation comparisons are made in (float64, or float32 to decide as an
    FP32 pipeline would on the rounded field)."""
    rho = deposit(pos, box_len, n, frac_bits)
    c = cwt(rho, box_len, kw, mode)
    cd = c.astype(decide_dtype)
    cell = segment(cd, tau)
    return {
        "rho": rho,
        "cwt": c,
        "maxima": maxima(cd, tau),
        "cell_label": cell,
        "particle_label": label(pos, box_len, n, cell, frac_bits),
    }
