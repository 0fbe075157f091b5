"""Seeded synthetic inputs for the CWT halo-finder hot path.

This module only draws random particle boxes, job streams and smooth test
fields.  It holds none of
the halo finder's arithmetic (no deposit, transform, maxima or segmentation), so
both the FP64 oracle and the GPU path can take their inputs from it.

Recipe (a stand-in for the paper's SIMBA m50n512 dark-matter snapshot,
Sec. 3, which is not available):

* ``halo_frac`` (60%) of the particles sit in NFW spheres.  Halo masses follow
  dN/dM ~ M^-1.9 on [50, 5000] particles (inverse CDF), then are scaled to the
  60% budget with largest-remainder rounding so the counts are exact integers.
* r_vir = (3 M / (4 pi 200 nbar))^(1/3) with nbar = N_p / L^3 (the r_200
  radius the paper compares halo extents with, Sec. 2.3), concentration
  c ~ U[4, 10], radii from the NFW enclosed-mass profile truncated at r_vir,
  isotropic directions.
* The remaining particles are uniform in the box.
* Positions are wrapped into [0, L), cast to the configured dtype and put in a
  seeded random order, so particle order carries no spatial locality.

All draws go through one ``torch.Generator``; the stream is fixed by
(seed, device).  CPU generation is used for everything the oracle checks at full
size; very large boxes may be drawn on the GPU, whose stream differs from the
CPU one for the same seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

HALO_FRAC = 0.6
M_MIN, M_MAX, MASS_SLOPE = 50.0, 5000.0, -1.9
C_LO, C_HI = 4.0, 10.0
DELTA_VIR = 200.0


@dataclass(frozen=True)
class BoxConfig:
    """One synthetic periodic box: side ``box_len`` (Mpc/h), grid ``n``^3."""

    name: str
    box_len: float
    n: int
    n_particles: int
    n_halos: int
    dtype: str  # "f32" or "f64"
    seed: int
    scales_cells: tuple = (2.0,)  # wavelet scale lengths 1/w, in grid cells

    @property
    def kw_list(self):
        # k_w = w L / 1000 (Sec. 2, step 1); w = 1/(a dx) with dx = L/n.
        return [self.n / (1000.0 * a) for a in self.scales_cells]


CONFIGS = {
    "M1": BoxConfig("M1", 100.0, 64, 64 ** 3, 200, "f64", 1, (2.0,)),
    "M2": BoxConfig("M2", 250.0, 256, 256 ** 3, 20000, "f32", 2, (2.0,)),
    "M3": BoxConfig("M3", 500.0, 512, 512 ** 3, 150000, "f32", 3, (1.0, 2.0, 4.0)),
    "M4": BoxConfig("M4", 1000.0, 1024, 1024 ** 3, 1200000, "f32", 4, (2.0,)),
}

SERVE_SIZES = (64, 96, 128, 192, 256)


def _torch_dtype(dtype: str):
    return {"f32": torch.float32, "f64": torch.float64}[dtype]


def halo_counts(gen: torch.Generator, n_halos: int, budget: int, device) -> torch.Tensor:
    """Integer particle counts per halo: power-law draw scaled to ``budget``."""
    if n_halos == 0 or budget == 0:
        return torch.zeros(n_halos, dtype=torch.int64, device=device)
    u = torch.rand(n_halos, generator=gen, dtype=torch.float64, device=device)
    e = 1.0 + MASS_SLOPE
    lo, hi = M_MIN ** e, M_MAX ** e
    m = (lo + u * (hi - lo)) ** (1.0 / e)
    raw = m * (budget / m.sum())
    base = torch.floor(raw)
    rem = int(budget - int(base.sum().item()))
    frac = raw - base
    order = torch.argsort(frac, descending=True, stable=True)
    counts = base.to(torch.int64)
    if rem > 0:
        counts[order[:rem]] += 1
    return counts


def nfw_radius(gen: torch.Generator, conc: torch.Tensor) -> torch.Tensor:
    """r / r_vir drawn from the NFW enclosed mass mu(x) = ln(1+x) - x/(1+x), x <= c."""
    u = torch.rand(conc.shape, generator=gen, dtype=torch.float64, device=conc.device)
    y = u * (torch.log1p(conc) - conc / (1.0 + conc))
    lo = torch.zeros_like(conc)
    hi = conc.clone()
    for _ in range(56):  # bisection; mu is increasing in x
        mid = 0.5 * (lo + hi)
        below = (torch.log1p(mid) - mid / (1.0 + mid)) < y
        lo = torch.where(below, mid, lo)
        hi = torch.where(below, hi, mid)
    return 0.5 * (lo + hi) / conc


def _draw_box(box_len: float, n_particles: int, n_halos: int, seed: int, device, halo_frac: float):
    """Unpermuted FP64 positions, halo membership and halo properties, then the
    permutation, all from one generator stream."""
    device = torch.device(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = torch.float64
    budget = int(round(halo_frac * n_particles)) if n_halos > 0 else 0
    counts = halo_counts(gen, n_halos, budget, device)
    n_in_halos = int(counts.sum().item()) if n_halos > 0 else 0
    centres = torch.rand((n_halos, 3), generator=gen, dtype=f64, device=device) * box_len
    conc = C_LO + (C_HI - C_LO) * torch.rand(n_halos, generator=gen, dtype=f64, device=device)
    nbar = n_particles / box_len ** 3
    r_vir = (3.0 * counts.to(f64) / (4.0 * math.pi * DELTA_VIR * nbar)) ** (1.0 / 3.0)

    pos = torch.empty((n_particles, 3), dtype=f64, device=device)
    owner = None
    if n_in_halos > 0:
        owner = torch.repeat_interleave(torch.arange(n_halos, device=device), counts)
        r = nfw_radius(gen, conc[owner]) * r_vir[owner]
        d = torch.randn((n_in_halos, 3), generator=gen, dtype=f64, device=device)
        d = d / torch.linalg.vector_norm(d, dim=1, keepdim=True).clamp_min(1e-300)
        pos[:n_in_halos] = centres[owner] + r[:, None] * d
        del r, d
    n_uniform = n_particles - n_in_halos
    if n_uniform > 0:
        pos[n_in_halos:] = torch.rand((n_uniform, 3), generator=gen, dtype=f64, device=device) * box_len
    pos = torch.remainder(pos, box_len)
    perm_gen = gen  # the permutation is the stream's last draw
    return pos, owner, counts, r_vir, n_in_halos, perm_gen


def _finish(pos: torch.Tensor, box_len: float, dtype: str) -> torch.Tensor:
    out = pos.to(_torch_dtype(dtype))
    top = torch.tensor(box_len, dtype=out.dtype, device=out.device)
    return torch.where(out >= top, out - top, out)  # values rounded up to L wrap to 0


def make_box(box_len: float, n_particles: int, n_halos: int, dtype: str, seed: int,
             device="cpu", halo_frac: float = HALO_FRAC) -> torch.Tensor:
    """Particle positions ``[n_particles, 3]`` (x, y, z) in [0, box_len)."""
    pos, owner, _, _, _, gen = _draw_box(box_len, n_particles, n_halos, seed, device, halo_frac)
    del owner
    out = _finish(pos, box_len, dtype)
    del pos
    perm = torch.randperm(n_particles, generator=gen, device=out.device)
    return out[perm].contiguous()


# Velocity model (for the self-boundness check of steps 9-10).  Units: km/s,
# Mpc/h, M_sun/h.  G in (Mpc/h) (km/s)^2 / (M_sun/h); the box is at the mean
# matter density of a flat universe with Omega_m = 0.3 (rho_crit = 2.775e11 h^2
# M_sun / Mpc^3), which fixes the equal particle mass.
G_MPC_KMS2_MSUN = 6.67430e-11 * 1.98841e30 / 3.0856775814913673e22 / 1.0e6
OMEGA_M = 0.3
RHO_CRIT = 2.775e11
SIGMA_BULK = 300.0       # km/s per axis: each halo's bulk velocity
SIGMA_FIELD = 400.0      # km/s per axis: the uniform background


def particle_mass(box_len: float, n_particles: int) -> float:
    """Equal particle mass (M_sun/h) of a box at the mean matter density."""
    return OMEGA_M * RHO_CRIT * box_len ** 3 / n_particles


def make_phase_box(box_len: float, n_particles: int, n_halos: int, dtype: str, seed: int, device="cpu",
                   halo_frac: float = HALO_FRAC):
    """Positions exactly as ``make_box`` and velocities [n_particles, 3] (km/s),
    in the same order, plus the particle mass (M_sun/h).

    A halo particle moves with its halo's bulk velocity (N(0, 300 km/s) per
    axis) plus an isotropic Gaussian of dispersion V_vir / sqrt(3) per axis,
    V_vir = sqrt(G M m_p / r_vir) (M its particle number); background particles
    draw N(0, 400 km/s) per axis.  The velocities come from a generator of
    their own, so the positions do not depend on whether they are drawn."""
    pos, owner, counts, r_vir, n_in, gen = _draw_box(box_len, n_particles, n_halos, seed, device, halo_frac)
    dev = pos.device
    f64 = torch.float64
    vgen = torch.Generator(device=dev)
    vgen.manual_seed(int(seed) * 1000003 + 17)
    m_p = particle_mass(box_len, n_particles)
    vel = torch.randn((n_particles, 3), generator=vgen, dtype=f64, device=dev) * SIGMA_FIELD
    if n_in > 0:
        bulk = torch.randn((n_halos, 3), generator=vgen, dtype=f64, device=dev) * SIGMA_BULK
        v_vir = torch.sqrt(G_MPC_KMS2_MSUN * counts.to(f64) * m_p / r_vir)
        vel[:n_in] = bulk[owner] + vel[:n_in] / SIGMA_FIELD * (v_vir[owner] / math.sqrt(3.0))[:, None]
    out = _finish(pos, box_len, dtype)
    del pos
    perm = torch.randperm(n_particles, generator=gen, device=dev)
    return out[perm].contiguous(), vel.to(_torch_dtype(dtype))[perm].contiguous(), m_p


def smooth_field(n: int, seed: int, device="cpu", half_width: int = 2, passes: int = 2) -> torch.Tensor:
    """A seeded smooth random FP32 field [n][n][n] with many local maxima, for
    testing maxima and segmentation on their own at any size.

    White noise U[0, 1) is smoothed by ``passes`` periodic moving averages of
    2 ``half_width`` + 1 cells along each axis (about a Gaussian of width
    half_width sqrt(passes) cells), and a weak long-wavelength ripple is added
    so that some ascent paths run across many cells.  This is an input
    generator, not a transform of the method: it only shapes test data."""
    device = torch.device(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f = torch.rand((n, n, n), generator=gen, dtype=torch.float32, device=device)
    for _ in range(passes):
        for axis in range(3):
            acc = f.clone()
            for d in range(1, half_width + 1):
                acc += torch.roll(f, d, axis)
                acc += torch.roll(f, -d, axis)
            f = acc / float(2 * half_width + 1)
            del acc
    g = torch.arange(n, dtype=torch.float32, device=device) * (2.0 * math.pi / n)
    ripple = torch.cos(g)[:, None, None] + torch.cos(2.0 * g)[None, :, None] + torch.cos(g)[None, None, :]
    f += 0.005 * ripple
    return (f - 0.5).contiguous()


def make_config_box(cfg: BoxConfig, device="cpu") -> torch.Tensor:
    return make_box(cfg.box_len, cfg.n_particles, cfg.n_halos, cfg.dtype, cfg.seed, device)


@dataclass(frozen=True)
class JobSpec:
    """One serving request: a periodic subvolume (grid n, side L = n Mpc/h) and a scale.

    The particles of a request come from a resident pool of boxes: ``box_seed``
    names the pool box; several requests may share one box with different scales.
    """

    job_id: int
    n: int
    box_len: float
    n_particles: int
    n_halos: int
    kw: float
    box_seed: int
    dtype: str = "f32"

    def positions(self, device="cpu") -> torch.Tensor:
        return make_box(self.box_len, self.n_particles, self.n_halos, self.dtype, self.box_seed, device)


def job_stream(n_jobs: int = 2000, seed: int = 5, sizes=SERVE_SIZES, boxes_per_size: int = 8) -> list:
    """Serving jobs: n uniform over ``sizes``, N_p = n^3 U[0.5,2], scale U[1,4] cells.

    Each subvolume has dx = 1 Mpc/h (L = n) and the halo number density of the
    1024^3 / 1000 Mpc/h box (1.2e-3 halos per (Mpc/h)^3).  Particle sets come
    from ``boxes_per_size`` pool boxes per grid size (N_p drawn once per box);
    every job draws its own scale.
    """
    gen = torch.Generator()
    gen.manual_seed(int(seed))
    pool = {}
    for n in sizes:
        for k in range(boxes_per_size):
            frac = 0.5 + 1.5 * float(torch.rand(1, generator=gen, dtype=torch.float64).item())
            pool[(n, k)] = (int(round(n ** 3 * frac)), 5_000_000 + 1000 * n + k)
    jobs = []
    for j in range(n_jobs):
        n = sizes[int(torch.randint(len(sizes), (1,), generator=gen).item())]
        k = int(torch.randint(boxes_per_size, (1,), generator=gen).item())
        a = 1.0 + 3.0 * float(torch.rand(1, generator=gen, dtype=torch.float64).item())
        np_, box_seed = pool[(n, k)]
        box_len = float(n)
        jobs.append(JobSpec(j, n, box_len, np_, int(round(1.2e-3 * box_len ** 3)), n / (1000.0 * a), box_seed))
    return jobs


def poisson_arrivals(n_jobs: int, rate_per_s: float, seed: int = 5) -> list:
    """Arrival times (s) of a Poisson process with the given rate."""
    gen = torch.Generator()
    gen.manual_seed(int(seed) + 1)
    gaps = -torch.log1p(-torch.rand(n_jobs, generator=gen, dtype=torch.float64)) / rate_per_s
    return torch.cumsum(gaps, 0).tolist()
