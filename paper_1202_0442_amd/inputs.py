"""Seeded synthetic workloads (geometry lists, initial fields, run parameters).

This module is the only code shared by the HIP path's tests/benchmark and the
oracle's tests.  It holds none of the lattice Boltzmann arithmetic: it draws
disc lists and initial density maps from a seed and returns plain Python /
NumPy data.  Each side rasterises obstacles and builds populations itself.

Workloads (node counts, x fastest):

* ``poiseuille``  -- 128x64 channel, solid rows y=0 and y=ny-1, periodic in x,
  tau=1, rho0=1, acceleration 1e-6 along e1 (the paper's Poiseuille
  application on a 128x64 channel).
* ``porous``      -- square lattice with non-overlapping discs, radius uniform
  in [8,24], random sequential addition with a minimum gap of one node on the
  periodic box until the disc area reaches 40 % (porosity 0.6), tau=0.8,
  acceleration 1e-5 along e1.
* ``sc_solute``   -- two-component Shan-Chen plus solute: discs radius
  [10,30] to porosity 0.7 kept two radii from the x walls, A-rich blobs of
  radius [8,32] covering ~30 % of the fluid, G=0.9, G_ads=+0.3 (A) / -0.3 (B),
  D2Q9 solute tau_s=0.7, Dirichlet C=1 at xlo, adiabatic xhi, reaction
  k_r=1e-3, C_s=0, b0=0, b_max=1.
* ``ensemble``    -- many independent porous lattices with log-uniform sides,
  overlapping (Boolean) discs of radius [4,20], porosity U[0.4,0.8],
  tau U[0.6,1.2], acceleration 1e-5.
* ``phase_separation``, ``surface_growth``, ``parallel_droplet`` -- the
  paper's own examples (phase separation, surface growth, the droplet of its
  parallelization section), with their printed parameters.

The paper uses no public dataset; these generators stand in for its
hand-built geometries (channel, random porous media, droplets).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

Disc = Tuple[int, int, float]  # (xc, yc, r)


def rsa_discs(nx: int, ny: int, rmin: float, rmax: float, solid_fraction: float,
              seed: int, gap: int = 1, x_margin: float | None = None,
              max_tries: int = 5_000_000) -> List[Disc]:
    """Random sequential addition of non-overlapping discs.

    Centres are integers, radii uniform in [rmin, rmax].  Two discs must be
    at least r1 + r2 + gap apart (minimum image on the periodic box).  Stops
    when the summed disc area pi r^2 reaches ``solid_fraction * nx * ny``.
    ``x_margin`` (if given) keeps every centre at least r + x_margin away
    from the columns x = 0 and x = nx - 1 (no wrap in x then).
    """
    rng = np.random.default_rng(seed)
    target = solid_fraction * nx * ny
    cell = 2.0 * rmax + gap
    gx, gy = max(1, int(nx // cell)), max(1, int(ny // cell))
    cw, ch = nx / gx, ny / gy
    grid: dict = {}
    discs: List[Disc] = []
    area = 0.0
    tries = 0
    batch = 4096
    while area < target and tries < max_tries:
        rs = rng.uniform(rmin, rmax, batch)
        xs = rng.integers(0, nx, batch)
        ys = rng.integers(0, ny, batch)
        for r, xc, yc in zip(rs.tolist(), xs.tolist(), ys.tolist()):
            tries += 1
            if x_margin is not None and (xc < r + x_margin or xc > nx - 1 - r - x_margin):
                continue
            ci, cj = int(xc / cw) % gx, int(yc / ch) % gy
            ok = True
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    for (ox, oy, orr) in grid.get(((ci + di) % gx, (cj + dj) % gy), ()):
                        dx = abs(xc - ox)
                        dx = min(dx, nx - dx)
                        dy = abs(yc - oy)
                        dy = min(dy, ny - dy)
                        lim = r + orr + gap
                        if dx * dx + dy * dy < lim * lim:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                continue
            d = (int(xc), int(yc), float(r))
            discs.append(d)
            grid.setdefault((ci, cj), []).append(d)
            area += math.pi * r * r
            if area >= target:
                break
    if area < target:
        raise RuntimeError("disc packing jammed before reaching the target solid fraction")
    return discs


def boolean_discs(nx: int, ny: int, rmin: float, rmax: float, solid_fraction: float,
                  seed: int) -> List[Disc]:
    """Overlapping (Boolean-model) discs: uniform centres and radii, added
    until the expected covered fraction 1 - exp(-sum(pi r^2) / A) reaches
    ``solid_fraction``."""
    rng = np.random.default_rng(seed)
    need = -math.log(1.0 - solid_fraction) * nx * ny
    discs: List[Disc] = []
    area = 0.0
    while area < need:
        r = float(rng.uniform(rmin, rmax))
        xc = int(rng.integers(0, nx))
        yc = int(rng.integers(0, ny))
        discs.append((xc, yc, r))
        area += math.pi * r * r
    return discs


def blob_map(nx: int, ny: int, blobs: List[Disc]) -> np.ndarray:
    """Boolean map of the nodes strictly inside any blob (minimum image on
    the periodic box).  Used only to build initial densities."""
    inside = np.zeros((ny, nx), dtype=bool)
    xs = np.arange(nx)
    ys = np.arange(ny)
    for xc, yc, r in blobs:
        dx = np.abs(xs - xc)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(ys - yc)
        dy = np.minimum(dy, ny - dy)
        rr = int(math.ceil(r))
        rows = np.nonzero(dy <= rr)[0]
        cols = np.nonzero(dx <= rr)[0]
        sub = dy[rows][:, None] ** 2 + dx[cols][None, :] ** 2 < r * r
        inside[np.ix_(rows, cols)] |= sub
    return inside


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    steps: int
    tau: float = 1.0
    accel_x: float = 0.0
    rho0: float = 1.0
    discs: List[Disc] = field(default_factory=list)
    rects: List[Tuple[int, int, int, int]] = field(default_factory=list)
    extra: dict = field(default_factory=dict)


def poiseuille(nx: int = 128, ny: int = 64, accel: float = 1e-6, tau: float = 1.0,
               steps: int = 5000) -> Workload:
    """Force-driven channel: solid rows y=0 and y=ny-1, periodic in x."""
    return Workload("poiseuille", nx, ny, steps, tau=tau, accel_x=accel,
                    rects=[(0, nx - 1, 0, 0), (0, nx - 1, ny - 1, ny - 1)])


def porous(n: int = 4096, seed: int = 2, porosity: float = 0.6, rmin: float = 8.0,
           rmax: float = 24.0, tau: float = 0.8, accel: float = 1e-5,
           steps: int = 10000, ny: int | None = None) -> Workload:
    """Single-fluid flow through non-overlapping discs on a periodic box."""
    ny = n if ny is None else ny
    discs = rsa_discs(n, ny, rmin, rmax, 1.0 - porosity, seed)
    return Workload("porous", n, ny, steps, tau=tau, accel_x=accel, discs=discs)


def sc_solute(n: int = 2048, seed: int = 3, blob_seed: int = 33, rng_seed: int = 333,
              steps: int = 20000, porosity: float = 0.7, kr: float = 1e-3,
              rmin: float = 10.0, rmax: float = 30.0, blob_rmin: float = 8.0,
              blob_rmax: float = 32.0, ny: int | None = None) -> Workload:
    """Two-component Shan-Chen + D2Q9 solute with surface growth."""
    ny = n if ny is None else ny
    discs = rsa_discs(n, ny, rmin, rmax, 1.0 - porosity, seed, x_margin=2.0)
    fluid_area = porosity * n * ny
    rng = np.random.default_rng(blob_seed)
    blobs: List[Disc] = []
    cover = 0.0
    while 1.0 - math.exp(-cover / fluid_area) < 0.3:
        r = float(rng.uniform(blob_rmin, blob_rmax))
        blobs.append((int(rng.integers(0, n)), int(rng.integers(0, ny)), r))
        cover += math.pi * r * r
    extra = dict(G=0.9, Gads=(0.3, -0.3), tau2=1.0, rho_major=1.0, rho_minor=0.05,
                 blobs=blobs, tau_s=0.7, C_in=1.0, kr=kr, Cs=0.0, b0=0.0, bmax=1.0,
                 rng_seed=rng_seed)
    return Workload("sc_solute", n, ny, steps, tau=1.0, discs=discs, extra=extra)


def sc_initial_fields(w: Workload):
    """Initial (rho_A, rho_B) maps of the two-component workload."""
    inside = blob_map(w.nx, w.ny, w.extra["blobs"])
    hi, lo = w.extra["rho_major"], w.extra["rho_minor"]
    rho_a = np.where(inside, hi, lo).astype(np.float64)
    rho_b = np.where(inside, lo, hi).astype(np.float64)
    return rho_a, rho_b


def ensemble(count: int = 256, seed: int = 5, smin: int = 256, smax: int = 1536,
             steps: int = 5000) -> List[Workload]:
    """Independent porous lattices of uneven size and parameters."""
    rng = np.random.default_rng(seed)
    out = []
    lo, hi = math.log(smin), math.log(smax)
    for k in range(count):
        nx = int(round(math.exp(rng.uniform(lo, hi))))
        ny = int(round(math.exp(rng.uniform(lo, hi))))
        phi = float(rng.uniform(0.4, 0.8))
        tau = float(rng.uniform(0.6, 1.2))
        sub = int(rng.integers(0, 2**31 - 1))
        discs = boolean_discs(nx, ny, 4.0, 20.0, 1.0 - phi, sub)
        out.append(Workload(f"ensemble{k}", nx, ny, steps, tau=tau, accel_x=1e-5,
                            discs=discs, extra=dict(porosity_target=phi)))
    return out


def phase_separation(n: int = 100, seed: int = 1202, d0: float = 200.0, G: float = -120.0,
                     psi0: float = 4.0, rho0: float = 200.0, steps: int = 20000) -> Workload:
    """The paper's phase-separation set-up (section Phase separation): one
    fluid in a periodic n x n box at rest with density d0 + U[0, 1],
    interforce(G, psi0, rho0), tau = 1.  The initial densities are in
    extra["rho"]."""
    rng = np.random.default_rng(seed)
    return Workload("phase", n, n, steps, tau=1.0, rho0=d0,
                    extra={"G": G, "psi0": psi0, "rho0": rho0, "rho": d0 + rng.uniform(0.0, 1.0, n * n)})


def surface_growth(kr: float, n: int = 200, side: int = 11, f0: float = 24.0, C0: float = 1.5,
                   Cs: float = 0.5, b0: float = 0.5, bmax: float = 1.0, seed: int = 2012,
                   steps: int = 20000) -> Workload:
    """The paper's surface-growth set-up (section Surface growth): periodic
    n x n box, one fluid at rest of density f0, a side x side solid seed in
    the centre, D2Q4 solute C0, surface_reaction(kr, Cs, growth, b0, bmax),
    tau = tau_s = 1; Da = kr L / D with L = n and D = (tau_s - 1/2)/2."""
    h, c = side // 2, n // 2
    return Workload("surface_growth", n, n, steps, tau=1.0, rho0=f0,
                    rects=[(c - h, c + h, c - h, c + h)],
                    extra={"kr": kr, "Cs": Cs, "b0": b0, "bmax": bmax, "C0": C0, "tau_s": 1.0,
                           "rng_seed": seed, "Da": kr * n / 0.25})


def parallel_droplet(Nx: int = 350, Ny: int = 200, L: int = 64, steps: int = 500) -> Workload:
    """The paper's parallelization example (section Parallelization):
    (Nx+1) x (Ny+1) nodes, the bottom row solid, periodic otherwise, two
    components with tau = 1; fluid 1 dense (2) and fluid 2 dilute (0.1) in
    the square x in [Nx/2-L, Nx/2+L], y in [0, 2L] on the wall, the reverse
    elsewhere; interforce G = 0.9, adhesion +0.3 (fluid 1) and -0.3
    (fluid 2).  The paper times 500 steps of it.  The initial densities of
    the two components are in extra["rho"]."""
    nx, ny = Nx + 1, Ny + 1
    x = np.tile(np.arange(nx), ny)
    y = np.repeat(np.arange(ny), nx)
    inside = (x >= Nx // 2 - L) & (x <= Nx // 2 + L) & (y <= 2 * L)
    rho = (np.where(inside, 2.0, 0.1), np.where(inside, 0.1, 2.0))
    return Workload("parallel_droplet", nx, ny, steps, tau=1.0, rects=[(0, nx - 1, 0, 0)],
                    extra={"G": 0.9, "Gads": (0.3, -0.3), "tau2": 1.0, "rho": rho})


def random_populations(shape, seed: int, scale: float = 0.01) -> np.ndarray:
    """Deviations uniform in [-scale, scale] for tests that start away from
    equilibrium."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=shape)
