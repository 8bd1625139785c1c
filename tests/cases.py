"""Builds the same seeded case on the HIP library and on the oracle.

A case is a plain dict of commands (lattice size, fluids, forces, obstacles,
initial fields, solute, reaction).  ``build_oracle`` and ``build_gpu`` apply
it to each side; both take their inputs from the same arrays, and no value
ever flows from the GPU side into the oracle.
"""
from __future__ import annotations

import numpy as np

from oracle import Oracle


def poiseuille_case(nx=128, ny=64, accel=1e-6, tau=1.0):
    return dict(nx=nx, ny=ny, tau=tau, accel=[(1, accel, 0)],
                rects=[(0, nx - 1, 0, 0), (0, nx - 1, ny - 1, ny - 1)])


def porous_case(nx, ny, seed, tau=0.8, accel=1e-5, nd=None, rmin=2.0, rmax=6.0, noise=0.02):
    rng = np.random.default_rng(seed)
    nd = nd if nd is not None else max(1, nx * ny // 300)
    circles = [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), float(rng.uniform(rmin, rmax)))
               for _ in range(nd)]
    n = nx * ny
    rho = 1.0 + noise * rng.uniform(-1, 1, n)
    ux = noise * 0.5 * rng.uniform(-1, 1, n)
    uy = noise * 0.5 * rng.uniform(-1, 1, n)
    return dict(nx=nx, ny=ny, tau=tau, accel=[(1, accel, 0)], circles=circles,
                fields={0: (rho, ux, uy)})


def sc_solute_case(nx, ny, seed, react=True, kr=0.01, bmax=0.2, G=0.9, gads=(0.3, -0.3),
                   openings=True, tau_s=0.7, nd=None, C0=0.05, b0=0.0, q=9):
    rng = np.random.default_rng(seed)
    nd = nd if nd is not None else max(2, nx * ny // 500)
    circles = []
    for _ in range(nd):
        r = float(rng.uniform(2.0, 5.0))
        xc = int(rng.integers(int(r) + 3, nx - int(r) - 3))
        circles.append((xc, int(rng.integers(0, ny)), r))
    n = nx * ny
    blob = rng.uniform(0, 1, n) < 0.3
    rho_a = np.where(blob, 1.0, 0.05) * (1 + 0.01 * rng.uniform(-1, 1, n))
    rho_b = np.where(blob, 0.05, 1.0) * (1 + 0.01 * rng.uniform(-1, 1, n))
    case = dict(nx=nx, ny=ny, tau=1.0, fluids=(1.0, 1.0), G=G, gads=gads, circles=circles,
                fields={0: (rho_a, None, None), 1: (rho_b, None, None)},
                solute=tau_s, q=q, C=np.full(n, C0), accel=[(1, 1e-5, 0)])
    if openings:
        case["openings"] = [("xlo", "dirichlet", 1.0), ("xhi", "adiabatic", 0.0)]
    if react:
        case["reaction"] = (kr, 0.0, b0, bmax, 4242 + seed)
    return case


def surface_growth_case(kr, n=200, side=11, f0=24.0, C0=1.5, Cs=0.5, b0=0.5, bmax=1.0, tau=1.0,
                        tau_s=1.0, q=4, seed=2012):
    """The paper's surface-growth example (section Surface growth and its
    script): an n x n periodic box, one fluid at rest of density f0, a
    side x side solid seed square in the centre, D2Q4 solute C0, reaction
    kr / Cs / b0 / bmax.  The fluid starts at its equilibrium (rho = f0)."""
    h = side // 2
    c = n // 2
    return dict(nx=n, ny=n, tau=tau, rects=[(c - h, c + h, c - h, c + h)],
                fields={0: (np.full(n * n, f0), None, None)}, solute=tau_s, q=q,
                C=np.full(n * n, C0), reaction=(kr, Cs, b0, bmax, seed))


def phase_case(nx, ny, seed, G=-120.0, psi0=4.0, rho0=200.0, d0=200.0, tau=1.0):
    """The paper's phase-separation set-up (section Phase separation): one
    fluid, density d0 + U[0, 1] at rest, interforce(G, psi0, rho0)."""
    rng = np.random.default_rng(seed)
    return dict(nx=nx, ny=ny, tau=tau, psi=(G, psi0, rho0),
                fields={0: (d0 + rng.uniform(0, 1, nx * ny), None, None)})


def contact_box_case(Gads, nx=201, ny=51, seed=5, G=-120.0, psi0=4.0, rho0=200.0):
    """The paper's contact-angle box (section Contact angles I): solid
    frame, fluid inside as in the phase-separation set-up, interforce and
    the one-component adhesiveforce(Gads, psi0, rho0)."""
    case = phase_case(nx, ny, seed, G, psi0, rho0)
    case["rects"] = [(0, 0, 0, ny - 1), (nx - 1, nx - 1, 0, ny - 1), (0, nx - 1, 0, 0), (0, nx - 1, ny - 1, ny - 1)]
    case["ads_psi"] = (Gads, psi0, rho0)
    return case


def two_fluid_contact_case(g1=0.2, g2=-0.2, Nx=200, Ny=50, base=51):
    """The paper's contact-angles II set-up (section Contact angles II and its
    script): a box of (Nx+1) x (Ny+1) nodes with solid walls on all four
    sides, fluid 1 dense (2) and fluid 2 dilute (0.1) inside a centred
    rectangle of the given base spanning the box height, the reverse
    elsewhere, G = 0.9, adhesion g1 (fluid 1) and g2 (fluid 2), tau = 1.
    The script's initial state holds each density in the rest population;
    here the nodes start at their equilibrium at rest (same densities)."""
    nx, ny = Nx + 1, Ny + 1
    x = np.tile(np.arange(nx), ny)
    inside = (x >= Nx // 2 - base // 2) & (x <= Nx // 2 + base // 2)
    rho1 = np.where(inside, 2.0, 0.1)
    rho2 = np.where(inside, 0.1, 2.0)
    rects = [(0, nx - 1, 0, 0), (0, nx - 1, ny - 1, ny - 1), (0, 0, 0, ny - 1), (nx - 1, nx - 1, 0, ny - 1)]
    return dict(nx=nx, ny=ny, tau=1.0, fluids=(1.0, 1.0), G=0.9, gads=(g1, g2), rects=rects,
                fields={0: (rho1, None, None), 1: (rho2, None, None)})


def parallel_droplet_case(Nx=350, Ny=200, L=64):
    """The paper's parallelization example (section Parallelization and its
    script; the workload generator states it).  The nodes start at their
    equilibrium at rest."""
    from paper_1202_0442_amd import inputs
    w = inputs.parallel_droplet(Nx, Ny, L)
    e = w.extra
    return dict(nx=w.nx, ny=w.ny, tau=w.tau, fluids=(w.tau, e["tau2"]), G=e["G"], gads=e["Gads"], rects=w.rects,
                fields={0: (e["rho"][0], None, None), 1: (e["rho"][1], None, None)})


def flat_coexistence(G, ny=96, steps=20000):
    """Bulk densities (major, minor) of a converged flat two-component
    Shan-Chen interface on the oracle: a slab of A across a periodic
    4 x ny strip, both tau = 1."""
    nx = 4
    yy = np.repeat(np.arange(ny), nx)
    slab = (yy >= ny // 4) & (yy < 3 * ny // 4)
    o = Oracle(nx, ny)
    o.fluids(2, 1.0, 1.0)
    o.interforce(G)
    o.set_fields(0, np.where(slab, 1.0, 0.05))
    o.set_fields(1, np.where(slab, 0.05, 1.0))
    o.iteration(steps)
    ra, _, _ = o.moments(0)
    return float(ra[ny // 2, 0]), float(ra[0, 0])


def droplet_fields(n, R, hi, lo):
    """(rho_A, rho_B) of a droplet of A of radius R at the centre of an
    n x n box: A-rich bulk densities (hi, lo) inside, (lo, hi) outside."""
    yy, xx = np.mgrid[0:n, 0:n]
    inside = ((xx - n / 2) ** 2 + (yy - n / 2) ** 2 < R * R).ravel()
    return np.where(inside, hi, lo), np.where(inside, lo, hi)


def laplace_jump(ra, rb, G):
    """Equivalent radius from the A-rich area and the pressure jump, with
    p = (rho_A + rho_B + G rho_A rho_B)/3, between the box centre and its
    corner."""
    n = ra.shape[0]
    p = (ra + rb + G * ra * rb) / 3
    return float(np.sqrt((ra > rb).sum() / np.pi)), float(p[n // 2, n // 2] - p[0, 0])


def channel_flow_case(nx, ny, seed, wall="xlo", inlet=("poiseuille", 0.04, 1.0),
                      outlet=("dirichlet", 0.0, 1.0), nd=4, tau=0.8):
    """Through-flow channel: solid side walls, an inlet on `wall` and an
    outlet on the opposite wall (inlet_momentum / outlet_momentum styles),
    a few random discs inside."""
    rng = np.random.default_rng(seed)
    opp = {"xlo": "xhi", "xhi": "xlo", "ylo": "yhi", "yhi": "ylo"}[wall]
    if wall in ("xlo", "xhi"):
        rects = [(0, nx - 1, 0, 0), (0, nx - 1, ny - 1, ny - 1)]
        lo, hi = 1, ny - 2
    else:
        rects = [(0, 0, 0, ny - 1), (nx - 1, nx - 1, 0, ny - 1)]
        lo, hi = 1, nx - 2
    circles = [(int(rng.integers(nx // 4, 3 * nx // 4)), int(rng.integers(ny // 4, 3 * ny // 4)),
                float(rng.uniform(1.5, 3.5))) for _ in range(nd)]
    mopen = [(wall, lo, hi, 0, "inlet", *inlet), (opp, lo, hi, 0, "outlet", *outlet)]
    return dict(nx=nx, ny=ny, tau=tau, rects=rects, circles=circles, mopen=mopen)


def _ordered_obstacles(side, case):
    """The case's "obstacles": (kind, args, styles) in order, after the
    rectangles and circles; styles = [(comp, style, R), ...] (hybrid
    boundary style) or None."""
    for kind, args, styles in case.get("obstacles", []):
        for comp, style, R in styles or []:
            side.obstacle_style(comp, style, R)
        if kind == "rect":
            side.obstacle_rect(*args)
        else:
            side.obstacle_circle(*args)


def slip_box_case(nx, ny, seed, style=("hybrid", 0.0), two=True, G=None, accel=1e-4, nob=10):
    """Periodic box with random rectangles and discs under a boundary style;
    under the hybrid style each obstacle draws its own style per component
    (noslip, slip or mixed with a random share).  One or two fluids with a
    random start and a body force along x."""
    rng = np.random.default_rng(seed)
    obstacles = []
    for k in range(nob):
        styles = None
        if style[0] == "hybrid":
            styles = [(0, ("noslip", "slip", "mixed")[k % 3], float(rng.uniform(0, 1)))]
            if two:
                styles.append((1, ("slip", "mixed", "noslip")[k % 3], float(rng.uniform(0, 1))))
        if k % 2:
            obstacles.append(("circle", (int(rng.integers(0, nx)), int(rng.integers(0, ny)),
                                         float(rng.uniform(1.5, 4.5))), styles))
        else:
            x0, y0 = int(rng.integers(0, nx - 7)), int(rng.integers(0, ny - 7))
            obstacles.append(("rect", (x0, x0 + int(rng.integers(0, 6)), y0, y0 + int(rng.integers(0, 6))), styles))
    n = nx * ny
    fields = {0: (0.6 + 0.1 * rng.uniform(0, 1, n), 0.02 * rng.uniform(-1, 1, n), 0.02 * rng.uniform(-1, 1, n))}
    case = dict(nx=nx, ny=ny, tau=0.8, style=style, obstacles=obstacles, fields=fields, accel=[(1, accel, 0)])
    if two:
        fields[1] = (0.4 + 0.1 * rng.uniform(0, 1, n), 0.02 * rng.uniform(-1, 1, n), 0.02 * rng.uniform(-1, 1, n))
        case["fluids"] = (0.8, 1.1)
        if G is not None:
            case["G"] = G
    return case


def intersolute_case(nx, ny, seed, q=4, tau_s=1.0, isol=(-5e-3, 1.0, 5e-3), C0=5e-3, noise=0.1, nd=0):
    """The paper's intersolute example (G = -5e-3, psi0 = 1, C0 = 5e-3):
    one fluid at rest, solute of mean C0 with a uniform random noise of
    relative size `noise`, optionally a few discs."""
    rng = np.random.default_rng(seed)
    circles = [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), float(rng.uniform(1.5, 4.0))) for _ in range(nd)]
    n = nx * ny
    return dict(nx=nx, ny=ny, tau=1.0, circles=circles, solute=tau_s, q=q, isol=isol,
                C=C0 * (1 + noise * rng.uniform(-1, 1, n)))


def build_oracle(case):
    o = Oracle(case["nx"], case["ny"])
    if "fluids" in case:
        o.fluids(2, *case["fluids"])
    else:
        o.fluids(1, case["tau"])
    for mode, v, comp in case.get("force", []):
        o.aveforce(mode, v, comp)
    for mode, v, comp in case.get("accel", []):
        o.aveacceleration(mode, v, comp)
    if case.get("G") is not None:
        o.interforce(case["G"])
    if case.get("gads") is not None:
        o.adhesiveforce(case["gads"][0], 0)
        o.adhesiveforce(case["gads"][1], 1)
    if case.get("psi") is not None:
        o.interforce(*case["psi"])
    if case.get("ads_psi") is not None:
        G, psi0, rho0 = case["ads_psi"]
        o.adhesiveforce(G, psi0=psi0, rho0=rho0)
    o.boundary_style(*case.get("style", ("noslip", 0.0)))
    for r in case.get("rects", []):
        o.obstacle_rect(*r)
    for c in case.get("circles", []):
        o.obstacle_circle(*c)
    _ordered_obstacles(o, case)
    for op in case.get("mopen", []):
        o.momentum_opening(*op)
    if case.get("mask") is not None:
        o.set_mask(np.maximum(o.get_mask(), case["mask"]))
    for comp, (rho, ux, uy) in case.get("fields", {}).items():
        o.set_fields(comp, rho, 0.0 if ux is None else ux, 0.0 if uy is None else uy)
    if "fluids" in case:
        for comp in (0, 1):
            if comp not in case.get("fields", {}):
                o.set_fields(comp, 1.0)
    elif 0 not in case.get("fields", {}):
        o.set_fields(0, 1.0)
    if case.get("solute") is not None:
        o.solute(case["solute"], case.get("q", 9))
        for wall, style, val in case.get("openings", []):
            o.solute_opening(wall, style, val)
        for op in case.get("sopen", []):
            o.solute_opening_range(*op)
        if case.get("reaction") is not None:
            o.surface_reaction(*case["reaction"])
        if case.get("isol") is not None:
            o.intersolute(*case["isol"])
        o.set_concentration(case.get("C", 0.0))
    return o


def build_gpu(case, storage="f32", bind=True, stream=None):
    from paper_1202_0442_amd import lb2d
    g = lb2d.Lattice(0)
    g.lattice("d2q9", case["nx"], case["ny"], case["tau"])
    if "fluids" in case:
        g.fluids(*case["fluids"])
    if case.get("solute") is not None:
        g.solute(case["solute"], case.get("q", 9))
        for wall, style, val in case.get("openings", []):
            g.solute_opening(wall, style, val)
        for op in case.get("sopen", []):
            g.solute_opening_range(*op)
        if case.get("isol") is not None:
            g.intersolute(*case["isol"])
    g.boundary_style(*case.get("style", ("noslip", 0.0)))
    for r in case.get("rects", []):
        g.obstacle_rect(*r)
    for c in case.get("circles", []):
        g.obstacle_circle(*c)
    _ordered_obstacles(g, case)
    for op in case.get("mopen", []):
        g.momentum_opening(*op)
    if case.get("mask") is not None:
        g.obstacle_mask(case["mask"])
    if case.get("reaction") is not None:
        kr, Cs, b0, bmax, seed = case["reaction"]
        g.surface_reaction(kr, Cs, "growth", b0, bmax, seed)
    for comp, (rho, ux, uy) in case.get("fields", {}).items():
        g.set_fields(comp, rho, ux, uy)
    if case.get("solute") is not None:
        g.set_concentration(case.get("C", np.zeros(case["nx"] * case["ny"])))
    for mode, v, comp in case.get("force", []):
        g.aveforce(mode, v, comp)
    for mode, v, comp in case.get("accel", []):
        g.aveacceleration(mode, v, comp)
    if case.get("G") is not None:
        g.interforce(case["G"])
    if case.get("gads") is not None:
        g.adhesiveforce(case["gads"][0], 0)
        g.adhesiveforce(case["gads"][1], 1)
    if case.get("psi") is not None:
        g.interforce(*case["psi"])
    if case.get("ads_psi") is not None:
        G, psi0, rho0 = case["ads_psi"]
        g.adhesiveforce(G, 0, psi0, rho0)
    if bind:
        g.bind(storage, stream=stream)
    return g


def rel_err(a, b, scale=None):
    scale = np.abs(b).max() if scale is None else scale
    return float(np.abs(a - b).max() / max(scale, 1e-300))
