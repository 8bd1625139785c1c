"""Slip, mixed and hybrid boundary styles (boundary_style command, Fig.
slip; per-obstacle styles of the obstacle command) on the GPU, through the
C ABI, against the FP64 oracle.  Bars: masks bit-identical, FP64 within
1e-12 relative, FP32 within 1e-5 (velocities of the Shan-Chen case within
the FP32 bound derived for the cohesion force, 1e-4: the force is a
difference of neighbouring densities).
"""
import numpy as np
import pytest

from cases import (build_gpu, build_oracle, channel_flow_case, poiseuille_case, porous_case, rel_err,
                   sc_solute_case, slip_box_case)

pytestmark = pytest.mark.gpu


def _cmp(g, o, ncomp, tol_rho, tol_u):
    for c in range(ncomp):
        gr, gx, gy = g.moments(c)
        orr, ox, oy = o.moments(c)
        solid = o.get_mask().astype(bool)
        er = rel_err(gr[~solid], orr[~solid])
        us = max(np.abs(ox).max(), np.abs(oy).max())   # one scale for both velocity components
        eu = max(rel_err(gx, ox, us), rel_err(gy, oy, us))
        print(f"comp {c}: rel rho err {er:.3e}, rel u err {eu:.3e}")
        assert er <= tol_rho and eu <= tol_u


@pytest.mark.parametrize("wall", ["horizontal", "vertical"])
@pytest.mark.parametrize("style,R", [("noslip", 0.0), ("slip", 1.0), ("mixed", 0.3)])
def test_lone_diagonal_mode_matches_oracle(wall, style, R):
    """One unit of f5 next to a flat wall: every population after one step
    equals the oracle's (the forward share lands two nodes along the
    wall, the rest bounces back)."""
    nx, ny = 12, 12
    rect = (0, nx - 1, 6, 6) if wall == "horizontal" else (4, 4, 0, ny - 1)
    case = dict(nx=nx, ny=ny, tau=1.0, style=(style, R), rects=[rect])
    o, g = build_oracle(case), build_gpu(case, "f64")
    f = o.get_f(0)
    f[5, 5, 3] += 1.0
    o.set_f(f, 0)
    g.set_populations(f, 0)
    o.iteration(1)
    g.iteration(1)
    assert np.abs(g.get_populations(0) - o.get_f(0)).max() <= 1e-14


# FP32 velocity bound of a uniformly forced run: every node of the (nearly)
# plug flow rounds the same way, so the half-ulp rounding of the forcing
# increment adds up linearly instead of averaging out; the velocity grows
# linearly too, so after N steps the relative error is about N 2^-24
# (2.4e-5 for 400 steps).  Densities keep the 1e-5 bar.
@pytest.mark.parametrize("storage,tol_rho,tol_u", [("f64", 1e-12, 1e-12), ("f32", 1e-5, 400 * 2.0 ** -24)])
@pytest.mark.parametrize("style", [("slip", 1.0), ("mixed", 0.35)])
def test_forced_channel_matches_oracle(storage, tol_rho, tol_u, style):
    case = poiseuille_case(nx=40, ny=37, accel=1e-5, tau=0.9)
    case["style"] = style
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(400)
    g.iteration(400)
    _cmp(g, o, 1, tol_rho, tol_u)
    if style[0] == "slip":
        _, ux, _ = g.moments(0)
        assert np.ptp(ux[1:-1]) <= (1e-15 if storage == "f64" else 1e-6) * 400


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_porous_mixed_ragged_matches_oracle(storage, tol):
    """Random discs (corners of every kind) on a ragged lattice (neither
    size a multiple of the tile), mixed style."""
    case = porous_case(133, 75, 17, nd=30)
    case["style"] = ("mixed", 0.6)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(150)
    g.iteration(150)
    _cmp(g, o, 1, tol, tol)


@pytest.mark.parametrize("storage,tol_rho,tol_u", [("f64", 1e-12, 1e-12), ("f32", 1e-5, 1e-5)])
def test_hybrid_two_fluids_matches_oracle(storage, tol_rho, tol_u):
    """Hybrid style: each obstacle has its own style per component."""
    case = slip_box_case(70, 45, 3, nob=14)
    o, g = build_oracle(case), build_gpu(case, storage)
    b0 = g.budgets()
    o.iteration(120)
    g.iteration(120)
    _cmp(g, o, 2, tol_rho, tol_u)
    b1 = g.budgets()
    for c in (0, 1):
        assert b1[f"mass{c}"] == pytest.approx(b0[f"mass{c}"], rel=1e-11 if storage == "f64" else 1e-5)


@pytest.mark.parametrize("storage,tol_rho,tol_u", [("f64", 1e-12, 1e-11), ("f32", 1e-5, 1e-4)])
def test_hybrid_shan_chen_matches_oracle(storage, tol_rho, tol_u):
    """Hybrid style with the two-component cohesion force (density tile
    with its halo next to slip and mixed solids)."""
    case = slip_box_case(66, 40, 9, G=0.9, nob=12)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(80)
    g.iteration(80)
    _cmp(g, o, 2, tol_rho, tol_u)


def test_growth_under_mixed_style_matches_oracle():
    """Solids made by growth take the style's share: masks identical and
    fields within the FP64 bar after growth next to mixed walls."""
    case = sc_solute_case(96, 64, 29, react=True, kr=0.02)
    case["style"] = ("mixed", 0.4)
    o, g = build_oracle(case), build_gpu(case, "f64")
    for chunk in (60, 140):
        o.iteration(chunk)
        g.iteration(chunk)
        assert np.array_equal(g.mask(), o.get_mask()), f"mask differs after {o.t} steps"
    assert o.budgets()["grown_nodes"] > 3
    _cmp(g, o, 2, 1e-11, 1e-11)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1.2e-4)])
def test_slip_walls_with_momentum_openings(storage, tol):
    """Zou-He inlet and outlet between full-slip side walls (FP32 velocity
    bound of the openings, c_s 1e-5 / u_max)."""
    case = channel_flow_case(60, 31, 4, inlet=("uniform", 0.04, 1.0))
    case["style"] = ("slip", 1.0)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(300)
    g.iteration(300)
    _cmp(g, o, 1, tol, tol)
