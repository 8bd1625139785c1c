"""Degenerate lattices on the GPU against the oracle: a lattice with no
fluid node, and lattices smaller than one tile in which every stencil (the
Shan-Chen density ring, the slip mask ring, the intersolute ring) wraps
onto itself several times."""
import numpy as np
import pytest

from cases import build_gpu, build_oracle, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("general", [False, True])
def test_lattice_without_fluid(general):
    nx, ny = 37, 11
    case = dict(nx=nx, ny=ny, tau=0.8, rects=[(0, nx - 1, 0, ny - 1)], accel=[(1, 1e-5, 0)])
    if general:
        case.update(fluids=(1.0, 1.0), G=0.9, solute=0.8, q=9, C=np.zeros(nx * ny),
                    reaction=(0.01, 0.0, 0.0, 0.2, 3))
    o, g = build_oracle(case), build_gpu(case, "f32")
    o.iteration(25)
    g.iteration(25)
    assert np.array_equal(g.mask(), o.get_mask())
    rho, ux, uy = g.moments(0)
    assert np.all(rho == -11.0) and np.all(ux == 0.0) and np.all(uy == 0.0)
    b = g.budgets()
    assert b["fluid_nodes"] == 0 and b["mass0"] == 0.0 and b["grown_nodes"] == 0


@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4), (3, 7)])
def test_tiny_two_fluid_solute_lattice_fp64(nx, ny):
    """Two fluids with cohesion and adhesion, a D2Q9 solute: a lattice far
    smaller than the 32 x 8 tile, so every ring node is a periodic image."""
    rng = np.random.default_rng(nx * 10 + ny)
    n = nx * ny
    m = np.zeros((ny, nx), np.uint8)
    m[0, 0] = 1
    case = dict(nx=nx, ny=ny, tau=1.0, fluids=(1.0, 0.9), G=0.9, gads=(0.3, -0.3), mask=m,
                fields={0: (0.5 + 0.3 * rng.uniform(size=n), None, None),
                        1: (0.5 + 0.3 * rng.uniform(size=n), None, None)},
                solute=0.8, q=9, C=0.1 + 0.05 * rng.uniform(size=n), accel=[(1, 1e-5, 0)])
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(60)
    g.iteration(60)
    for c in (0, 1):
        gr, gx, gy = g.moments(c)
        orr, ox, oy = o.moments(c)
        assert rel_err(gr, orr) <= 1e-12
        us = max(np.abs(ox).max(), np.abs(oy).max())
        assert rel_err(gx, ox, us) <= 1e-11 and rel_err(gy, oy, us) <= 1e-11
    Cg, _ = g.solute_state()
    Co, _ = o.solute_state()
    assert rel_err(Cg, Co) <= 1e-12


@pytest.mark.parametrize("nx,ny", [(4, 3), (6, 5)])
def test_tiny_lattice_with_slip_and_intersolute_fp64(nx, ny):
    """Slip and mixed solids (two-node mask ring) and the intersolute ring
    on lattices narrower than those rings."""
    rng = np.random.default_rng(nx + ny)
    n = nx * ny
    case = dict(nx=nx, ny=ny, tau=0.9, style=("mixed", 0.4), rects=[(1, 1, 1, 1)],
                fields={0: (1.0 + 0.1 * rng.uniform(size=n), 0.02 * rng.uniform(-1, 1, n), None)},
                solute=1.0, q=4, isol=(-5e-3, 1.0, 5e-3), C=5e-3 * (1 + 0.2 * rng.uniform(-1, 1, n)))
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(40)
    g.iteration(40)
    gr, gx, gy = g.moments(0)
    orr, ox, oy = o.moments(0)
    us = max(np.abs(ox).max(), np.abs(oy).max())
    assert rel_err(gr, orr) <= 1e-12 and rel_err(gx, ox, us) <= 1e-11 and rel_err(gy, oy, us) <= 1e-11
    Cg, _ = g.solute_state()
    Co, _ = o.solute_state()
    assert rel_err(Cg, Co) <= 1e-12
