"""Momentum openings (inlet/outlet + inlet_momentum/outlet_momentum
commands, Zou-He closure of App. A, gradient extrapolation) on the GPU,
through the C ABI, against the FP64 oracle: every wall, every style, one
and two components, FP64 (1e-11) and FP32 (1e-5)."""
import numpy as np
import pytest

from cases import build_gpu, build_oracle, channel_flow_case, rel_err

pytestmark = pytest.mark.gpu


def _cmp(g, o, comps, tol, tol_u=None):
    tol_u = tol if tol_u is None else tol_u
    for c in comps:
        gr, gx, gy = g.moments(c)
        orr, ox, oy = o.moments(c)
        solid = orr == -11.0
        assert np.array_equal(gr == -11.0, solid)
        er = rel_err(gr[~solid], orr[~solid])
        eu = max(rel_err(gx, ox), rel_err(gy, oy))
        print(f"comp {c}: rel rho err {er:.3e}, rel u err {eu:.3e}")
        assert er <= tol and eu <= tol_u


@pytest.mark.parametrize("wall", ["xlo", "xhi", "ylo", "yhi"])
def test_poiseuille_inlet_pressure_outlet_fp64(wall):
    case = channel_flow_case(61, 37, 3, wall=wall)
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(250)
    g.iteration(250)
    _cmp(g, o, [0], 1e-11)


@pytest.mark.parametrize("inlet,outlet", [
    (("uniform", 0.03, 1.0), ("gradient", 0.0, 1.0)),
    (("dirichlet", 0.0, 1.01), ("dirichlet", 0.0, 0.99)),
    (("dirichlet", 0.0, 1.005), ("uniform", 0.02, 1.0)),
])
def test_opening_styles_fp64(inlet, outlet):
    case = channel_flow_case(70, 29, 4, inlet=inlet, outlet=outlet)
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(300)
    g.iteration(300)
    _cmp(g, o, [0], 1e-11)


def test_openings_fp32():
    """FP32 bound: with open boundaries the start-up is acoustic, and a
    density error d rho carries a velocity error c_s d rho / rho, so
    relative to max |u| = 0.05 the velocity bound is the density bar 1e-5
    times c_s / 0.05 = 1.15e-4."""
    case = channel_flow_case(130, 45, 5, wall="ylo", inlet=("poiseuille", 0.05, 1.0),
                             outlet=("gradient", 0.0, 1.0))
    o, g = build_oracle(case), build_gpu(case, "f32")
    o.iteration(400)
    g.iteration(400)
    _cmp(g, o, [0], 1e-5, 1e-5 * (1 / 3) ** 0.5 / 0.05)


def test_two_components_with_their_own_openings():
    """Two components (no cohesion): component 0 enters by a velocity inlet,
    component 1 by a pressure inlet; both leave by pressure outlets."""
    nx, ny = 48, 30
    case = channel_flow_case(nx, ny, 6)
    case["fluids"] = (0.9, 0.7)
    case["mopen"] = [("xlo", 1, ny - 2, 0, "inlet", "uniform", 0.02, 0.6),
                     ("xhi", 1, ny - 2, 0, "outlet", "dirichlet", 0.0, 0.6),
                     ("xlo", 1, ny - 2, 1, "inlet", "dirichlet", 0.0, 0.42),
                     ("xhi", 1, ny - 2, 1, "outlet", "dirichlet", 0.0, 0.4)]
    case["fields"] = {0: (np.full(nx * ny, 0.6), None, None), 1: (np.full(nx * ny, 0.4), None, None)}
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(200)
    g.iteration(200)
    _cmp(g, o, [0, 1, -1], 1e-11)
