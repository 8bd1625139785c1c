"""The intersolute force (tau_s F / C added to the solute equilibrium
velocity, F = -G psi(x) sum_{i=1..4} psi(x + e_i) e_i, psi = psi0
exp(-C0 / C)) on the GPU, through the C ABI, against the FP64 oracle.

The paper's example (G = -5e-3, psi0 = 1, C0 = 5e-3) with tau_s = 1 makes
the uniform state unstable near C = C0 (the force's anti-diffusion
2 tau_s G psi psi' reaches 0.27, above the diffusivity D = 1/4 on D2Q4 and
1/6 on D2Q9), which is how it forms interfaces.  A rounding difference then
grows with the unstable modes: a relative change of 6e-8 in the initial
concentrations is amplified A(N) times after N steps, measured on the
oracle at the test's size: A(100) = 0.55 (D2Q4), 26 (D2Q9); A(300) = 0.66,
161.  So element-wise parity is checked over a few hundred steps and the
late state through properties.  FP32 bound: every step rounds every value
(relative 2^-24 = 6e-8), each such error growing by at most A(N) by step
N, so the error is below N A(N) 2^-24: 3.3e-6 on D2Q4 (the 1e-5 bar
holds) and 1.6e-4 on D2Q9 after 100 steps.
"""
import math

import numpy as np
import pytest

from cases import build_gpu, build_oracle, intersolute_case, rel_err, sc_solute_case, slip_box_case

pytestmark = pytest.mark.gpu


def _cmp(g, o, tol_c, tol_b=None):
    Cg, bg = g.solute_state()
    Co, bo = o.solute_state()
    ec = rel_err(Cg, Co)
    print(f"rel C err {ec:.3e}")
    assert ec <= tol_c
    if tol_b is not None:
        assert rel_err(bg, bo) <= tol_b


@pytest.mark.parametrize("q,storage,steps,tol", [(4, "f64", 300, 1e-11), (9, "f64", 300, 1e-11),
                                                  (4, "f32", 100, 1e-5), (9, "f32", 100, 100 * 26 * 2.0 ** -24)])
def test_paper_example_matches_oracle(q, storage, steps, tol):
    """The paper's parameters on a ragged lattice with a few discs."""
    case = intersolute_case(90, 70, 11, q=q, nd=4)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(steps)
    g.iteration(steps)
    _cmp(g, o, tol)


def test_paper_example_forms_interfaces():
    """100 x 100, the paper's parameters: the concentration separates into
    high and low domains (relative spread above 0.2 after 2000 steps) while
    without the force the noise diffuses away; the solute is conserved."""
    spread = {}
    for G in (-5e-3, 0.0):
        g = build_gpu(intersolute_case(100, 100, 5, isol=(G, 1.0, 5e-3)), "f64")
        s0 = g.budgets()["solute"]
        g.iteration(2000)
        C, _ = g.solute_state()
        spread[G] = C.std() / C.mean()
        assert g.budgets()["solute"] == pytest.approx(s0, rel=1e-12)
    print(spread)
    assert spread[-5e-3] > 0.2 and spread[0.0] < 0.01


@pytest.mark.parametrize("q,tau_s,G,Cl,Cg", [(4, 5.0, -0.01, 0.01094, 0.002342),
                                              (9, 5.0, -0.007, 0.01216, 0.002111)])
def test_flat_interface_balance_on_gpu(q, tau_s, G, Cl, Cg):
    """The exact balance of a steady flat interface (see the oracle's pin):
    (D / tau_s) C + G psi^2 equal in both bulk phases; the profile matches
    the oracle's."""
    nx, ny = 4, 128
    yy = np.repeat(np.arange(ny), nx).astype(float)
    C = Cg + (Cl - Cg) * 0.5 * (np.tanh((yy - ny / 4) / 4.0) - np.tanh((yy - 3 * ny / 4) / 4.0))
    case = dict(nx=nx, ny=ny, tau=1.0, solute=tau_s, q=q, isol=(G, 1.0, 5e-3), C=C)
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(20000)
    g.iteration(20000)
    Cgpu, _ = g.solute_state()
    Co, _ = o.solute_state()
    assert rel_err(Cgpu, Co) <= 1e-10
    cl, cg = Cgpu[64].mean(), Cgpu[0].mean()
    D = (0.5 if q == 4 else 1.0 / 3.0) * (tau_s - 0.5)
    p = lambda c: D / tau_s * c + G * math.exp(-5e-3 / c) ** 2
    assert cl > 4 * cg
    assert p(cl) == pytest.approx(p(cg), rel=1e-9)


@pytest.mark.parametrize("q", [4, 9])
def test_intersolute_with_openings_on_every_wall_and_growth_fp64(q):
    """Flux, dirichlet and adiabatic openings on all four walls (the psi
    stencil stops at closed walls; flux nodes carry psi of their imposed
    concentration), reactive walls and growth, a forced flow."""
    rng = np.random.default_rng(19)
    nx, ny = 40, 36
    circles = [(int(rng.integers(8, 32)), int(rng.integers(8, 28)), float(rng.uniform(2, 4))) for _ in range(5)]
    case = dict(nx=nx, ny=ny, tau=1.0, accel=[(1, 2e-5, 0)], circles=circles, solute=0.9, q=q,
                C=0.3 * (1 + 0.2 * rng.uniform(-1, 1, nx * ny)), isol=(-0.1, 1.0, 0.3),
                sopen=[("xlo", 2, 30, "inlet", "flux", 1.0, 0.05), ("xhi", 0, 35, "outlet", "adiabatic", 0.0, 0.0),
                       ("ylo", 4, 20, "inlet", "dirichlet", 0.7, 0.0), ("yhi", 10, 30, "outlet", "flux", 0.1, 0.3)],
                reaction=(0.02, 0.0, 0.003, 0.2, 9))
    o, g = build_oracle(case), build_gpu(case, "f64")
    for chunk in (61, 120, 119):
        o.iteration(chunk)
        g.iteration(chunk)
        assert np.array_equal(g.mask(), o.get_mask())
    bo, bg = o.budgets(), g.budgets()
    assert bo["grown_nodes"] > 0 and bg["grown_nodes"] == bo["grown_nodes"]
    _cmp(g, o, 1e-11, 1e-11)
    for k in ("solute", "deposit", "inflow", "outflow"):
        assert bg[k] == pytest.approx(bo[k], rel=1e-11, abs=1e-12), k


def test_intersolute_with_two_fluids_fp64():
    """Two-component Shan-Chen flow, D2Q9 solute with the x openings of the
    benchmark workload, reaction and growth, plus intersolute."""
    case = sc_solute_case(96, 64, 31, react=True, kr=0.02, q=9)
    case["isol"] = (-0.01, 1.0, 0.05)
    o, g = build_oracle(case), build_gpu(case, "f64")
    for chunk in (70, 130):
        o.iteration(chunk)
        g.iteration(chunk)
        assert np.array_equal(g.mask(), o.get_mask()), f"mask differs after {o.t} steps"
    _cmp(g, o, 1e-11, 1e-11)


def test_intersolute_with_slip_solids_fp64():
    """Hybrid slip/mixed obstacles and intersolute in one lattice."""
    case = slip_box_case(70, 45, 21, two=False, nob=10)
    rng = np.random.default_rng(3)
    case.update(solute=1.0, q=4, isol=(-5e-3, 1.0, 5e-3), C=5e-3 * (1 + 0.1 * rng.uniform(-1, 1, 70 * 45)))
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(200)
    g.iteration(200)
    _cmp(g, o, 1e-11)
