"""Solute openings on every wall (inlet/outlet + inlet_solute /
outlet_solute commands, App. B): dirichlet, adiabatic and flux styles on
node ranges, closed (impermeable) wall parts, with the D2Q4 and D2Q9
solute lattices, against the FP64 oracle through the C ABI."""
import numpy as np
import pytest

from cases import build_gpu, build_oracle, rel_err

pytestmark = pytest.mark.gpu


def _case(q, react=True, seed=17, growth=True):
    rng = np.random.default_rng(seed)
    nx, ny = 40, 36
    circles = [(int(rng.integers(8, 32)), int(rng.integers(8, 28)), float(rng.uniform(2, 4))) for _ in range(5)]
    case = dict(nx=nx, ny=ny, tau=1.0, accel=[(1, 2e-5, 0)], circles=circles, solute=0.9, q=q,
                C=np.full(nx * ny, 0.3),
                sopen=[("xlo", 2, 30, "inlet", "flux", 1.0, 0.05), ("xhi", 0, 35, "outlet", "adiabatic", 0.0, 0.0),
                       ("ylo", 4, 20, "inlet", "dirichlet", 0.7, 0.0), ("yhi", 10, 30, "outlet", "flux", 0.1, 0.3)])
    if react:
        case["reaction"] = (0.02, 0.0, 0.003, 0.2 if growth else 1e30, 9)
    return case


def _cmp(g, o, tol):
    Cg, bg = g.solute_state()
    Co, bo = o.solute_state()
    ec, eb = rel_err(Cg, Co), rel_err(bg, bo)
    print(f"rel C err {ec:.3e}, rel b err {eb:.3e}")
    assert ec <= tol and eb <= tol


@pytest.mark.parametrize("q", [4, 9])
def test_openings_on_every_wall_fp64(q):
    case = _case(q)
    o, g = build_oracle(case), build_gpu(case, "f64")
    for chunk in (61, 120, 119):
        o.iteration(chunk)
        g.iteration(chunk)
        assert np.array_equal(g.mask(), o.get_mask())
    bo, bg = o.budgets(), g.budgets()
    assert bo["grown_nodes"] > 0 and bg["grown_nodes"] == bo["grown_nodes"]
    _cmp(g, o, 1e-11)
    for k in ("solute", "deposit", "inflow", "outflow", "consumed_deposit", "removed_solute"):
        assert bg[k] == pytest.approx(bo[k], rel=1e-11, abs=1e-12), k


def test_openings_on_every_wall_fp32():
    case = _case(9, growth=False)
    o, g = build_oracle(case), build_gpu(case, "f32")
    o.iteration(300)
    g.iteration(300)
    _cmp(g, o, 1e-5)


@pytest.mark.parametrize("kind", ["inlet", "outlet"])
def test_flux_opening_steady_profile_on_gpu(kind):
    """The closed form of the oracle's pin (tau_s = 1, D2Q4): linear steady
    profile C(x) = a (1 - x/(nx-1)) with a fixed by the flux rule."""
    nx, ny, C0 = 20, 3, 1.0
    v = 0.1 if kind == "inlet" else 0.5
    D = 0.25
    case = dict(nx=nx, ny=ny, tau=1.0, solute=1.0, q=4, C=np.zeros(nx * ny),
                sopen=[("xlo", 0, ny - 1, kind, "flux", C0, v), ("xhi", 0, ny - 1, "outlet", "dirichlet", 0.0, 0.0)])
    g = build_gpu(case, "f64")
    g.iteration(40000)
    C, _ = g.solute_state()
    k = 1 - 1 / (nx - 1)
    a = v * C0 / (D + v - D * k) if kind == "inlet" else v * C0 / (v - D + D * k)
    np.testing.assert_allclose(C.reshape(ny, nx)[1], a * (1 - np.arange(nx) / (nx - 1)), rtol=1e-12, atol=1e-14)


def _mirror_case(nx, ny, q, width=None, seed=44, uy=0.03):
    """Dirichlet xlo (C = 1) and, on xhi, an adiabatic opening (width None)
    or a dirichlet one on a strip of `width` nodes whose initial
    concentration is the mirror image of the nx-node strip's about its
    column nx - 1; one fluid flowing along the walls."""
    rng = np.random.default_rng(seed)
    C = 0.2 + 0.5 * rng.uniform(0, 1, (ny, nx))
    w = nx if width is None else width
    if width is not None:
        C = np.concatenate([C, C[:, -2::-1]], axis=1)
    xhi = ("xhi", 0, ny - 1, "outlet", "adiabatic" if width is None else "dirichlet", 1.0, 0.0)
    return dict(nx=w, ny=ny, tau=1.0, solute=0.7, q=q, C=C.ravel(),
                fields={0: (np.ones(w * ny), np.zeros(w * ny), np.full(w * ny, uy))},
                sopen=[("xlo", 0, ny - 1, "inlet", "dirichlet", 1.0, 0.0), xhi])


@pytest.mark.parametrize("q", [4, 9])
@pytest.mark.parametrize("nx,ny", [(13, 8), (77, 45)])
def test_adiabatic_wall_is_a_mirror_plane_fp64(q, nx, ny):
    """The adiabatic opening (g3 = g1 on xhi, each unknown copies its
    mirror) on the GPU: every solute population equals the oracle's, and
    the strip equals the oracle's mirrored strip of 2 nx - 1 nodes with
    dirichlet walls on both sides (the pin of the oracle's adiabatic rule)."""
    case = _mirror_case(nx, ny, q)
    o, g = build_oracle(case), build_gpu(case, "f64")
    wide = build_oracle(_mirror_case(nx, ny, q, width=2 * nx - 1))
    for side in (o, g, wide):
        side.iteration(60)
    np.testing.assert_allclose(g.get_populations(-1), o.get_g(), rtol=0, atol=1e-14)
    Cg, _ = g.solute_state()
    Cw, _ = wide.solute_state()
    np.testing.assert_allclose(Cg.reshape(ny, nx), Cw.reshape(ny, 2 * nx - 1)[:, :nx], rtol=1e-12)


def test_adiabatic_wall_fp32():
    case = _mirror_case(77, 45, 9)
    o, g = build_oracle(case), build_gpu(case, "f32")
    o.iteration(300)
    g.iteration(300)
    _cmp(g, o, 1e-5)
