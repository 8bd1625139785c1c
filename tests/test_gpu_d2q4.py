"""GPU parity of the paper's D2Q4 solute lattice (solute command,
g_eq = C/4 (1 + 2 e.u)) against the FP64 oracle, through the C ABI: the
openings with a single unknown population, the reactive rule of App. C as
printed, growth, and the paper's surface-growth example (periodic 200x200
box, 11x11 seed, f0 = 24, C0 = 1.5, Cs = 0.5, b0 = 0.5, bmax = 1).
Bars as for D2Q9: masks bit-identical, FP64 within 1e-12 relative (1e-11
for concentrations after hundreds of steps), FP32 within 1e-5.
"""
import numpy as np
import pytest

from cases import build_gpu, build_oracle, rel_err, sc_solute_case, surface_growth_case

pytestmark = pytest.mark.gpu


def _cmp_solute(g, o, tol_c, tol_b):
    Cg, bg = g.solute_state()
    Co, bo = o.solute_state()
    ec, eb = rel_err(Cg, Co), rel_err(bg, bo)
    print(f"rel C err {ec:.3e}, rel b err {eb:.3e}")
    assert ec <= tol_c
    assert eb <= tol_b


def test_d2q4_sc_solute_growth_fp64_matches_oracle():
    """Two components with adhesion, D2Q4 solute with a Dirichlet inlet and
    an adiabatic outlet, reactive walls and growth, FP64."""
    case = sc_solute_case(96, 80, 21, react=True, q=4)
    o, g = build_oracle(case), build_gpu(case, "f64")
    for chunk in (41, 120, 139):
        o.iteration(chunk)
        g.iteration(chunk)
        assert np.array_equal(g.mask(), o.get_mask()), f"mask differs after {o.t} steps"
    bo, bg = o.budgets(), g.budgets()
    assert bo["grown_nodes"] > 5 and bg["grown_nodes"] == bo["grown_nodes"]
    _cmp_solute(g, o, 1e-11, 1e-12)
    for k in ("mass0", "mass1", "solute", "deposit", "removed_solute", "inflow", "outflow",
              "consumed_deposit"):
        assert bg[k] == pytest.approx(bo[k], rel=1e-11, abs=1e-12), k


def test_d2q4_fp32_matches_oracle_without_growth():
    case = sc_solute_case(130, 72, 22, react=True, kr=0.05, bmax=1e30, q=4)
    o, g = build_oracle(case), build_gpu(case, "f32")
    o.iteration(250)
    g.iteration(250)
    _cmp_solute(g, o, 1e-5, 1e-5)


def test_d2q4_raw_populations():
    """Raw g: the four D2Q4 planes match the oracle's, planes 0 and 5..8
    read as zero; a set with a nonzero absent plane is rejected."""
    from paper_1202_0442_amd import lb2d
    case = sc_solute_case(70, 37, 23, react=True, kr=0.02, q=4)
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(33)
    g.iteration(33)
    gg, go = g.get_populations(-1), o.get_g()
    assert np.all(gg[[0, 5, 6, 7, 8]] == 0.0)
    assert rel_err(gg, go) <= 1e-12
    g.set_populations(gg, -1)
    assert np.array_equal(g.get_populations(-1), gg)
    bad = gg.copy()
    bad[5, 3, 3] = 1e-3
    with pytest.raises(lb2d.LB2DError) as e:
        g.set_populations(bad, -1)
    assert e.value.code == lb2d.E_INVAL


@pytest.mark.parametrize("kr,steps", [(5e-3, 600), (0.1, 400)])
def test_surface_growth_example_fp64_matches_oracle(kr, steps):
    """The paper's surface-growth set-up (Da = 4 and 80) for the first
    hundreds of steps: identical masks and deposits in FP64."""
    case = surface_growth_case(kr)
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(steps)
    g.iteration(steps)
    assert np.array_equal(g.mask(), o.get_mask())
    bo, bg = o.budgets(), g.budgets()
    print(f"kr {kr}: grown {bo['grown_nodes']}")
    assert bo["grown_nodes"] > 0 and bg["grown_nodes"] == bo["grown_nodes"]
    _cmp_solute(g, o, 1e-11, 1e-12)


def test_surface_growth_budget_closes_on_gpu():
    """Periodic box, no openings: solute + deposit + consumed deposit +
    solute removed by growth - b0 per grown node stays at its start value."""
    case = surface_growth_case(0.05)
    g = build_gpu(case, "f64")
    b0 = g.budgets()
    g.iteration(1000)
    b1 = g.budgets()
    assert b1["grown_nodes"] > 0
    lhs = (b1["solute"] + b1["deposit"] + b1["removed_solute"] + b1["consumed_deposit"]
           - 0.5 * b1["grown_nodes"])
    rhs = b0["solute"] + b0["deposit"]
    assert lhs == pytest.approx(rhs, rel=1e-12)
    assert b1["inflow"] == 0.0 and b1["outflow"] == 0.0


def test_paper_surface_growth_sweep_full_size():
    """The paper's Da sweep (Da = 4, 20, 40, 80) at its full 20 000 steps
    in FP64: every final mask is bit-identical to the FP64 oracle's (stored
    by tests/golden/make_surface_growth_sweep.py, which calls only the
    oracle), the grown structure is less compact -- larger perimeter per
    square root of area -- as Da grows (Fig. surface), and the solute
    budget closes in every run."""
    import hashlib
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "surface_growth_sweep.json")))
    shape = []
    for kr in (5e-3, 0.025, 0.05, 0.1):
        g = build_gpu(surface_growth_case(kr), "f64")
        b0 = g.budgets()
        g.iteration(20000)
        b1 = g.budgets()
        ref = gold["runs"][repr(kr)]
        assert hashlib.sha256(g.mask().astype("uint8").tobytes()).hexdigest() == ref["mask_sha256"]
        assert int(b1["grown_nodes"]) == ref["grown_nodes"]
        assert b1["solute"] == pytest.approx(ref["solute"], rel=1e-10)
        assert b1["deposit"] == pytest.approx(ref["deposit"], rel=1e-10)
        lhs = (b1["solute"] + b1["deposit"] + b1["removed_solute"] + b1["consumed_deposit"]
               - 0.5 * b1["grown_nodes"])
        assert lhs == pytest.approx(b0["solute"] + b0["deposit"], rel=1e-11)
        m = g.mask().astype(int)
        per = (np.abs(np.diff(m, axis=0, append=m[:1])).sum()
               + np.abs(np.diff(m, axis=1, append=m[:, :1])).sum())
        shape.append(per / np.sqrt(m.sum()))
    print("perimeter / sqrt(area):", shape)
    assert all(a < b for a, b in zip(shape, shape[1:]))
