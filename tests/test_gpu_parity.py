"""GPU (gfx950) parity against the FP64 oracle, through the C ABI.

Element-by-element comparisons on seeded inputs at sizes the oracle finishes
in seconds, spanning several tiles and ragged tails.  Bars: masks and growth
bit-identical; FP64 storage within 1e-12 (relative to the field's scale);
FP32 storage within 1e-5; 16-bit storage within the bounds stated in each
test.
"""
import numpy as np
import pytest

from cases import (build_gpu, build_oracle, poiseuille_case, porous_case, rel_err,
                   sc_solute_case)

pytestmark = pytest.mark.gpu


def _cmp_fluid(g, o, comps, tol_u, tol_rho):
    for comp in comps:
        gr, gx, gy = g.moments(comp)
        orr, ox, oy = o.moments(comp)
        solid = orr == -11.0
        assert np.array_equal(gr == -11.0, solid)
        uscale = max(np.abs(ox).max(), np.abs(oy).max(), 1e-30)
        eu = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / uscale
        er = np.abs(gr - orr)[~solid].max() / np.abs(orr[~solid]).max()
        print(f"comp {comp}: rel u err {eu:.3e}, rel rho err {er:.3e}")
        assert eu <= tol_u, (comp, eu)
        assert er <= tol_rho, (comp, er)


def test_poiseuille_fp64_matches_oracle():
    case = poiseuille_case()
    o, g = build_oracle(case), build_gpu(case, "f64")
    assert np.array_equal(g.mask(), o.get_mask())
    o.iteration(5000)
    g.iteration(5000)
    _cmp_fluid(g, o, [0], 1e-12, 1e-12)
    bo, bg = o.budgets(), g.budgets()
    assert bg["mass0"] == pytest.approx(bo["mass0"], rel=1e-12)
    assert bg["mom_x"] == pytest.approx(bo["mom_x"], rel=1e-11)
    assert bg["steps"] == 5000 and bg["fluid_nodes"] == bo["fluid_nodes"]


@pytest.mark.parametrize("nx,ny,seed", [(250, 190, 1), (64, 64, 2), (97, 33, 3)])
def test_porous_fp32_matches_oracle(nx, ny, seed):
    case = porous_case(nx, ny, seed)
    o, g = build_oracle(case), build_gpu(case, "f32")
    assert np.array_equal(g.mask(), o.get_mask())
    o.iteration(300)
    g.iteration(300)
    _cmp_fluid(g, o, [0], 1e-5, 1e-5)
    assert g.budgets()["mass0"] == pytest.approx(o.budgets()["mass0"], rel=1e-6)


def test_porous_fp64_matches_oracle():
    case = porous_case(130, 70, 4)
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(257)
    g.iteration(257)
    _cmp_fluid(g, o, [0], 1e-12, 1e-12)
    np.testing.assert_allclose(g.get_populations(0), o.get_f(0), rtol=0, atol=1e-13)


@pytest.mark.parametrize("storage,tol", [("f16", 3e-2), ("bf16", 2e-1)])
def test_porous_16bit_storage_error_bound(storage, tol):
    """16-bit shifted storage, FP32 arithmetic: errors of u and rho against
    the oracle stay within the stated bound (relative to max |u|)."""
    case = porous_case(200, 120, 5, accel=1e-5)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(400)
    g.iteration(400)
    _cmp_fluid(g, o, [0], tol, tol * 1e-2)


def test_two_component_shan_chen_fp64_matches_oracle():
    case = sc_solute_case(96, 80, 7, react=False, openings=False)
    case.pop("solute")
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(300)
    g.iteration(300)
    _cmp_fluid(g, o, [0, 1, -1], 1e-11, 1e-12)


def test_sc_solute_growth_fp64_matches_oracle():
    """Two components, adhesion, D2Q9 solute with openings, reactive walls
    and growth in FP64: masks and deposits agree exactly / to 1e-12."""
    case = sc_solute_case(96, 80, 11, react=True)
    o, g = build_oracle(case), build_gpu(case, "f64")
    for chunk in (37, 100, 163):
        o.iteration(chunk)
        g.iteration(chunk)
        assert np.array_equal(g.mask(), o.get_mask()), f"mask differs after {o.t} steps"
    bo, bg = o.budgets(), g.budgets()
    print({k: (bo[k], bg[k]) for k in bo})
    assert bo["grown_nodes"] > 5 and bg["grown_nodes"] == bo["grown_nodes"]
    _cmp_fluid(g, o, [0, 1, -1], 1e-11, 1e-12)
    Cg, bgd = g.solute_state()
    Co, bod = o.solute_state()
    assert rel_err(Cg, Co) <= 1e-11
    assert rel_err(bgd, bod) <= 1e-12
    for k in ("mass0", "mass1", "solute", "deposit", "removed_mass0", "removed_mass1",
              "removed_solute", "inflow", "outflow", "consumed_deposit"):
        assert bg[k] == pytest.approx(bo[k], rel=1e-11, abs=1e-12), k


def test_sc_solute_fp32_matches_oracle_without_growth():
    case = sc_solute_case(130, 72, 12, react=True, kr=0.05, bmax=1e30)
    o, g = build_oracle(case), build_gpu(case, "f32")
    o.iteration(250)
    g.iteration(250)
    _cmp_fluid(g, o, [0, 1, -1], 1e-5, 1e-5)
    Cg, bgd = g.solute_state()
    Co, bod = o.solute_state()
    assert rel_err(Cg, Co) <= 1e-5
    assert rel_err(bgd, bod) <= 1e-5


def test_sc_solute_fp32_growth_mask_protocol():
    """FP32 with growth: every step where the GPU takes a growth decision
    the oracle does not (or the reverse) must have an oracle decision
    deposit within the FP32 error bound of b_max; the protocol
    (tests/test_gpu_growth.py) checks each such step and continues from the
    oracle's state."""
    from test_gpu_growth import growth_protocol
    first, events, grown = growth_protocol(sc_solute_case(96, 80, 13, react=True), 300)
    assert grown > 5


def test_solute_budget_closes_on_gpu():
    case = sc_solute_case(120, 64, 14, react=True, b0=0.003)
    g = build_gpu(case, "f64")
    b0 = g.budgets()
    g.iteration(300)
    b1 = g.budgets()
    assert b1["grown_nodes"] > 0
    lhs = (b1["solute"] + b1["deposit"] + b1["removed_solute"] + b1["consumed_deposit"]
           - 0.003 * b1["grown_nodes"])
    rhs = b0["solute"] + b0["deposit"] + b1["inflow"] - b1["outflow"]
    assert lhs == pytest.approx(rhs, rel=1e-12)
    for c in (0, 1):
        assert b1[f"mass{c}"] + b1[f"removed_mass{c}"] == pytest.approx(b0[f"mass{c}"], rel=1e-12)


def test_growth_picks_hashed_neighbour_on_gpu():
    """5x5 lattice with a preset deposit above b_max: the GPU grows exactly
    the node the oracle grows."""
    for seed in range(6):
        case = dict(nx=5, ny=5, tau=1.0, rects=[(2, 2, 2, 2), (2, 2, 3, 3)], solute=1.0,
                    C=np.full(25, 0.4), reaction=(0.0, 0.0, 0.25, 1.0, seed))
        o, g = build_oracle(case), build_gpu(case, "f64")
        b = np.zeros((5, 5))
        b[2, 2] = 1.5
        b[3, 2] = 0.25
        o.set_b(b)
        g.set_deposit(b)
        o.iteration(1)
        g.iteration(1)
        assert np.array_equal(g.mask(), o.get_mask())
        np.testing.assert_array_equal(g.get_deposit(), o.get_b())
        assert g.budgets()["grown_nodes"] == 1


def test_runs_are_bitwise_deterministic():
    case = sc_solute_case(100, 60, 15, react=True)
    outs = []
    for _ in range(2):
        g = build_gpu(case, "f32")
        g.iteration(150)
        outs.append((g.get_populations(0), g.get_populations(1), g.get_populations(-1), g.mask(),
                     g.get_deposit(), g.budgets()))
    for a, b in zip(outs[0][:5], outs[1][:5]):
        assert np.array_equal(a, b)
    assert outs[0][5] == outs[1][5]


@pytest.mark.parametrize("kind", ["plain", "full"])
def test_graph_launch_equals_single_launches(kind):
    case = porous_case(150, 90, 16) if kind == "plain" else sc_solute_case(96, 64, 16)
    a = build_gpu(case, "f32")
    a.iteration(70)  # a graph of 60 steps and a 10-step tail graph
    b = build_gpu(case, "f32")
    b.set_timing(True)
    b.iteration(70)
    ms, k = b.kernel_time()
    assert k == 70 and ms > 0
    assert np.array_equal(a.get_populations(0), b.get_populations(0))
    assert np.array_equal(a.mask(), b.mask())


@pytest.mark.parametrize("kind,storage", [("plain", "f32"), ("plain", "f16sr"), ("full", "f32"), ("full", "f16sr")])
def test_graphs_of_every_length_equal_single_launches(kind, storage):
    """lb2d_iteration launches graphs of 60 steps and one graph of the
    remaining steps, captured per starting parity (ahead by lb2d_prepare or
    on first use): calls of 1, 2, 5, 33, 63 and 7 steps (odd and even
    starts) equal the same steps launched one by one, also
    with stochastic rounding, whose random stream is keyed on the step."""
    case = porous_case(150, 90, 17) if kind == "plain" else sc_solute_case(96, 64, 17)
    st = storage[:3]

    def lattice():
        g = build_gpu(case, st, bind=False)
        if storage.endswith("sr"):
            g.rounding("stochastic", 5)
        g.bind(st)
        return g
    a, b = lattice(), lattice()
    b.set_timing(True)
    for n in (1, 2, 5, 33, 63, 7):
        a.prepare(n)
        a.iteration(n)
        b.iteration(n)
        assert a.step_count() == b.step_count()
        assert np.array_equal(a.get_populations(0), b.get_populations(0)), n
    if kind == "full":
        assert np.array_equal(a.get_populations(-1), b.get_populations(-1))
        assert np.array_equal(a.mask(), b.mask())


def test_minimum_lattice_and_zero_steps():
    case = dict(nx=3, ny=3, tau=0.9, accel=[(5, 1e-4, 0)],
                fields={0: (np.linspace(0.9, 1.1, 9), None, None)})
    o, g = build_oracle(case), build_gpu(case, "f64")
    g.iteration(0)
    np.testing.assert_allclose(g.get_populations(0), o.get_f(0), rtol=0, atol=1e-15)
    o.iteration(41)
    g.iteration(41)
    _cmp_fluid(g, o, [0], 1e-12, 1e-12)


def test_fully_blocked_rows_and_isolated_pockets():
    """Solid rows, a fluid node enclosed by solids and a solid column."""
    nx, ny = 20, 12
    m = np.zeros((ny, nx), np.uint8)
    m[0, :] = 1
    m[5:8, 9:12] = 1
    m[6, 10] = 0          # isolated fluid pocket
    m[:, 15] = 1
    case = dict(nx=nx, ny=ny, tau=0.7, accel=[(1, 1e-4, 0)], mask=m,
                fields={0: (1 + 0.1 * np.random.default_rng(3).uniform(size=nx * ny), None, None)})
    o, g = build_oracle(case), build_gpu(case, "f64")
    assert np.array_equal(g.mask(), o.get_mask())
    o.iteration(60)
    g.iteration(60)
    _cmp_fluid(g, o, [0], 1e-12, 1e-12)


def test_paper_two_fluid_contact_box_matches_oracle_fp64():
    """The paper's contact-angles II set-up: FP64 parity over the first 300
    steps (interfaces sharpen, walls on all four sides)."""
    from cases import two_fluid_contact_case
    case = two_fluid_contact_case()
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(300)
    g.iteration(300)
    _cmp_fluid(g, o, [0, 1], 1e-10, 1e-11)


def test_paper_two_fluid_contact_angles_are_complementary():
    """The paper's contact-angles II run (201 x 51 nodes, 20 000 steps): with
    the paper's adhesion signs one bridge of fluid 1 remains in the middle
    of the box, and the signs set complementary contact angles.  With the printed force
    F = -G_c rho_c sum w_i s e_i, G_1 = +0.2 repels fluid 1 from the walls
    and G_2 = -0.2 draws fluid 2 to them, so the fluid-1 bridge is narrower
    along the walls than at mid-height; exchanging the signs widens it
    there.  Both components' masses are conserved."""
    from cases import two_fluid_contact_case
    from scipy import ndimage
    widths = {}
    for sign in (1.0, -1.0):
        g = build_gpu(two_fluid_contact_case(0.2 * sign, -0.2 * sign), "f64")
        b0 = g.budgets()
        g.iteration(20000)
        b1 = g.budgets()
        for c in (0, 1):
            assert b1[f"mass{c}"] == pytest.approx(b0[f"mass{c}"], rel=1e-12)
        r1, _, _ = g.moments(0)
        dense = r1 > 1.0
        if sign > 0:                       # the paper's signs: a single fluid-1 region
            assert ndimage.label(dense)[1] == 1
        widths[sign] = (dense[1].sum() + dense[-2].sum()) / 2.0, float(dense[25].sum())
    print("fluid-1 width at the walls / mid-height:", widths)
    wall_p, mid_p = widths[1.0]
    wall_m, mid_m = widths[-1.0]
    assert wall_p < mid_p and wall_m > mid_m


def test_paper_parallel_droplet_matches_oracle_fp64():
    """The paper's parallelization example (351 x 201 nodes, a square of
    fluid 1 on a solid bottom row, periodic elsewhere): FP64 parity over the
    first 200 steps."""
    from cases import parallel_droplet_case
    case = parallel_droplet_case()
    o, g = build_oracle(case), build_gpu(case, "f64")
    o.iteration(200)
    g.iteration(200)
    _cmp_fluid(g, o, [0, 1], 1e-10, 1e-11)


def test_paper_parallel_droplet_is_hydrophobic():
    """The same run for 20 000 steps: the square of fluid 1 becomes a
    single droplet sitting on the wall, which it does not wet (contact
    angle above 90 degrees, since G_1 = +0.3 repels fluid 1 from solids):
    the droplet is narrower where it touches the wall than at its widest,
    and it stays clear of the solid row seen through the periodic top.
    Both components' masses are conserved."""
    from cases import parallel_droplet_case
    from scipy import ndimage
    g = build_gpu(parallel_droplet_case(), "f64")
    b0 = g.budgets()
    g.iteration(20000)
    b1 = g.budgets()
    for c in (0, 1):
        assert b1[f"mass{c}"] == pytest.approx(b0[f"mass{c}"], rel=1e-12)
    r1, _, _ = g.moments(0)
    dense = r1 > 1.0
    widths = dense.sum(axis=1)
    rows = np.nonzero(widths)[0]
    print(f"droplet rows {rows.min()}..{rows.max()}, width at the wall {widths[1]}, widest {widths.max()} "
          f"at row {widths.argmax()}")
    assert ndimage.label(dense)[1] == 1
    assert widths[1] > 0 and widths[1] < widths.max()
    assert widths[-1] == 0


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_paper_poiseuille_application(storage, tol):
    """The paper's Poiseuille application (61 x 31 nodes, initial
    populations 4 for the rest and slow modes and 1 for the fast ones, so
    rho = 24 off equilibrium, g from the printed formula, 10 000 steps) on
    the GPU: the same populations as the oracle's, and the profile of
    Eq. (profile) with u_max = 0.07."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "poiseuille_application.json")))
    Nx, Ny, tau, umax = gold["Nx"], gold["Ny"], gold["tau"], gold["u_max"]
    acc = 4.0 / 3.0 * umax * (2 * tau - 1) / (Ny - 1) ** 2
    case = dict(nx=Nx + 1, ny=Ny + 1, tau=tau, accel=[(1, acc, 0)], rects=[(0, Nx, 0, 0), (0, Nx, Ny, Ny)],
                fields={0: (np.full((Nx + 1) * (Ny + 1), 24.0), None, None)})
    o, g = build_oracle(case), build_gpu(case, storage)
    init = np.array([gold["pop_rest_slow"]] * 5 + [gold["pop_fast"]] * 4)
    f0 = np.broadcast_to(init[:, None, None], (9, Ny + 1, Nx + 1)).copy()
    f0[:, 0, :] = 0.0
    f0[:, Ny, :] = 0.0
    o.set_f(f0, 0)
    g.set_populations(f0, 0)
    o.iteration(gold["steps"])
    g.iteration(gold["steps"])
    _cmp_fluid(g, o, [0], tol, tol)
    _, ux, _ = g.moments(0)
    y = np.arange(1, Ny)
    prof = 3 * acc / (2 * tau - 1) * (((Ny - 1) / 2) ** 2 - (y - Ny / 2) ** 2)
    np.testing.assert_allclose(ux[1:Ny, 7], prof, atol=5e-3 * umax)
