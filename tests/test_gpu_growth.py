"""Surface growth on the benchmark's two-component + solute workload
(surface_reaction command, App. C) against the FP64 oracle.

The workload generator's lattice (discs r 10..30 to porosity 0.7, A/B blobs,
G = 0.9, adhesion +-0.3, D2Q9 solute tau_s = 0.7 with a dirichlet inlet
C = 1 at xlo and an adiabatic xhi, b_max = 1) at 256 x 256 nodes, with the
reaction rate raised from 1e-3 to 0.2 so that a few hundred nodes grow in
600 steps (at 1e-3 the first node grows after thousands of steps).

FP64 storage: masks bit-identical after every chunk, C and b within 1e-11.
FP32 storage: the growth-mask protocol.  A run stepped one step at a time
next to the oracle may take a different growth decision only where the
oracle's decision deposit lies within the FP32 error bound of b_max; every
such event is checked, then the GPU is set to the oracle's state and the
run goes on, so every divergence of the whole run is checked.
"""
import numpy as np
import pytest

from cases import build_gpu, build_oracle, rel_err, sc_solute_case

pytestmark = pytest.mark.gpu

KR = 0.2


def generator_case(n=256, kr=KR):
    """The two-component + solute workload at n x n from its generator."""
    from paper_1202_0442_amd import inputs
    w = inputs.sc_solute(n=n, kr=kr)
    e = w.extra
    ra, rb = inputs.sc_initial_fields(w)
    return dict(nx=w.nx, ny=w.ny, tau=w.tau, fluids=(w.tau, e["tau2"]), G=e["G"], gads=e["Gads"],
                circles=w.discs, fields={0: (ra.ravel(), None, None), 1: (rb.ravel(), None, None)},
                solute=e["tau_s"], q=9, C=np.zeros(w.nx * w.ny),
                openings=[("xlo", "dirichlet", e["C_in"]), ("xhi", "adiabatic", 0.0)],
                reaction=(kr, e["Cs"], e["b0"], e["bmax"], e["rng_seed"]))


def test_generator_workload_fp64_growth_matches_oracle():
    case = generator_case()
    o, g = build_oracle(case), build_gpu(case, "f64")
    assert np.array_equal(g.mask(), o.get_mask())
    for _ in range(6):
        o.iteration(100)
        g.iteration(100)
        assert np.array_equal(g.mask(), o.get_mask()), f"mask differs after {o.t} steps"
    bo, bg = o.budgets(), g.budgets()
    print(f"grown {bo['grown_nodes']:.0f} nodes in {o.t} steps")
    assert bo["grown_nodes"] > 100 and bg["grown_nodes"] == bo["grown_nodes"]
    Cg, b_g = g.solute_state()
    Co, b_o = o.solute_state()
    assert rel_err(Cg, Co) <= 1e-11
    assert rel_err(b_g, b_o) <= 1e-11
    for comp in (0, 1):
        gr, gx, gy = g.moments(comp)
        orr, ox, oy = o.moments(comp)
        assert rel_err(gr, orr) <= 1e-12
        assert max(rel_err(gx, ox), rel_err(gy, oy, np.abs(ox).max())) <= 1e-10


def _link_rate_sum(q=9):
    """Largest sum of the link rates k_i / kr around one solid node: all
    eight links, k_i = kr w_i / W with W = 1/6 (D2Q9)."""
    return (4 / 9 + 4 / 36) / (1 / 6) if q == 9 else 4.0


def growth_protocol(case, steps, tol_c=1e-5):
    """Steps the FP32 GPU run and the oracle one step at a time.

    Bound on the deposit error: each step adds sum_i k_i (C_i - C_s) to a
    solid's deposit.  While the concentrations meet the FP32 bar
    |dC| <= tol_c max C, a step's deposit differs by at most
    sum_i k_i tol_c max C <= (10/3) kr tol_c max C, so after t steps
    |b_gpu - b_oracle| <= t (10/3) kr tol_c max C =: eps_b(t).  A growth
    decision may therefore differ only at a solid whose oracle decision
    deposit is within eps_b of b_max.  At every step the test checks the
    concentrations against the bar and the deposits against eps_b, and
    every node where the masks or deposits differ against that margin; then
    it copies the oracle's state into the GPU run (eps_b restarts at 0).
    Returns (first divergence step or None, number of divergent steps,
    grown nodes)."""
    kr, _, _, bmax, _ = case["reaction"]
    o, g = build_oracle(case), build_gpu(case, "f32")
    per_step = _link_rate_sum(case.get("q", 9)) * kr * tol_c
    t_sync = 0
    first, events, worst_b = None, 0, 0.0
    mask = o.get_mask()
    for t in range(1, steps + 1):
        o.iteration(1)
        g.iteration(1)
        Co, bo = o.solute_state()
        Cg, bg = g.solute_state()
        cmax = max(np.abs(Co).max(), 1e-30)
        assert np.abs(Cg - Co).max() <= tol_c * cmax, f"step {t}: C beyond the FP32 bar"
        eps_b = (t - t_sync) * per_step * cmax
        mo, mg = o.get_mask(), g.mask()
        solid_both = (mo == 1) & (mg == 1)
        db = np.abs(bg - bo) * solid_both
        off_b = db > eps_b
        off_m = mo != mg
        worst_b = max(worst_b, float(db[~off_b].max(initial=0.0)))
        if not off_b.any() and not off_m.any():
            mask = mo
            continue
        events += 1
        first = t if first is None else first
        bdec = o.get_bdec()
        near = (mask == 1) & (np.abs(bdec - bmax) < eps_b)   # solids at the start of the step
        # a differing deposit: a trigger taken on one side only
        assert np.all(near[off_b]), f"step {t}: deposits differ away from b_max"
        # a differing mask node: grown from a near-threshold direct neighbour
        nb = np.zeros_like(near)
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            nb |= np.roll(np.roll(near, dy, axis=0), dx, axis=1)
        assert np.all(nb[off_m]), f"step {t}: mask differs away from a near-threshold trigger"
        print(f"step {t}: {int(off_m.sum())} mask / {int(off_b.sum())} deposit nodes differ "
              f"(margin bound {eps_b:.2e})")
        # continue from the oracle's state
        g.set_mask(mo)
        g.set_deposit(o.get_b())
        for comp in range(2 if "fluids" in case else 1):
            g.set_populations(o.get_f(comp), comp)
        g.set_populations(o.get_g(), -1)
        t_sync = t
        mask = mo
    grown = o.budgets()["grown_nodes"]
    print(f"first divergence {first}, divergent steps {events}, grown {grown:.0f}, "
          f"largest deposit error where decisions agreed {worst_b:.2e}")
    return first, events, grown


def test_generator_workload_fp32_growth_protocol():
    first, events, grown = growth_protocol(generator_case(), 600)
    assert grown > 100


def test_growth_across_row_segments_and_the_periodic_seam_fp64():
    """The growth kernel visits only the 256-node row segments that hold a
    trigger's target.  Discs straddle the segment boundary at x = 256 and
    the periodic seam (x = 0 / nx - 1) of a 300 x 40 lattice with a
    periodic solute (uniform C = 1, kr = 0.01, b_max = 1), so triggers in
    one segment grow nodes in the other, on both sides of the seam.  FP64:
    masks bit-identical every 50 steps for 300 steps, C and b within 1e-11."""
    nx, ny = 300, 40
    case = dict(nx=nx, ny=ny, tau=1.0, solute=0.8, q=9,
                circles=[(256, 10, 3), (1, 28, 3), (298, 10, 3), (128, 20, 4)],
                fields={0: (np.ones(nx * ny), None, None)}, C=np.full(nx * ny, 1.0),
                reaction=(0.01, 0.0, 0.5, 1.0, 7))
    o, g = build_oracle(case), build_gpu(case, "f64")
    m0 = o.get_mask().copy()
    assert np.array_equal(g.mask(), m0)
    for _ in range(6):
        o.iteration(50)
        g.iteration(50)
        assert np.array_equal(g.mask(), o.get_mask()), f"mask differs after {o.t} steps"
    grown_x = set(np.argwhere((o.get_mask() != 0) & (m0 == 0))[:, 1].tolist())
    print(f"grown {len(np.argwhere((o.get_mask() != 0) & (m0 == 0)))} nodes")
    assert {0, nx - 1, 255, 256} <= grown_x
    Cg, b_g = g.solute_state()
    Co, b_o = o.solute_state()
    assert rel_err(Cg, Co) <= 1e-11
    assert rel_err(b_g, b_o) <= 1e-11
