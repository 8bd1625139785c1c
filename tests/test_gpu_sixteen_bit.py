"""16-bit storage (FP16, BF16) of the general step -- two fluids with
Shan-Chen forces, the D2Q9 and D2Q4 solutes, reactive walls, openings,
slip solids, the psi forces and intersolute -- against the FP64 oracle,
through the C ABI.  The arithmetic is FP32; every stored deviation is
rounded to nearest with a relative error of at most eps = 2^-11 (FP16) or
2^-8 (BF16).  Bounds are stated in units of eps: densities within 2 eps of
the largest density, velocities within 20 eps of the largest velocity
(small velocities are differences of stored populations), concentrations
and deposits within 4 eps (8 eps with the intersolute force, whose
anti-diffusion amplifies differences), after a few hundred steps.  Budgets
close to within eps.  Stochastic rounding moves a value to either
neighbouring 16-bit number, so its per-rounding error bound, and the
parity bounds, double; its gain is the absence of bias over long runs.
"""
import numpy as np
import pytest

from cases import (build_gpu, build_oracle, channel_flow_case, intersolute_case, phase_case, rel_err,
                   sc_solute_case)

pytestmark = pytest.mark.gpu

EPS = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
STORAGES = ["f16", "bf16"]


def _fluid_errs(g, o, ncomp):
    er = eu = 0.0
    for c in range(ncomp):
        gr, gx, gy = g.moments(c)
        orr, ox, oy = o.moments(c)
        solid = orr == -11.0
        assert np.array_equal(gr == -11.0, solid)
        us = max(np.abs(ox).max(), np.abs(oy).max())
        er = max(er, rel_err(gr[~solid], orr[~solid]))
        eu = max(eu, rel_err(gx, ox, us), rel_err(gy, oy, us))
    return er, eu


@pytest.mark.parametrize("q", [9, 4])
@pytest.mark.parametrize("storage", STORAGES)
def test_two_fluids_and_solute(storage, q):
    eps = EPS[storage]
    case = sc_solute_case(96, 64, 41, react=True, bmax=1e30, q=q)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(200)
    g.iteration(200)
    er, eu = _fluid_errs(g, o, 2)
    Cg, bg = g.solute_state()
    Co, bo = o.solute_state()
    ec, eb = rel_err(Cg, Co), rel_err(bg, bo)
    print(f"{storage} q{q}: rho {er:.2e} u {eu:.2e} C {ec:.2e} b {eb:.2e} (eps {eps:.1e})")
    assert er <= 2 * eps and eu <= 20 * eps and ec <= 4 * eps and eb <= 4 * eps


@pytest.mark.parametrize("storage", STORAGES)
def test_openings_between_slip_walls(storage):
    case = channel_flow_case(60, 31, 4, inlet=("uniform", 0.04, 1.0))
    case["style"] = ("slip", 1.0)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(300)
    g.iteration(300)
    er, eu = _fluid_errs(g, o, 1)
    print(f"{storage}: rho {er:.2e} u {eu:.2e}")
    assert er <= 2 * EPS[storage] and eu <= 20 * EPS[storage]


@pytest.mark.parametrize("storage", STORAGES)
def test_psi_phase_separation(storage):
    case = phase_case(70, 45, 31)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(25)
    g.iteration(25)
    er, eu = _fluid_errs(g, o, 1)
    print(f"{storage}: rho {er:.2e} u {eu:.2e}")
    assert er <= 2 * EPS[storage] and eu <= 20 * EPS[storage]


@pytest.mark.parametrize("storage", STORAGES)
def test_intersolute_d2q4(storage):
    case = intersolute_case(90, 70, 11, q=4, nd=4)
    o, g = build_oracle(case), build_gpu(case, storage)
    o.iteration(100)
    g.iteration(100)
    Cg, _ = g.solute_state()
    Co, _ = o.solute_state()
    ec = rel_err(Cg, Co)
    print(f"{storage}: C {ec:.2e}")
    assert ec <= 8 * EPS[storage]


@pytest.mark.parametrize("storage", STORAGES)
def test_budgets_close_with_growth(storage):
    """Growth on 16-bit storage: the solute budget (solute + deposit +
    solute and deposit removed by growth + outflow - inflow) and each
    component's mass (plus the mass removed by growth) stay within eps."""
    eps = EPS[storage]
    g = build_gpu(sc_solute_case(96, 64, 11, react=True), storage)
    b0 = g.budgets()
    g.iteration(300)
    b1 = g.budgets()
    assert b1["grown_nodes"] > 0
    sol = lambda d: (d["solute"] + d["deposit"] + d["removed_solute"] + d["consumed_deposit"] + d["outflow"]
                     - d["inflow"])
    assert abs(sol(b1) - sol(b0)) <= eps * b1["inflow"]
    for c in (0, 1):
        m0, m1 = b0[f"mass{c}"], b1[f"mass{c}"] + b1[f"removed_mass{c}"]
        assert abs(m1 - m0) <= eps * m0


def test_d2q4_raw_populations_round_trip_in_16bit():
    """D2Q4 solute planes keep directions 1..4: their 16-bit scale follows
    the direction, so raw populations read back as stored."""
    case = sc_solute_case(40, 24, 7, react=False, q=4)
    g = build_gpu(case, "f16")
    g.iteration(5)
    a = g.get_populations(-1)
    g.set_populations(a, -1)
    assert np.array_equal(g.get_populations(-1), a)
    C, _ = g.solute_state()
    assert np.allclose(C, a.sum(axis=0) * (g.mask() == 0), rtol=1e-6, atol=0)


def _sr_gpu(case, storage, seed):
    g = build_gpu(case, storage, bind=False)
    g.rounding("stochastic", seed)
    g.bind(storage)
    return g


@pytest.mark.parametrize("storage", STORAGES)
def test_stochastic_rounding_matches_oracle(storage):
    """Stochastic rounding moves a value to one of its two neighbouring
    16-bit numbers: a relative error below 2 eps per rounding, twice the
    nearest bound, so the bounds of the nearest test double."""
    eps = EPS[storage]
    case = sc_solute_case(96, 64, 41, react=True, bmax=1e30, q=9)
    o, g = build_oracle(case), _sr_gpu(case, storage, 7)
    o.iteration(200)
    g.iteration(200)
    er, eu = _fluid_errs(g, o, 2)
    Cg, bg = g.solute_state()
    Co, bo = o.solute_state()
    ec, eb = rel_err(Cg, Co), rel_err(bg, bo)
    print(f"{storage} stochastic: rho {er:.2e} u {eu:.2e} C {ec:.2e} b {eb:.2e} (eps {eps:.1e})")
    assert er <= 4 * eps and eu <= 40 * eps and ec <= 8 * eps and eb <= 8 * eps


def test_stochastic_rounding_is_keyed_on_seed_and_step():
    """The random words depend on the seed, the node and the step count
    only: one run of 150 steps equals runs of 70 + 80 and 1 + 149 steps;
    another seed gives other populations."""
    case = sc_solute_case(50, 30, 5, react=True, kr=0.02, q=4)
    runs = {}
    for key, seed, chunks in (("a", 5, (150,)), ("b", 5, (70, 80)), ("c", 5, (1, 149)), ("d", 6, (150,))):
        g = _sr_gpu(case, "bf16", seed)
        for n in chunks:
            g.iteration(n)
        runs[key] = [g.get_populations(c) for c in (0, 1, -1)]
        g.close()
    for k in ("b", "c"):
        assert all(np.array_equal(x, y) for x, y in zip(runs["a"], runs[k])), k
    assert not any(np.array_equal(x, y) for x, y in zip(runs["a"], runs["d"]))


def _mass_drift(case, storage, rounding, steps, comps):
    g = build_gpu(case, storage, bind=False)
    g.rounding(rounding, 3)
    g.bind(storage)
    b0 = g.budgets()
    g.iteration(steps)
    b1 = g.budgets()
    g.close()
    return max(abs(b1[f"mass{c}"] - b0[f"mass{c}"]) / b0[f"mass{c}"] for c in comps)


@pytest.mark.parametrize("which", ["two_fluids", "psi_phase"])
@pytest.mark.parametrize("storage", STORAGES)
def test_stochastic_rounding_keeps_mass_over_long_runs(storage, which):
    """Rounding to nearest is biased once the state is nearly steady (the
    same values round the same way step after step), so mass drifts by
    many eps over 10^4 steps; stochastic rounding is unbiased and the
    drift stays a small random walk: at least ten times smaller, and below
    eps / 2."""
    if which == "two_fluids":
        case, comps = sc_solute_case(96, 64, 11, react=False, openings=False), (0, 1)
    else:
        case, comps = phase_case(70, 45, 31), (0,)
    rne = _mass_drift(case, storage, "nearest", 10000, comps)
    sr = _mass_drift(case, storage, "stochastic", 10000, comps)
    print(f"{storage} {which}: mass drift nearest {rne:.2e}, stochastic {sr:.2e} (eps {EPS[storage]:.1e})")
    assert sr <= rne / 10 and sr <= EPS[storage] / 2


@pytest.mark.parametrize("storage", STORAGES)
def test_stochastic_rounding_with_extended_features(storage):
    """Stochastic rounding through the extended step (openings between slip
    walls, the psi forces, intersolute): the doubled nearest bounds."""
    eps = EPS[storage]
    case = channel_flow_case(60, 31, 4, inlet=("uniform", 0.04, 1.0))
    case["style"] = ("slip", 1.0)
    o, g = build_oracle(case), _sr_gpu(case, storage, 5)
    o.iteration(300)
    g.iteration(300)
    er, eu = _fluid_errs(g, o, 1)
    assert er <= 4 * eps and eu <= 40 * eps
    case = phase_case(70, 45, 31)
    o, g = build_oracle(case), _sr_gpu(case, storage, 6)
    o.iteration(25)
    g.iteration(25)
    er2, eu2 = _fluid_errs(g, o, 1)
    assert er2 <= 4 * eps and eu2 <= 40 * eps
    case = intersolute_case(90, 70, 11, q=4, nd=4)
    o, g = build_oracle(case), _sr_gpu(case, storage, 7)
    o.iteration(100)
    g.iteration(100)
    Cg, _ = g.solute_state()
    Co, _ = o.solute_state()
    ec = rel_err(Cg, Co)
    print(f"{storage} stochastic: slip channel rho {er:.2e} u {eu:.2e}; psi rho {er2:.2e} u {eu2:.2e}; "
          f"intersolute C {ec:.2e} (eps {eps:.1e})")
    assert ec <= 16 * eps
