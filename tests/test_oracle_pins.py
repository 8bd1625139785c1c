"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: identities
of the equilibrium printed with the fluids command, exact invariants of the
scheme, closed-form solutions (Poiseuille, diffusion spreading, a reactive
diffusion slab), the paper's own worked numbers (tests/golden/), Laplace's
law, and brute-force statistics of the growth rule.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import Oracle
from oracle import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------- equilibrium

@pytest.mark.parametrize("k", range(4))
def test_equilibrium_moments_match_fluids_command(k):
    """sum f_eq = rho, sum f_eq e = rho u, sum f_eq e e = rho cs^2 I + rho u u
    with cs^2 = (3/5)(1 - alpha) as printed with the fluids command."""
    g = golden("fluids_alpha.json")
    alpha, cs2 = g["alphas"][k], g["cs2"][k]
    rng = np.random.default_rng(k)
    for _ in range(20):
        rho = rng.uniform(0.05, 30.0)
        ux, uy = rng.uniform(-0.1, 0.1, 2)
        f = np.array([orc.feq(i, rho, ux, uy, alpha) for i in range(9)])
        assert abs(f.sum() - rho) <= 1e-14 * rho
        assert abs((f * EX).sum() - rho * ux) <= 1e-14 * rho
        assert abs((f * EY).sum() - rho * uy) <= 1e-14 * rho
        assert abs((f * EX * EX).sum() - (rho * cs2 + rho * ux * ux)) <= 1e-13 * rho
        assert abs((f * EY * EY).sum() - (rho * cs2 + rho * uy * uy)) <= 1e-13 * rho
        assert abs((f * EX * EY).sum() - rho * ux * uy) <= 1e-13 * rho


def test_equilibrium_alpha_default_is_eq_eq():
    """alpha = 4/9 reproduces Eq. (eq) with cs^2 = 1/3 (A_i = 1)."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rho, ux, uy = 1.3, 0.03, -0.02
    for i in range(9):
        eu = EX[i] * ux + EY[i] * uy
        ref = w[i] * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))
        assert orc.feq(i, rho, ux, uy, 4 / 9) == pytest.approx(ref, rel=1e-15, abs=1e-17)


def test_solute_equilibrium_is_linear_and_conserving():
    """Eq. (ueq) for D2Q4: g_i = C/4 (1 + 2 e.u); the D2Q9 form has the same
    zeroth and first moments (C and C u)."""
    C, ux, uy = 0.7, 0.02, -0.01
    for i in range(1, 5):
        eu = EX[i] * ux + EY[i] * uy
        assert orc.geq(4, i, C, ux, uy) == pytest.approx(C / 4 * (1 + 2 * eu), rel=1e-15)
    for q, idx in ((4, range(1, 5)), (9, range(9))):
        g = np.array([orc.geq(q, i, C, ux, uy) for i in idx])
        e = np.array(list(idx))
        assert g.sum() == pytest.approx(C, rel=1e-15)
        assert (g * EX[e]).sum() == pytest.approx(C * ux, rel=1e-13)
        assert (g * EY[e]).sum() == pytest.approx(C * uy, rel=1e-13)


# ------------------------------------------------------------ stream + walls

def _frozen(nx, ny):
    """A lattice whose collision changes nothing (tau so large that
    (f - f_eq)/tau is below half an ulp of f): a pure streaming operator."""
    o = Oracle(nx, ny)
    o.fluids(1, 1e300)
    return o


def test_streaming_moves_e1_by_one_node_in_x():
    """Velocity numbering: e1 = (1,0), e2 = (0,1), e5 = (1,1)."""
    o = _frozen(7, 5)
    f = np.ones((9, 5, 7))
    f[1, 2, 3] = 2.0
    f[2, 2, 3] = 3.0
    f[5, 2, 3] = 4.0
    o.set_f(f)
    o.iteration(1)
    g = o.get_f()
    assert g[1, 2, 4] == 2.0 and g[2, 3, 3] == 3.0 and g[5, 3, 4] == 4.0
    assert g.sum() == f.sum() and (g == 1.0).sum() == g.size - 3


def test_streaming_is_periodic_permutation():
    """Without obstacles, after lcm(nx, ny) steps every value returns bitwise."""
    nx, ny = 6, 4
    o = _frozen(nx, ny)
    f0 = np.random.default_rng(1).uniform(0, 1, (9, ny, nx))
    o.set_f(f0)
    o.iteration(1)
    assert not np.array_equal(o.get_f(), f0)
    o.iteration(math.lcm(nx, ny) - 1)
    assert np.array_equal(o.get_f(), f0)


def test_half_way_bounce_back_reverses_at_wall():
    """noslip: a population sent towards a solid neighbour comes back to the
    sender reversed after one step (boundary_style noslip)."""
    o = _frozen(6, 5)
    o.obstacle_rect(4, 4, 0, 4)           # solid column x = 4
    f = np.ones((9, 5, 6))
    f[:, :, 4] = 0.0
    f[1, 2, 3] = 2.0                       # moving +x from x = 3 into the wall
    f[5, 2, 3] = 3.0                       # moving (+1,+1) into (4, 3), solid
    o.set_f(f)
    o.iteration(1)
    g = o.get_f()
    assert g[3, 2, 3] == 2.0               # back as e3 at the same node
    assert g[7, 2, 3] == 3.0               # back as e7
    assert g.sum() == f.sum()


def test_streaming_preserves_values_with_obstacles():
    """With bounce-back the stream operator is still a permutation of the
    fluid populations: the multiset of values is kept exactly."""
    nx, ny = 9, 7
    o = _frozen(nx, ny)
    o.obstacle_circle(4, 3, 1.5)
    m = o.get_mask().astype(bool)
    f0 = np.random.default_rng(2).uniform(0, 1, (9, ny, nx))
    f0[:, m] = 0.0
    o.set_f(f0)
    for _ in range(5):
        o.iteration(1)
        assert np.array_equal(np.sort(o.get_f().ravel()), np.sort(f0.ravel()))


# ----------------------------------------------------------------- invariants

def test_mass_exact_with_bounce_back_and_forcing():
    nx, ny = 40, 30
    o = Oracle(nx, ny)
    o.fluids(1, 0.7)
    for xc, yc, r in ((10, 10, 4.5), (30, 20, 6.0), (25, 5, 3.0)):
        o.obstacle_circle(xc, yc, r)
    o.aveacceleration(1, 1e-4)
    rng = np.random.default_rng(3)
    o.set_fields(0, 1.0 + 0.05 * rng.uniform(-1, 1, nx * ny),
                 0.02 * rng.uniform(-1, 1, nx * ny), 0.02 * rng.uniform(-1, 1, nx * ny))
    m0 = o.budgets()["mass0"]
    o.iteration(400)
    assert abs(o.budgets()["mass0"] - m0) <= 1e-12 * m0


def test_momentum_grows_by_total_force_per_step():
    """Periodic box, one fluid: the velocity shift adds exactly F per node
    and step to the post-collision momentum (aveforce along e5 = (v, v))."""
    nx, ny = 12, 10
    o = Oracle(nx, ny)
    o.fluids(1, 0.9)
    o.aveforce(5, 2e-5)
    o.aveforce(1, 1e-5)
    rng = np.random.default_rng(4)
    o.set_fields(0, 1 + 0.1 * rng.uniform(-1, 1, nx * ny), 0.01 * rng.uniform(-1, 1, nx * ny), 0.0)
    b0 = o.budgets()
    o.iteration(50)
    b1 = o.budgets()
    n = nx * ny
    assert b1["mom_x"] - b0["mom_x"] == pytest.approx(50 * n * 3e-5, rel=1e-10)
    assert b1["mom_y"] - b0["mom_y"] == pytest.approx(50 * n * 2e-5, rel=1e-10)


def test_two_component_shan_chen_conserves_total_momentum():
    """Pair forces are antisymmetric: sum_x (F_A + F_B) = 0 on a periodic box."""
    nx, ny = 16, 14
    o = Oracle(nx, ny)
    o.fluids(2, 1.0, 0.8)
    o.interforce(1.7)
    rng = np.random.default_rng(5)
    o.set_fields(0, rng.uniform(0.1, 1.0, nx * ny))
    o.set_fields(1, rng.uniform(0.1, 1.0, nx * ny))
    b0 = o.budgets()
    o.iteration(30)
    b1 = o.budgets()
    assert abs(b1["mom_x"] - b0["mom_x"]) < 1e-12
    assert abs(b1["mom_y"] - b0["mom_y"]) < 1e-12
    assert b1["mass0"] == pytest.approx(b0["mass0"], rel=1e-13)
    assert b1["mass1"] == pytest.approx(b0["mass1"], rel=1e-13)


# --------------------------------------------------------------------- forces

def test_shan_chen_force_is_gradient_of_other_component():
    """For a quadratic density field, sum_i w_i rho(x + e_i) e_i is exactly
    grad(rho)/3 (odd moments of the D2Q9 weights vanish), so the interforce
    formula gives F_A = -G rho_A grad(rho_B) / 3 in the interior."""
    nx, ny = 20, 18
    G = 0.9
    o = Oracle(nx, ny)
    o.fluids(2, 1.0, 1.0)
    o.interforce(G)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    rho_b = 1.0 + 0.01 * x + 0.02 * y + 0.001 * x * x - 0.0005 * x * y + 0.0007 * y * y
    rho_a = 0.3 + 0.0 * x
    o.set_fields(0, rho_a)
    o.set_fields(1, rho_b)
    Fx, Fy = o.forces(0)
    gx = 0.01 + 0.002 * x - 0.0005 * y
    gy = 0.02 - 0.0005 * x + 0.0014 * y
    sl = (slice(1, ny - 1), slice(1, nx - 1))
    np.testing.assert_allclose(Fx[sl], -G * 0.3 * gx[sl] / 3, rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(Fy[sl], -G * 0.3 * gy[sl] / 3, rtol=1e-12, atol=1e-16)


def test_adhesion_next_to_flat_wall():
    """Node above a solid row: sum_i w_i s(x + e_i) e_i = (0, -1/6), so the
    adhesiveforce formula gives F = +G_c rho_c / 6 along +y (away from the
    wall for G_c > 0)."""
    nx, ny = 10, 8
    o = Oracle(nx, ny)
    o.fluids(2, 1.0, 1.0)
    o.adhesiveforce(0.3, 0)
    o.adhesiveforce(-0.3, 1)
    o.obstacle_rect(0, nx - 1, 0, 0)
    o.set_fields(0, 0.8)
    o.set_fields(1, 0.2)
    for comp, G, rho in ((0, 0.3, 0.8), (1, -0.3, 0.2)):
        Fx, Fy = o.forces(comp)
        np.testing.assert_allclose(Fy[1, :], G * rho / 6, rtol=1e-14)
        np.testing.assert_allclose(Fx[1, :], 0.0, atol=1e-17)
        np.testing.assert_allclose(Fy[3, :], 0.0, atol=1e-17)


# ------------------------------------------------------------------ Poiseuille

def test_poiseuille_application_matches_eq_profile():
    """The paper's Poiseuille application (golden numbers): g from the printed
    formula equals the printed 1.11e-4, and after 10000 steps the profile is
    Eq. (profile) with u_max = 0.07."""
    g = golden("poiseuille_application.json")
    Nx, Ny, tau, umax = g["Nx"], g["Ny"], g["tau"], g["u_max"]
    acc = 4.0 / 3.0 * umax * (2 * tau - 1) / (Ny - 1) ** 2
    assert acc == pytest.approx(g["g_printed"], rel=2e-3)
    o = Oracle(Nx + 1, Ny + 1)
    o.fluids(1, tau)
    o.obstacle_rect(0, Nx, 0, 0)
    o.obstacle_rect(0, Nx, Ny, Ny)
    o.aveacceleration(1, acc)
    # Initial populations 4 (rest and slow modes) and 1 (fast modes):
    # rho = 24 at rest, not the rest equilibrium; set them as given.
    init = np.array([g["pop_rest_slow"]] * 5 + [g["pop_fast"]] * 4)
    f0 = np.broadcast_to(init[:, None, None], (9, Ny + 1, Nx + 1)).copy()
    f0[:, 0, :] = 0.0
    f0[:, Ny, :] = 0.0
    o.set_f(f0)
    assert o.budgets()["mass0"] == pytest.approx(24.0 * (Nx + 1) * (Ny - 1))
    o.iteration(g["steps"])
    _, ux, _ = o.moments(0)
    y = np.arange(1, Ny)
    prof = 3 * acc / (2 * tau - 1) * (((Ny - 1) / 2) ** 2 - (y - Ny / 2) ** 2)
    assert prof.max() == pytest.approx(umax, rel=2e-3)
    np.testing.assert_allclose(ux[1:Ny, 7], prof, atol=5e-3 * umax)
    # u_x is uniform along the periodic x axis
    assert np.ptp(ux[1:Ny, :], axis=1).max() < 1e-12


def test_poiseuille_start_up_series_128x64():
    """Channel of 128x64 nodes, walls at y = 0.5 and 62.5 (H = 62), g = 1e-6,
    tau = 1 (nu = 1/6), 5000 steps: compare with the start-up solution of the
    force-driven channel, u = g/(2 nu) [(H/2)^2 - eta^2]
    - sum_{n odd} 4 g H^2 / (nu pi^3 n^3) sin(n pi xi / H) exp(-nu n^2 pi^2 t / H^2)."""
    nx, ny, acc, tau, steps = 128, 64, 1e-6, 1.0, 5000
    o = Oracle(nx, ny)
    o.fluids(1, tau)
    o.obstacle_rect(0, nx - 1, 0, 0)
    o.obstacle_rect(0, nx - 1, ny - 1, ny - 1)
    o.aveacceleration(1, acc)
    o.set_fields(0, 1.0)
    m0 = o.budgets()["mass0"]
    o.iteration(steps)
    assert abs(o.budgets()["mass0"] - m0) <= 1e-12 * m0
    _, ux, _ = o.moments(0)
    nu = (tau - 0.5) / 3
    H = ny - 2.0
    y = np.arange(1, ny - 1, dtype=float)
    xi = y - 0.5
    eta = y - (ny - 1) / 2
    u = acc / (2 * nu) * ((H / 2) ** 2 - eta ** 2)
    for n in range(1, 200, 2):
        u -= 4 * acc * H ** 2 / (nu * math.pi ** 3 * n ** 3) * np.sin(n * math.pi * xi / H) \
            * math.exp(-nu * n * n * math.pi ** 2 * steps / H ** 2)
    umax = acc * H * H / (8 * nu)
    assert ux[1:-1, 0].max() == pytest.approx(0.882 * umax, rel=2e-2)
    np.testing.assert_allclose(ux[1:-1, 0], u, atol=2e-3 * umax)


def test_poiseuille_steady_second_difference():
    """At steady state the bulk profile is exactly quadratic with second
    difference -g/nu (nu = (tau - 1/2)/3, Matlab script of the Scripts
    section)."""
    nx, ny, acc, tau = 4, 18, 1e-5, 0.8
    o = Oracle(nx, ny)
    o.fluids(1, tau)
    o.obstacle_rect(0, nx - 1, 0, 0)
    o.obstacle_rect(0, nx - 1, ny - 1, ny - 1)
    o.aveacceleration(1, acc)
    o.set_fields(0, 1.0)
    o.iteration(8000)
    _, ux, _ = o.moments(0)
    u = ux[:, 1]
    d2 = u[3:ny - 1] - 2 * u[2:ny - 2] + u[1:ny - 3]
    nu = (tau - 0.5) / 3
    np.testing.assert_allclose(d2, -acc / nu, rtol=1e-8)


# ---------------------------------------------------------- solute transport

def _variance_closed_form(n, tau_s, cs2):
    lam = 1.0 - 1.0 / tau_s
    return cs2 * (n * (2 * tau_s - 1) - 2 * lam * (1 - lam ** n) / (1 - lam) ** 2)


@pytest.mark.parametrize("q,cs2", [(9, 1.0 / 3.0), (4, 0.5)])
@pytest.mark.parametrize("tau_s", [0.7, 1.0, 1.6])
def test_solute_spreading_variance_closed_form(q, cs2, tau_s):
    """Equilibrium start at rest: Var_x(n) - Var_x(0)
    = cs^2 [n (2 tau_s - 1) - 2 lam (1 - lam^n) / (1 - lam)^2], lam = 1 - 1/tau_s
    (moment recursion of the BGK solute scheme; long-time slope 2D with
    D = cs^2 (tau_s - 1/2), which is the solute command's D for Q = 4)."""
    nx, ny, nsteps = 160, 3, 60
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.solute(tau_s, q)
    C = np.zeros((ny, nx))
    C[:, 80] = 1.0
    C[:, 81] = 0.5
    o.set_fields(0, 1.0)
    o.set_concentration(C)
    x = np.arange(nx, dtype=float)

    def var():
        c, _ = o.solute_state()
        p = c.sum(axis=0)
        m = p.sum()
        mu = (p * x).sum() / m
        return (p * x * x).sum() / m - mu * mu, m, mu

    v0, m0, mu0 = var()
    o.iteration(nsteps)
    v1, m1, mu1 = var()
    assert m1 == pytest.approx(m0, rel=1e-14)
    assert mu1 == pytest.approx(mu0, abs=1e-12)
    assert v1 - v0 == pytest.approx(_variance_closed_form(nsteps, tau_s, cs2), rel=1e-11)


@pytest.mark.parametrize("q", [9, 4])
def test_solute_advection_mean_moves_by_u(q):
    """Uniform solvent velocity u and equilibrium start: the centre of mass
    moves by exactly u per step (first moment of g_eq is C u)."""
    nx, ny, nsteps = 120, 4, 40
    ux, uy = 0.05, 0.0
    o = Oracle(nx, ny)
    o.fluids(1, 0.9)
    o.solute(0.8, q)
    o.set_fields(0, 1.0, ux, uy)
    C = np.zeros((ny, nx))
    C[:, 40:44] = 1.0
    o.set_concentration(C, ux, uy)
    x = np.arange(nx, dtype=float)
    c0, _ = o.solute_state()
    o.iteration(nsteps)
    c1, _ = o.solute_state()
    mu0 = (c0.sum(0) * x).sum() / c0.sum()
    mu1 = (c1.sum(0) * x).sum() / c1.sum()
    assert mu1 - mu0 == pytest.approx(nsteps * ux, rel=1e-10)


def test_damkohler_numbers_of_surface_growth_application():
    """D2Q4, tau_s = 1: the measured diffusion coefficient is 1/4 and
    Da = k_r L / D with L = 200 gives the printed 4, 20, 40, 80."""
    g = golden("surface_growth_damkohler.json")
    n = 400
    v = _variance_closed_form(n, g["tau_s"], 0.5)
    D_measured = v / (2 * n)
    o = Oracle(300, 3)
    o.fluids(1, 1.0)
    o.solute(g["tau_s"], 4)
    C = np.zeros((3, 300))
    C[:, 150] = 1.0
    o.set_fields(0, 1.0)
    o.set_concentration(C)
    o.iteration(100)
    c, _ = o.solute_state()
    p = c.sum(0)
    x = np.arange(300.0)
    mu = (p * x).sum() / p.sum()
    var = (p * (x - mu) ** 2).sum() / p.sum()
    assert var == pytest.approx(_variance_closed_form(100, 1.0, 0.5), rel=1e-11)
    assert D_measured == pytest.approx(0.25, rel=1e-12)
    for kr, Da in zip(g["kr"], g["Da"]):
        assert kr * g["L"] / D_measured == pytest.approx(Da, rel=1e-12)


# ------------------------------------------------------------- reactive wall

@pytest.mark.parametrize("g_out", [0.0, 0.013, 0.21, 1.7])
@pytest.mark.parametrize("kr,Cs", [(0.25, 1.0), (5e-3, 0.5), (0.1, 0.0)])
def test_reactive_link_reduces_to_d2q4_rule(g_out, kr, Cs):
    """For Q = 4 the per-link rule is the surface_reaction command's
    C = (2 g_chi + kr Cs)/(kr + 1/2), g_i = -g_chi + C/2, with deposit
    kr (C - Cs) when positive (else plain bounce-back)."""
    for i in range(1, 5):
        db, gi = orc.reactive_link(4, i, kr, Cs, g_out)
        C = (2 * g_out + kr * Cs) / (kr + 0.5)
        if kr * (C - Cs) > 0:
            assert gi == pytest.approx(-g_out + C / 2, rel=1e-14, abs=1e-17)
            assert db == pytest.approx(kr * (C - Cs), rel=1e-13, abs=1e-17)
        else:
            assert gi == g_out and db == 0.0


@pytest.mark.parametrize("q", [9, 4])
def test_reactive_slab_steady_state_closed_form(q):
    """1-D slab: Dirichlet C = 1 at x = 0, reactive solid column at x = nx-1
    (half-way wall at x_w = nx - 1.5), at rest.  The steady state is exactly
    linear, C = 1 + b x, with the diffusive flux -D b equal to the reaction
    flux k_r (C(x_w) - C_s): b = -k_r (1 - C_s) / (D + k_r x_w)."""
    nx, ny, kr, Cs, tau_s = 16, 3, 0.05, 0.2, 1.0
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.solute(tau_s, q)
    o.solute_opening("xlo", "dirichlet", 1.0)
    o.solute_opening("xhi", "adiabatic")       # behind the solid column
    o.obstacle_rect(nx - 1, nx - 1, 0, ny - 1)
    o.surface_reaction(kr, Cs, 0.0, 1e300, 1)
    o.set_fields(0, 1.0)
    C0 = np.full((ny, nx), 0.5)
    o.set_concentration(C0)
    o.iteration(20000)
    C, b = o.solute_state()
    D = (tau_s - 0.5) / 3 if q == 9 else (tau_s - 0.5) / 2
    xw = nx - 1.5
    slope = -kr * (1 - Cs) / (D + kr * xw)
    x = np.arange(nx - 1, dtype=float)
    np.testing.assert_allclose(C[:, :nx - 1], np.broadcast_to(1 + slope * x, (ny, nx - 1)),
                               rtol=1e-10)
    # deposit per step on the wall equals the diffusive flux through it
    bud0 = o.budgets()
    dep0 = b.sum()
    o.iteration(10)
    _, b1 = o.solute_state()
    assert (b1.sum() - dep0) / 10 == pytest.approx(-D * slope * ny, rel=1e-9)
    bud1 = o.budgets()
    assert (bud1["inflow"] - bud1["outflow"]) - (bud0["inflow"] - bud0["outflow"]) == \
        pytest.approx(b1.sum() - dep0, rel=1e-9)


def test_solute_budget_closes_with_growth():
    """sum C + sum b + removed solute + deposits consumed by growth
    - b0 per grown node = initial + inflow - outflow (FP64, exact up to
    rounding) in a run where nodes grow; fluid mass + removed is kept."""
    nx, ny = 40, 24
    o = Oracle(nx, ny)
    o.fluids(2, 1.0, 1.0)
    o.interforce(0.9)
    o.adhesiveforce(0.3, 0)
    o.adhesiveforce(-0.3, 1)
    o.obstacle_circle(20, 12, 4.0)
    o.obstacle_circle(30, 4, 3.0)
    o.solute(0.7, 9)
    o.solute_opening("xlo", "dirichlet", 1.0)
    o.solute_opening("xhi", "adiabatic")
    o.surface_reaction(0.2, 0.0, 0.01, 0.05, 7)
    rng = np.random.default_rng(8)
    o.set_fields(0, rng.uniform(0.05, 1.0, nx * ny))
    o.set_fields(1, rng.uniform(0.05, 1.0, nx * ny))
    o.set_concentration(0.3)
    b0 = o.budgets()
    o.iteration(300)
    b1 = o.budgets()
    assert b1["grown_nodes"] > 0
    lhs = (b1["solute"] + b1["deposit"] + b1["removed_solute"] + b1["consumed_deposit"]
           - 0.01 * b1["grown_nodes"])
    rhs = b0["solute"] + b0["deposit"] + b1["inflow"] - b1["outflow"]
    assert lhs == pytest.approx(rhs, rel=1e-12)
    for c in (0, 1):
        assert b1[f"mass{c}"] + b1[f"removed_mass{c}"] == pytest.approx(b0[f"mass{c}"], rel=1e-12)


# --------------------------------------------------------------------- growth

def test_growth_flips_the_hashed_neighbour():
    """5x5 box, one solid node with b > b_max: exactly one of its direct
    fluid neighbours (E,N,W,S order) becomes solid -- the one the
    counter-based hash picks -- b resets to 0, the new solid gets b0 and its
    fluid and solute mass is tallied as removed."""
    for seed in range(12):
        o = Oracle(5, 5)
        o.fluids(1, 1.0)
        o.solute(1.0, 9)
        o.obstacle_rect(2, 2, 2, 2)
        o.obstacle_rect(2, 2, 3, 3)          # N neighbour solid: 3 candidates
        o.surface_reaction(0.0, 0.0, 0.25, 1.0, seed)
        o.set_fields(0, 1.0)
        o.set_concentration(0.4)
        b = np.zeros((5, 5))
        b[2, 2] = 1.5
        b[3, 2] = 0.25
        o.set_b(b)
        o.iteration(1)
        cands = [(3, 2), (1, 2), (2, 1)]    # (x, y) of E, W, S
        h = orc.splitmix64(seed ^ (1 * 25 + 2 * 5 + 2))
        tx, ty = cands[orc.pick(h, 3)]
        m = o.get_mask()
        expect = np.zeros((5, 5), np.uint8)
        expect[2, 2] = expect[3, 2] = 1
        expect[ty, tx] = 1
        assert np.array_equal(m, expect)
        bb = o.get_b()
        assert bb[2, 2] == 0.0 and bb[ty, tx] == 0.25 and bb[3, 2] == 0.25
        bud = o.budgets()
        assert bud["grown_nodes"] == 1
        assert bud["removed_mass0"] == pytest.approx(1.0, rel=1e-14)
        assert bud["removed_solute"] == pytest.approx(0.4, rel=1e-14)


def test_growth_choice_is_equiprobable():
    """Chi-square over many hashed picks among m candidates (surface_reaction:
    every occurrence is equiprobable)."""
    from scipy.stats import chisquare
    for m in (2, 3, 4):
        counts = np.zeros(m)
        for s in range(60000):
            counts[orc.pick(orc.splitmix64(0xC0FFEE ^ (7 * 1000003 + s)), m)] += 1
        assert chisquare(counts).pvalue > 1e-3


def test_growth_run_is_deterministic():
    def run():
        o = Oracle(24, 20)
        o.fluids(1, 1.0)
        o.obstacle_circle(12, 10, 3.0)
        o.solute(1.0, 9)
        o.surface_reaction(0.1, 0.5, 0.5, 1.0, 99)
        o.set_fields(0, 1.0)
        o.set_concentration(1.5)
        o.iteration(400)
        return o.get_mask(), o.get_b(), o.budgets()
    m1, b1, d1 = run()
    m2, b2, d2 = run()
    assert d1["grown_nodes"] > 3
    assert np.array_equal(m1, m2) and np.array_equal(b1, b2) and d1 == d2


# -------------------------------------------------------------------- Laplace

@pytest.mark.slow
def test_laplace_law_two_component_droplets():
    """Laplace's law for converged two-component Shan-Chen droplets: the
    pressure jump with p = (rho_A + rho_B + G rho_A rho_B)/3 is sigma / R.
    Droplets start at the bulk densities of a converged flat interface (so
    they only adjust to their curvature) and are converged after 10^4
    steps (the jump moves by less than 1e-3 relative over the last 2000);
    dp R is then the same for R = 8, 12 and 16 within 2 %, and a linear fit
    in 1/R passes within 2 % of the smallest jump through the origin."""
    from cases import droplet_fields, flat_coexistence, laplace_jump
    n, G = 64, 2.6
    hi, lo = flat_coexistence(G)
    assert hi > 1.0 and lo < 0.01
    inv_r, dp = [], []
    for R in (8.0, 12.0, 16.0):
        o = Oracle(n, n)
        o.fluids(2, 1.0, 1.0)
        o.interforce(G)
        ra0, rb0 = droplet_fields(n, R, hi, lo)
        o.set_fields(0, ra0)
        o.set_fields(1, rb0)
        jumps = []
        for steps in (8000, 2000):
            o.iteration(steps)
            Re, jump = laplace_jump(o.moments(0)[0], o.moments(1)[0], G)
            jumps.append(jump)
        assert abs(jumps[1] / jumps[0] - 1.0) < 1e-3
        inv_r.append(1.0 / Re)
        dp.append(jumps[1])
    sig = np.array(dp) / np.array(inv_r)
    assert sig.max() / sig.min() - 1.0 <= 0.02
    slope, icpt = np.polyfit(inv_r, dp, 1)
    assert slope > 0 and abs(icpt) <= 0.02 * min(dp)


# ----------------------------------------------------------- rasterisation

def test_circle_rasterisation_counts():
    """obstacle(circle): solid iff dx^2 + dy^2 <= r^2 (integer lattice
    points in a disc; Gauss circle counts for r^2 = 1, 2, 4, 5, 25)."""
    for r2, count in ((1, 5), (2, 9), (4, 13), (5, 21), (25, 81)):
        o = Oracle(31, 31)
        o.obstacle_circle(15, 15, math.sqrt(r2) if r2 != 25 else 5.0)
        assert int(o.get_mask().sum()) == count
    # minimum image across the periodic edge
    o = Oracle(20, 20)
    o.obstacle_circle(0, 0, 1.0)
    m = o.get_mask()
    assert m[0, 0] and m[0, 19] and m[19, 0] and m[0, 1] and m[1, 0] and m.sum() == 5


def test_results_do_not_depend_on_thread_count():
    """Row loops run in parallel; every reduction is ordered, so 1 and many
    threads give bitwise the same state and budgets."""
    def run(threads):
        orc.set_threads(threads)
        o = Oracle(40, 30)
        o.fluids(2, 1.0, 0.8)
        o.interforce(1.2)
        o.adhesiveforce(0.2, 0)
        o.obstacle_circle(20, 15, 4.0)
        o.solute(0.8, 9)
        o.solute_opening("xlo", "dirichlet", 1.0)
        o.solute_opening("xhi", "adiabatic")
        o.surface_reaction(0.05, 0.0, 0.0, 0.02, 3)
        rng = np.random.default_rng(9)
        o.set_fields(0, rng.uniform(0.1, 1.0, 1200))
        o.set_fields(1, rng.uniform(0.1, 1.0, 1200))
        o.set_concentration(0.1)
        o.iteration(120)
        return o.get_f(0), o.get_g(), o.get_mask(), o.budgets()
    n0 = orc.set_threads(0)
    try:
        a, b = run(1), run(max(2, n0))
    finally:
        orc.set_threads(n0)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert a[3] == b[3]


# ------------------------------------------- one-component Shan-Chen (psi)

def _psi(rho, psi0, rho0):
    return psi0 * np.exp(-rho0 / rho)


def test_psi_cohesion_is_psi_gradient():
    """interforce(G, psi0, rho0), one component: for psi quadratic in x, y the
    stencil sum_i w_i psi(x + e_i) e_i is exactly grad(psi)/3, so the force is
    -G psi grad(psi)/3.  The density field is built from the inverse of
    psi = psi0 exp(-rho0/rho)."""
    nx, ny, G, psi0, rho0 = 20, 18, -120.0, 4.0, 200.0
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    psi = 1.2 + 0.01 * x + 0.015 * y + 0.0008 * x * x - 0.0004 * x * y + 0.0006 * y * y
    rho = -rho0 / np.log(psi / psi0)
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.interforce(G, psi0, rho0)
    o.set_fields(0, rho)
    Fx, Fy = o.forces(0)
    gx = 0.01 + 0.0016 * x - 0.0004 * y
    gy = 0.015 - 0.0004 * x + 0.0012 * y
    sl = (slice(1, ny - 1), slice(1, nx - 1))
    np.testing.assert_allclose(Fx[sl], -G * psi[sl] * gx[sl] / 3, rtol=1e-10)
    np.testing.assert_allclose(Fy[sl], -G * psi[sl] * gy[sl] / 3, rtol=1e-10)


def test_psi_adhesion_next_to_flat_wall():
    """adhesiveforce(G, psi0, rho0), one component: a node beside a flat
    solid row has sum_i w_i s(x + e_i) e_i = -n/6 (n: unit normal into the
    fluid), so F = +G psi n / 6: towards the wall for G < 0."""
    nx, ny, G, psi0, rho0 = 10, 8, -250.0, 4.0, 200.0
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.adhesiveforce(G, psi0=psi0, rho0=rho0)
    o.obstacle_rect(0, nx - 1, 0, 0)
    o.set_fields(0, 300.0)
    Fx, Fy = o.forces(0)
    p = _psi(300.0, psi0, rho0)
    np.testing.assert_allclose(Fy[1], G * p / 6, rtol=1e-13)        # above the wall: n = +y
    np.testing.assert_allclose(Fy[ny - 1], -G * p / 6, rtol=1e-13)  # below it (periodic): n = -y
    assert np.all(Fx == 0.0) and np.all(Fy[2:ny - 1] == 0.0)


def test_psi_cohesion_conserves_momentum():
    """The cohesion sum pairs each link with its opposite, so over a periodic
    box without solids the forces add to zero and the total momentum of a
    separating fluid stays at its initial value (zero)."""
    nx, ny = 48, 40
    rng = np.random.default_rng(9)
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.interforce(-120.0, 4.0, 200.0)
    o.set_fields(0, 200.0 + rng.uniform(0, 1, nx * ny))
    b0 = o.budgets()
    o.iteration(300)
    b = o.budgets()
    _, ux, _ = o.moments(0)
    assert np.abs(ux).max() > 1e-3          # the fluid does move (separation)
    assert abs(b["mom_x"]) <= 1e-9 * b0["mass0"]
    assert abs(b["mom_y"]) <= 1e-9 * b0["mass0"]
    assert b["mass0"] == pytest.approx(b0["mass0"], rel=1e-13)


def test_flat_interface_has_equal_bulk_pressures():
    """Steady flat liquid-vapour interface of the one-component model: the
    cohesion force of a row is -(G/6) psi(y) (psi(y+1) - psi(y-1)), whose sum
    over an interface telescopes to -(G/6)(psi_l^2 - psi_g^2); the momentum
    balance with the bulk fluxes rho/3 then makes p = rho/3 + G psi^2/6 equal
    in both bulk phases.  Also the phases are distinct (a density ratio
    above 3).  The start is a smooth (tanh) slab: a step start also excites
    the lattice's period-2 momentum mode, whose j^2/rho adds to the bulk
    fluxes."""
    nx, ny, G, psi0, rho0 = 4, 128, -120.0, 4.0, 200.0
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.interforce(G, psi0, rho0)
    yy = np.repeat(np.arange(ny), nx).astype(float)
    o.set_fields(0, 86.0 + 438.0 * 0.5 * (np.tanh((yy - 32) / 3) - np.tanh((yy - 96) / 3)))
    o.iteration(40000)
    rho, _, _ = o.moments(0)
    rl, rg = rho[64].mean(), rho[0].mean()
    p = lambda r: r / 3 + G * _psi(r, psi0, rho0) ** 2 / 6
    assert rl > 3 * rg
    assert p(rl) == pytest.approx(p(rg), rel=1e-9)


def _perimeter_per_root_area(mask):
    m = mask.astype(int)
    per = (np.abs(np.diff(m, axis=0, append=m[:1])).sum()
           + np.abs(np.diff(m, axis=1, append=m[:, :1])).sum())
    return per / np.sqrt(m.sum())


def test_surface_growth_more_dendritic_with_damkohler():
    """The paper's surface-growth example (Fig. surface: 200 x 200, seed
    square 11 x 11, C0 = 1.5, Cs = 0.5, b0 = 0.5, bmax = 1, D2Q4 solute):
    the grown structure is less compact -- larger perimeter per square root
    of area -- as Da = kr L / D grows through 4, 20, 40, 80."""
    from cases import build_oracle, surface_growth_case
    shape = []
    for kr in (5e-3, 0.025, 0.05, 0.1):
        o = build_oracle(surface_growth_case(kr))
        o.iteration(4000)
        assert o.budgets()["grown_nodes"] > 1000
        shape.append(_perimeter_per_root_area(o.get_mask()))
    assert all(a < b for a, b in zip(shape, shape[1:])), shape


# ------------------------------------------------------ momentum openings

def _opening_channel(wall_in, style_in, nx=30, ny=24, tau=0.8, v=0.04, rho_out=1.0, outlet_style="dirichlet"):
    """Channel between two solid walls, flowing from wall_in to the opposite
    wall: inlet with style_in, outlet with outlet_style."""
    o = Oracle(nx, ny)
    o.fluids(1, tau)
    opp = {"xlo": "xhi", "xhi": "xlo", "ylo": "yhi", "yhi": "ylo"}[wall_in]
    if wall_in in ("xlo", "xhi"):
        o.obstacle_rect(0, nx - 1, 0, 0)
        o.obstacle_rect(0, nx - 1, ny - 1, ny - 1)
        lo, hi = 1, ny - 2
    else:
        o.obstacle_rect(0, 0, 0, ny - 1)
        o.obstacle_rect(nx - 1, nx - 1, 0, ny - 1)
        lo, hi = 1, nx - 2
    o.momentum_opening(wall_in, lo, hi, 0, "inlet", style_in, v, 1.0)
    o.momentum_opening(opp, lo, hi, 0, "outlet", outlet_style, 0.0, rho_out)
    o.set_fields(0, 1.0)
    return o, lo, hi, opp


def _line(a, wall):
    return {"xlo": a[:, 0], "xhi": a[:, -1], "ylo": a[0, :], "yhi": a[-1, :]}[wall]


@pytest.mark.parametrize("wall", ["xlo", "xhi", "ylo", "yhi"])
def test_velocity_inlet_and_pressure_outlet_hold_exactly(wall):
    """Zou-He closure (inlet_momentum command, App. A): after any step the
    inlet nodes move with exactly the prescribed velocity -- the paper's
    parabolic profile v(y) = 4 v_max/L^2 [(L/2)^2 - ((2y - y0 - y1)/2)^2],
    along the inward normal, zero tangential -- and the dirichlet outlet
    nodes hold exactly the prescribed density."""
    v, rho_out = 0.04, 0.995
    o, lo, hi, opp = _opening_channel(wall, "poiseuille", v=v, rho_out=rho_out)
    o.iteration(37)
    rho, ux, uy = o.moments(0)
    L = hi - lo + 1
    k = np.arange(lo, hi + 1)
    prof = 4 * v / L ** 2 * (L ** 2 / 4 - ((2 * k - lo - hi) / 2) ** 2)
    normal = {"xlo": (1, 0), "xhi": (-1, 0), "ylo": (0, 1), "yhi": (0, -1)}[wall]
    un = _line(ux, wall)[lo:hi + 1] * normal[0] + _line(uy, wall)[lo:hi + 1] * normal[1]
    ut = _line(ux, wall)[lo:hi + 1] * normal[1] + _line(uy, wall)[lo:hi + 1] * normal[0]
    np.testing.assert_allclose(un, prof, rtol=1e-12, atol=1e-16)
    assert np.abs(ut).max() <= 1e-15
    np.testing.assert_allclose(_line(rho, opp)[lo:hi + 1], rho_out, rtol=1e-14)
    # the flow has come through: the density changed inside
    assert np.abs(rho[rho != -11.0] - 1.0).max() > 1e-4


@pytest.mark.parametrize("wall", ["xhi", "ylo"])
def test_uniform_outlet_velocity_and_pressure_inlet(wall):
    """The reverse pairing: dirichlet inlet (rho 1.004) and a uniform
    velocity outlet (0.02 out of the domain)."""
    nx, ny = 26, 20
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    inlet = {"xhi": "xlo", "ylo": "yhi"}[wall]
    if wall == "xhi":
        o.obstacle_rect(0, nx - 1, 0, 0)
        o.obstacle_rect(0, nx - 1, ny - 1, ny - 1)
        lo, hi = 1, ny - 2
    else:
        o.obstacle_rect(0, 0, 0, ny - 1)
        o.obstacle_rect(nx - 1, nx - 1, 0, ny - 1)
        lo, hi = 1, nx - 2
    o.momentum_opening(inlet, lo, hi, 0, "inlet", "dirichlet", 0.0, 1.004)
    o.momentum_opening(wall, lo, hi, 0, "outlet", "uniform", 0.02, 1.0)
    o.set_fields(0, 1.0)
    o.iteration(23)
    rho, ux, uy = o.moments(0)
    out = {"xhi": ux[lo:hi + 1, -1], "ylo": -uy[0, lo:hi + 1]}[wall]
    np.testing.assert_allclose(out, 0.02, rtol=1e-12)
    np.testing.assert_allclose(_line(rho, inlet)[lo:hi + 1], 1.004, rtol=1e-14)


def test_gradient_outlet_extrapolates_populations():
    """Gradient style: after the collision each population of the outlet
    node equals 2 f(one node in) - f(two nodes in)."""
    o, lo, hi, opp = _opening_channel("xlo", "uniform", v=0.03, outlet_style="gradient")
    o.iteration(15)
    f = o.get_f(0)
    np.testing.assert_allclose(f[:, lo:hi + 1, -1], 2 * f[:, lo:hi + 1, -2] - f[:, lo:hi + 1, -3],
                               rtol=1e-13, atol=1e-15)


def test_openings_start_from_their_state():
    """The opening nodes start at equilibrium with the opening's density and
    velocity (the inlet/outlet commands override earlier settings)."""
    o, lo, hi, opp = _opening_channel("ylo", "uniform", v=0.03, rho_out=0.99)
    rho, ux, uy = o.moments(0)
    np.testing.assert_allclose(uy[0, lo:hi + 1], 0.03, rtol=1e-13)
    np.testing.assert_allclose(rho[-1, lo:hi + 1], 0.99, rtol=1e-14)


# -------------------------------------------------------- solute openings

@pytest.mark.parametrize("q", [4, 9])
@pytest.mark.parametrize("kind", ["inlet", "outlet"])
def test_solute_flux_opening_steady_profile(q, kind):
    """Flux opening (inlet_solute / outlet_solute, App. B) on xlo of a
    diffusion strip at rest, dirichlet C = 0 on xhi, tau_s = 1: the steady
    profile is linear, C(x) = a (1 - x/(nx-1)), and the opening rule fixes
    a: a (D + v) = v C0 + D C(1) for an inlet, a (v - D) = v C0 - D C(1)
    for an outlet, with C(1) = a (1 - 1/(nx-1))."""
    nx, ny, C0 = 20, 3, 1.0
    v = 0.1 if kind == "inlet" else 0.5
    D = 0.5 * 0.5 if q == 4 else 0.5 / 3
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.solute(1.0, q)
    o.solute_opening_range("xlo", 0, ny - 1, kind, "flux", C0, v)
    o.solute_opening_range("xhi", 0, ny - 1, "outlet", "dirichlet", 0.0)
    o.set_fields(0, 1.0)
    o.set_concentration(0.0)
    o.iteration(40000)
    C, _ = o.solute_state()
    k = 1 - 1 / (nx - 1)
    a = v * C0 / (D + v - D * k) if kind == "inlet" else v * C0 / (v - D + D * k)
    np.testing.assert_allclose(C[1], a * (1 - np.arange(nx) / (nx - 1)), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("q", [4, 9])
def test_solute_openings_on_y_walls_and_closed_wall_parts(q):
    """A dirichlet opening on part of ylo holds C = Cbar on its nodes after
    every step; the rest of the ylo and yhi walls is impermeable, so with
    an adiabatic opening on part of yhi the solute budget
    (solute + outflow - inflow) stays at its start value."""
    nx, ny = 24, 16
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.aveacceleration(2, 1e-5)
    o.solute(0.8, q)
    o.solute_opening_range("ylo", 5, 14, "inlet", "dirichlet", 1.0)
    o.solute_opening_range("yhi", 8, 20, "outlet", "adiabatic")
    o.set_fields(0, 1.0)
    o.set_concentration(0.2)
    b0 = o.budgets()
    for _ in range(3):
        o.iteration(57)
        C, _ = o.solute_state()
        np.testing.assert_allclose(C[0, 5:15], 1.0, rtol=1e-13)
    b = o.budgets()
    assert b["inflow"] > 0 and b["outflow"] > 0
    assert b["solute"] - b["inflow"] + b["outflow"] == pytest.approx(b0["solute"], rel=1e-12)



@pytest.mark.parametrize("q", [4, 9])
def test_adiabatic_walls_keep_tangential_equilibrium(q):
    """Adiabatic openings on both x walls (inlet_solute / outlet_solute,
    zero normal flux: g3 = g1 on xhi) under a uniform flow along the walls:
    a uniform concentration is an exact steady state, so every population of
    every node, wall nodes included, stays at g_eq(C, u) = w_i C (1 + e.u/c_s^2)."""
    nx, ny, C0, uy = 9, 7, 0.37, 0.02
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.solute(0.8, q)
    o.solute_opening_range("xlo", 0, ny - 1, "inlet", "adiabatic")
    o.solute_opening_range("xhi", 0, ny - 1, "outlet", "adiabatic")
    o.set_fields(0, 1.0, 0.0, uy)
    o.set_concentration(C0, 0.0, uy)
    o.iteration(100)
    g = o.get_g()
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4 if q == 9 else [0] + [0.25] * 4 + [0] * 4
    ics2 = 3.0 if q == 9 else 2.0
    for i in range(9):
        np.testing.assert_allclose(g[i], w[i] * C0 * (1 + ics2 * EY[i] * uy), rtol=1e-13, atol=0)


@pytest.mark.parametrize("q", [4, 9])
def test_adiabatic_wall_is_a_mirror_plane(q):
    """An adiabatic wall node is a symmetry plane of the solute (the unknown
    populations copy their mirror images): a strip of nx nodes with a
    dirichlet xlo and an adiabatic xhi evolves exactly as the first nx
    columns of a strip of 2 nx - 1 nodes with dirichlet walls on both
    sides and the mirrored initial concentration, here under a flow along
    the walls and a concentration that varies along them."""
    nx, ny, uy, Cbar = 13, 8, 0.03, 1.0
    rng = np.random.default_rng(44)
    C = 0.2 + 0.5 * rng.uniform(0, 1, (ny, nx))
    wide = 2 * nx - 1
    Cw = np.concatenate([C, C[:, -2::-1]], axis=1)

    def run(width, xhi_style, C0):
        o = Oracle(width, ny)
        o.fluids(1, 1.0)
        o.solute(0.7, q)
        o.solute_opening_range("xlo", 0, ny - 1, "inlet", "dirichlet", Cbar)
        o.solute_opening_range("xhi", 0, ny - 1, "outlet", xhi_style, Cbar)
        o.set_fields(0, 1.0, 0.0, uy)
        o.set_concentration(C0.ravel(), 0.0, uy)
        o.iteration(60)
        return o.solute_state()[0]

    half = run(nx, "adiabatic", C)
    full = run(wide, "dirichlet", Cw)
    np.testing.assert_allclose(full[:, nx - 1:], full[:, nx - 1::-1], rtol=1e-12)  # the wide run stays symmetric
    np.testing.assert_allclose(half, full[:, :nx], rtol=1e-12)
    assert np.ptp(half[:, -1]) > 1e-4    # the wall column still varies along the wall

def test_solute_budget_closes_with_openings_on_every_wall():
    """Openings of all three styles on all four walls, reactive walls and
    growth: solute + deposit + consumed deposit + removed solute - b0 per
    grown node - inflow + outflow equals its start value."""
    rng = np.random.default_rng(17)
    nx, ny = 40, 36
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.aveacceleration(1, 2e-5)
    o.solute(0.9, 9)
    for _ in range(5):
        o.obstacle_circle(int(rng.integers(8, 32)), int(rng.integers(8, 28)), float(rng.uniform(2, 4)))
    o.solute_opening_range("xlo", 2, 30, "inlet", "flux", 1.0, 0.05)
    o.solute_opening_range("xhi", 0, 35, "outlet", "adiabatic")
    o.solute_opening_range("ylo", 4, 20, "inlet", "dirichlet", 0.7)
    o.solute_opening_range("yhi", 10, 30, "outlet", "flux", 0.1, 0.2)
    o.surface_reaction(0.02, 0.0, 0.003, 0.2, 9)
    o.set_fields(0, 1.0)
    o.set_concentration(0.3)
    b0 = o.budgets()
    o.iteration(300)
    b = o.budgets()
    assert b["grown_nodes"] > 0
    lhs = (b["solute"] + b["deposit"] + b["consumed_deposit"] + b["removed_solute"] - 0.003 * b["grown_nodes"]
           - b["inflow"] + b["outflow"])
    assert lhs == pytest.approx(b0["solute"] + b0["deposit"], rel=1e-12)


# ------------------------------------------------- slip / mixed boundaries

def _lone_mode(style, R, wall):
    """One unit of f5 at P = (3, 5) next to a flat wall (boundary_style
    command, Fig. slip): after one step the node masses and momenta."""
    nx, ny = 12, 12
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.boundary_style(style, R)
    if wall == "horizontal":
        o.obstacle_rect(0, nx - 1, 6, 6)     # row above P
    else:
        o.obstacle_rect(4, 4, 0, ny - 1)     # column right of P
    o.set_fields(0, 1.0)                       # fluid at rest, rho = 1 ...
    f = o.get_f(0)
    f[5, 5, 3] += 1.0                          # ... plus one unit of f5 at P
    o.set_f(f, 0)
    o.iteration(1)
    g = o.get_f(0)
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    solid = o.get_mask().astype(bool)
    # the uniform rest state streams onto itself, so node mass above 1 and
    # the momentum are the unit's
    return np.where(solid, 0.0, g.sum(0) - 1.0), np.tensordot(ex, g, 1), np.tensordot(ey, g, 1)


@pytest.mark.parametrize("wall", ["horizontal", "vertical"])
@pytest.mark.parametrize("style,R", [("noslip", 0.0), ("slip", 1.0), ("mixed", 0.3)])
def test_diagonal_mode_at_flat_wall(wall, style, R):
    """Slip rule of the boundary_style command: f5 leaving (i, j) towards a
    solid (i+1, j+1) on a horizontal wall lands on (i+2, j) as f8, on a
    vertical wall on (i, j+2) as f6; noslip bounces it back to (i, j) as f7;
    mixed sends the share R forward and 1 - R back.  Mass and momentum move
    with the populations (one BGK step conserves both per node)."""
    rho, jx, jy = _lone_mode(style, R, wall)
    land, e = ((5, 5), (1, -1)) if wall == "horizontal" else ((3, 7), (-1, 1))
    assert rho[5, 3] == pytest.approx(1.0 - R, abs=1e-15)
    assert (jx[5, 3], jy[5, 3]) == pytest.approx((-(1.0 - R), -(1.0 - R)), abs=1e-15)
    assert rho[land[1], land[0]] == pytest.approx(R, abs=1e-15)
    assert (jx[land[1], land[0]], jy[land[1], land[0]]) == pytest.approx((R * e[0], R * e[1]), abs=1e-15)
    assert rho.sum() == pytest.approx(1.0, rel=1e-13)
    others = np.ones_like(rho, bool)
    others[5, 3] = others[land[1], land[0]] = False
    assert np.abs(rho[others]).max() <= 1e-15 and np.abs(jx[others]).max() <= 1e-15


def test_slip_channel_is_plug_flow():
    """Full-slip flat walls take no x momentum (the diagonal modes reflect
    specularly, the axial ones carry none along the wall): a forced
    channel's momentum grows by exactly the total force each step and the
    profile stays flat; noslip loses momentum to the walls."""
    nx, ny, a = 8, 20, 1e-5
    out = {}
    for style in ("noslip", "mixed", "slip"):
        o = Oracle(nx, ny)
        o.fluids(1, 0.9)
        o.boundary_style(style, 0.5)
        o.obstacle_rect(0, nx - 1, 0, 0)
        o.obstacle_rect(0, nx - 1, ny - 1, ny - 1)
        o.aveacceleration(1, a)
        o.set_fields(0, 1.0)
        m0 = o.budgets()["mass0"]
        o.iteration(500)
        b = o.budgets()
        _, ux, _ = o.moments(0)
        out[style] = b["mom_x"]
        assert b["mass0"] == pytest.approx(m0, rel=1e-13)
        if style == "slip":
            assert b["mom_x"] == pytest.approx(500 * a * m0, rel=1e-12)
            assert np.ptp(ux[1:-1]) <= 1e-15
    assert out["noslip"] < out["mixed"] < out["slip"]


def test_hybrid_obstacles_conserve_mass():
    """Hybrid style: obstacles with their own styles (noslip, slip, mixed
    shares) in a periodic box with a random start; every mode that hits a
    solid is sent back or forward, never lost: the mass is conserved."""
    rng = np.random.default_rng(23)
    nx, ny = 40, 34
    o = Oracle(nx, ny)
    o.fluids(2, 0.8, 1.1)
    o.boundary_style("hybrid")
    for k in range(10):
        o.obstacle_style(0, ("noslip", "slip", "mixed")[k % 3], float(rng.uniform(0, 1)))
        o.obstacle_style(1, ("slip", "mixed", "noslip")[k % 3], float(rng.uniform(0, 1)))
        if k % 2:
            o.obstacle_circle(int(rng.integers(0, nx)), int(rng.integers(0, ny)), float(rng.uniform(1.5, 4)))
        else:
            x0, y0 = int(rng.integers(0, nx - 6)), int(rng.integers(0, ny - 6))
            o.obstacle_rect(x0, x0 + int(rng.integers(0, 5)), y0, y0 + int(rng.integers(0, 5)))
    n = nx * ny
    o.set_fields(0, 0.6 + 0.1 * rng.uniform(0, 1, n), 0.02 * rng.uniform(-1, 1, n), 0.02 * rng.uniform(-1, 1, n))
    o.set_fields(1, 0.4 + 0.1 * rng.uniform(0, 1, n), 0.02 * rng.uniform(-1, 1, n), 0.02 * rng.uniform(-1, 1, n))
    o.aveacceleration(1, 1e-4, 0)
    b0 = o.budgets()
    o.iteration(200)
    b = o.budgets()
    for c in (0, 1):
        assert b[f"mass{c}"] == pytest.approx(b0[f"mass{c}"], rel=1e-13)


# ------------------------------------------------------------- intersolute

def _flat_solute_interface(q, tau_s, G, Cl, Cg, steps, psi0=1.0, C0=5e-3, nx=4, ny=128):
    """A solute slab (tanh profile along y, periodic box) in a fluid at
    rest under the intersolute force; the concentration profile after
    `steps` steps."""
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.set_fields(0, 1.0)
    o.solute(tau_s, q)
    o.intersolute(G, psi0, C0)
    yy = np.repeat(np.arange(ny), nx).astype(float)
    o.set_concentration(Cg + (Cl - Cg) * 0.5 * (np.tanh((yy - ny / 4) / 4.0) - np.tanh((yy - 3 * ny / 4) / 4.0)))
    o.iteration(steps)
    C, _ = o.solute_state()
    return C


@pytest.mark.parametrize("q,tau_s,G,Cl,Cg", [(4, 5.0, -0.01, 0.01094, 0.002342),
                                              (9, 5.0, -0.007, 0.01216, 0.002111)])
def test_intersolute_flat_interface_balance(q, tau_s, G, Cl, Cg):
    """A steady flat solute interface carries no flux across any link.
    Summing the zero-flux condition across the interface (the force stencil
    F = -G psi(x) [psi(x+e) - psi(x-e)] telescopes over products
    psi(x) psi(x+e)) fixes a quantity that is equal in the two bulk phases:
    p = (D / tau_s) C + G psi(C)^2, D = c_s^2 (tau_s - 1/2) the solute
    diffusivity (c_s^2 = 1/2 on D2Q4, 1/3 on D2Q9) -- the tau_s of the
    velocity term tau_s F / C turns D into D / tau_s.  A missing tau_s, a
    weighted or eight-neighbour stencil, or a wrong sign breaks either the
    equality or the phase contrast."""
    C = _flat_solute_interface(q, tau_s, G, Cl, Cg, 20000)
    cl, cg = C[64].mean(), C[0].mean()
    D = (0.5 if q == 4 else 1.0 / 3.0) * (tau_s - 0.5)
    p = lambda c: D / tau_s * c + G * math.exp(-5e-3 / c) ** 2
    assert cl > 4 * cg
    assert np.ptp(C[56:72]) <= 1e-9 * cl and np.ptp(C[:8]) <= 1e-9 * cl   # flat bulk phases
    assert p(cl) == pytest.approx(p(cg), rel=1e-9)


def test_intersolute_without_strength_changes_nothing():
    """G = 0: the run equals the one without the command, bit for bit."""
    nx, ny = 30, 22
    runs = []
    for with_cmd in (False, True):
        o = Oracle(nx, ny)
        o.fluids(1, 0.9)
        o.set_fields(0, 1.0, 0.01, 0.0)
        o.obstacle_circle(10, 10, 3.0)
        o.solute(0.8, 4)
        if with_cmd:
            o.intersolute(0.0, 1.0, 5e-3)
        o.set_concentration(5e-3 * (1 + 0.1 * np.sin(np.arange(nx * ny))))
        o.iteration(40)
        runs.append(o.get_g())
    assert np.array_equal(runs[0], runs[1])


def test_intersolute_conserves_solute_momentum():
    """The force is antisymmetric between neighbour pairs, so on a periodic
    box with the solvent at rest and tau_s = 1 the solute momentum after a
    step, sum C u' = tau_s sum F, is zero while the local fluxes are not."""
    rng = np.random.default_rng(8)
    nx, ny = 24, 20
    o = Oracle(nx, ny)
    o.fluids(1, 1.0)
    o.set_fields(0, 1.0)
    o.solute(1.0, 9)
    o.intersolute(-5e-3, 1.0, 5e-3)
    o.set_concentration(5e-3 * (1 + 0.5 * rng.uniform(-1, 1, nx * ny)))
    o.iteration(1)
    g = o.get_g()
    jx, jy = np.tensordot(EX, g, 1), np.tensordot(EY, g, 1)
    assert np.abs(jx).max() > 1e-6
    assert abs(jx.sum()) <= 1e-16 * nx * ny and abs(jy.sum()) <= 1e-16 * nx * ny
