"""The three-step kernel of the one-fluid lattice (temporal blocking: the
first step of a tile and two rings of nodes around it, and the second step of
the tile and the inner ring, kept in LDS; the third written to HBM) against
the one-step kernel and the FP64 oracle.

Launch graphs run the one-fluid step as three-step launches on lattices of
at least 66 x 18 nodes (34 x 18 in FP64), then single steps; timing mode
launches single steps.  So a lattice stepped through graphs and the same
lattice stepped with timing on must agree bit for bit, in every storage
format and with stochastic rounding, whose random words are keyed on each
node and step.  The lattice shapes cover the smallest lattice the kernel
takes (its rings then wrap onto the far side of the lattice), tiles
overhanging the lattice by a few nodes and by all but a few, and lattices
one node too small for the kernel in either direction.
"""
import numpy as np
import pytest

from cases import build_gpu, build_oracle, porous_case

pytestmark = pytest.mark.gpu

SHAPES = [(66, 18), (67, 19), (65, 18), (66, 17), (127, 31), (150, 90), (34, 18), (35, 47), (33, 47), (200, 20)]


def _pair(case, storage, rounding):
    def lattice():
        g = build_gpu(case, storage, bind=False)
        if rounding == "stochastic":
            g.rounding("stochastic", 11)
        g.bind(storage)
        return g
    a, b = lattice(), lattice()
    b.set_timing(True)
    return a, b


@pytest.mark.parametrize("storage,rounding", [("f64", "nearest"), ("f32", "nearest"), ("f16", "nearest"),
                                              ("bf16", "nearest"), ("f16", "stochastic"),
                                              ("bf16", "stochastic")])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_three_step_launches_equal_single_steps(nx, ny, storage, rounding):
    """101 steps (one step, then from the odd step count two 48-step graphs
    and a 4-step tail: a three-step launch and a single step) through graphs
    equal 101 single launches, bit for bit."""
    case = porous_case(nx, ny, 40 + nx + ny, tau=0.7)
    a, b = _pair(case, storage, rounding)
    a.iteration(1)
    b.iteration(1)
    a.prepare(100)
    a.iteration(100)
    b.iteration(100)
    assert a.step_count() == b.step_count() == 101
    assert np.array_equal(a.get_populations(0), b.get_populations(0))
    assert np.array_equal(a.mask(), b.mask())


def test_steps_per_launch_follows_the_lattice_extent():
    """The three-step kernel runs exactly where the lattice has the extent it
    needs (its tile plus two nodes each way)."""
    for (nx, ny, st, want) in [(66, 18, "f32", 3), (65, 18, "f32", 1), (66, 17, "f32", 1), (66, 18, "f16", 3),
                               (34, 18, "f64", 3), (33, 18, "f64", 1), (4096, 4096, "f32", 3)]:
        g = build_gpu(porous_case(nx, ny, 3) if nx * ny < 1e6 else dict(nx=nx, ny=ny, tau=0.8), st)
        assert g.steps_per_launch() == want, (nx, ny, st)
        g.close()


@pytest.mark.parametrize("nx,ny", [(66, 18), (67, 19), (150, 90), (35, 47)])
def test_three_step_launches_match_oracle(nx, ny):
    """Graph-stepped lattices against the oracle after 160 steps: FP64 within
    1e-12 of the largest velocity and density, FP32 within 1e-5."""
    case = porous_case(nx, ny, 70 + nx, tau=0.9)
    o = build_oracle(case)
    o.iteration(160)
    orr, ox, oy = o.moments(0)
    solid = orr == -11.0
    uscale = max(np.abs(ox).max(), np.abs(oy).max())
    for storage, tol in (("f64", 1e-12), ("f32", 1e-5)):
        g = build_gpu(case, storage)
        g.iteration(160)
        gr, gx, gy = g.moments(0)
        assert np.array_equal(gr == -11.0, solid)
        eu = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / uscale
        er = np.abs(gr - orr)[~solid].max() / np.abs(orr[~solid]).max()
        print(f"{nx}x{ny} {storage}: rel u err {eu:.2e}, rel rho err {er:.2e}")
        assert eu <= tol and er <= tol


def test_three_step_launches_conserve_mass_exactly_in_fp64():
    """Periodic box with bounce-back obstacles: the total mass after 400
    graph-launched steps equals the initial mass to rounding (FP64)."""
    case = porous_case(96, 48, 5, tau=0.8)
    g = build_gpu(case, "f64")
    m0 = g.budgets()["mass0"]
    g.iteration(400)
    m1 = g.budgets()["mass0"]
    assert abs(m1 - m0) <= 1e-12 * m0
