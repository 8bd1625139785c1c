"""The multi-step kernel of the one-fluid lattice (temporal blocking, five
steps per launch: the first step of a tile and four rings of nodes around it,
then each further step on one ring fewer, kept in LDS; the fifth written to
HBM) against the one-step kernel and the FP64 oracle.

Launch graphs run the one-fluid step as five-step launches on lattices of
at least 72 x 24 nodes (40 x 24 in FP64), then single steps; timing mode
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

SHAPES = [(72, 24), (73, 25), (71, 24), (72, 23), (127, 31), (150, 90), (40, 24), (41, 47), (39, 47), (200, 26)]


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
def test_multi_step_launches_equal_single_steps(nx, ny, storage, rounding):
    """101 steps (one step, then from the odd step count a 60-step graph and
    a 40-step tail graph of eight five-step launches) through graphs equal
    101 single launches, bit for bit."""
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
    """The multi-step kernel runs exactly where the lattice has the extent it
    needs (its tile plus four nodes each way)."""
    for (nx, ny, st, want) in [(72, 24, "f32", 5), (71, 24, "f32", 1), (72, 23, "f32", 1), (72, 24, "f16", 5),
                               (40, 24, "f64", 5), (39, 24, "f64", 1), (4096, 4096, "f32", 5)]:
        g = build_gpu(porous_case(nx, ny, 3) if nx * ny < 1e6 else dict(nx=nx, ny=ny, tau=0.8), st)
        assert g.steps_per_launch() == want, (nx, ny, st)
        g.close()


@pytest.mark.parametrize("nx,ny", [(72, 24), (73, 25), (150, 90), (41, 47)])
def test_multi_step_launches_match_oracle(nx, ny):
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


def test_multi_step_launches_conserve_mass_exactly_in_fp64():
    """Periodic box with bounce-back obstacles: the total mass after 400
    graph-launched steps equals the initial mass to rounding (FP64)."""
    case = porous_case(96, 48, 5, tau=0.8)
    g = build_gpu(case, "f64")
    m0 = g.budgets()["mass0"]
    g.iteration(400)
    m1 = g.budgets()["mass0"]
    assert abs(m1 - m0) <= 1e-12 * m0
