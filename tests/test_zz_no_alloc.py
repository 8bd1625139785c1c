"""lb2d_budgets_noalloc (budgets for callers that cannot allocate device
memory) against lb2d_budgets through the C ABI: the same kernels and
summation order, so the two agree bit for bit; the library's static scratch
keeps the last call's contents, so a second, smaller lattice checks that
nothing carries over between calls."""
import pytest

from cases import build_gpu, porous_case, sc_solute_case

pytestmark = pytest.mark.gpu


def test_noalloc_budgets_equal_workspace_budgets():
    big = build_gpu(sc_solute_case(120, 96, 21, react=True), "f32")
    big.iteration(200)
    first = big.budgets_noalloc()
    assert first == big.budgets()
    assert first["grown_nodes"] > 0 and first["inflow"] > 0
    small = build_gpu(porous_case(40, 24, 3), "f64")     # fewer rows, no solute: no tallies
    small.iteration(30)
    second = small.budgets_noalloc()
    assert second == small.budgets()
    assert second["inflow"] == 0.0 and second["grown_nodes"] == 0.0
    assert big.budgets_noalloc() == first


def test_noalloc_budgets_reject_rows_beyond_the_scratch():
    from paper_1202_0442_amd import lb2d
    L = lb2d.Lattice(0)
    L.lattice("d2q9", 3, 65534, 1.0)
    L.bind("f32")
    with pytest.raises(lb2d.LB2DError) as e:
        L.budgets_noalloc()
    assert e.value.code == lb2d.E_SIZE
    assert L.budgets()["fluid_nodes"] == 3 * 65534
    ok = lb2d.Lattice(0)
    ok.lattice("d2q9", 3, 65533, 1.0)
    ok.bind("f32")
    assert ok.budgets_noalloc() == ok.budgets()
