"""Checkpoint and restart: a run saved after N steps and continued, in a
fresh lattice set up by the same commands, for M more steps equals the
uninterrupted run of N + M steps bit for bit (populations of every
component and the solute, mask, deposits, budgets including the running
tallies, step count), for the general step with growth (FP64, FP32, FP16
with stochastic rounding) and the one-fluid step."""
import numpy as np
import pytest

from cases import build_gpu, porous_case, sc_solute_case

pytestmark = pytest.mark.gpu


def _lattice(case, storage, rounding):
    g = build_gpu(case, storage, bind=False)
    if rounding != "nearest":
        g.rounding(rounding, 77)
    g.bind(storage)
    return g


def _state(g, comps, deposit=True):
    return ([g.get_populations(c) for c in comps], g.mask(), g.get_deposit() if deposit else None, g.budgets(),
            g.step_count())


def _same(a, b):
    pa, ma, ba, ua, ta = a
    pb, mb, bb, ub, tb = b
    assert ta == tb
    for x, y in zip(pa, pb):
        assert np.array_equal(x, y)
    assert np.array_equal(ma, mb) and (ba is None and bb is None or np.array_equal(ba, bb))
    assert ua == ub


@pytest.mark.parametrize("kind,storage,rounding", [("full", "f64", "nearest"), ("full", "f32", "nearest"),
                                                   ("full", "f16", "stochastic"), ("plain", "f32", "nearest")])
def test_restart_equals_uninterrupted_run(kind, storage, rounding):
    if kind == "full":
        case, comps = sc_solute_case(96, 80, 31, react=True), (0, 1, -1)
    else:
        case, comps = porous_case(131, 77, 31), (0,)
    whole = _lattice(case, storage, rounding)
    whole.iteration(150)
    full = kind == "full"
    want = _state(whole, comps, full)
    if kind == "full":
        assert want[3]["grown_nodes"] > 0
    first = _lattice(case, storage, rounding)
    first.iteration(71)                      # odd step count: the restart begins at odd parity
    ck = first.checkpoint()
    resumed = _lattice(case, storage, rounding)
    resumed.restore(ck)
    assert resumed.step_count() == 71
    resumed.iteration(79)
    _same(_state(resumed, comps, full), want)
    first.iteration(40)                      # the saved lattice rewinds to its checkpoint
    first.restore(ck)
    first.iteration(79)
    _same(_state(first, comps, full), want)


def test_restore_refuses_other_lattices_and_truncated_data():
    from paper_1202_0442_amd import lb2d
    case = porous_case(64, 40, 3)
    a = build_gpu(case, "f32")
    a.iteration(5)
    ck = a.checkpoint()
    for other in (build_gpu(porous_case(64, 41, 3), "f32"), build_gpu(case, "f64"),
                  build_gpu(dict(case, tau=0.7, fields={0: (np.full(64 * 40, 1.3), None, None)}), "f32")):
        with pytest.raises(lb2d.LB2DError) as e:
            other.restore(ck)
        assert e.value.code == lb2d.E_INVAL
    with pytest.raises(lb2d.LB2DError) as e:
        a.restore(ck[:-16])
    assert e.value.code == lb2d.E_SIZE
