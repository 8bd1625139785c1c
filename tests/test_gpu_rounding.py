"""Stochastic rounding of 16-bit storage (gfx950 hardware converts keyed by
a counter-based hash), through the C ABI, against the FP64 oracle.

A channel start-up with a body force of 1e-6 changes each population by
about 1e-4 of its stored value per step: below half an FP16 ulp and far
below a BF16 ulp, so round-to-nearest drops the forcing and the start-up
stalls, while stochastic rounding keeps it on average.  Bounds were set
from the rounding-error analysis (ulp 2^-11 / 2^-8 relative, averaged
over the profile) with a margin.
"""
import numpy as np
import pytest

from cases import build_gpu, build_oracle, porous_case, poiseuille_case, rel_err

pytestmark = pytest.mark.gpu


def _gpu(case, storage, mode, seed=7):
    g = build_gpu(case, storage, bind=False)
    g.rounding(mode, seed)
    g.bind(storage)
    return g


def _u_err(g, o):
    _, gx, _ = g.moments(0)
    _, ox, _ = o.moments(0)
    fl = ox != 0.0
    return rel_err(gx[fl], ox[fl])


@pytest.mark.parametrize("storage,tol_sr,min_gain", [("f16", 5e-3, 5.0), ("bf16", 2e-2, 5.0)])
def test_channel_start_up_does_not_stall(storage, tol_sr, min_gain):
    case = poiseuille_case(nx=8, ny=66, accel=1e-6, tau=1.0)
    o = build_oracle(case)
    o.iteration(6000)
    errs = {}
    for mode in ("nearest", "stochastic"):
        g = _gpu(case, storage, mode)
        g.iteration(6000)
        errs[mode] = _u_err(g, o)
    print(storage, errs)
    assert errs["stochastic"] <= tol_sr
    assert errs["nearest"] >= min_gain * errs["stochastic"]


@pytest.mark.parametrize("storage,tol", [("f16", 3e-2), ("bf16", 2e-1)])
def test_porous_stochastic_within_16bit_bound(storage, tol):
    case = porous_case(200, 120, 5, accel=1e-5)
    o, g = build_oracle(case), _gpu(case, storage, "stochastic")
    o.iteration(400)
    g.iteration(400)
    e = _u_err(g, o)
    print(storage, e)
    assert e <= tol


def test_stochastic_rounding_is_reproducible_and_seeded():
    case = porous_case(97, 45, 6)
    a, b, c = (_gpu(case, "f16", "stochastic", s) for s in (11, 11, 12))
    for g in (a, b, c):
        g.iteration(70)
    fa, fb, fc = (g.get_populations(0) for g in (a, b, c))
    assert np.array_equal(fa, fb)
    assert not np.array_equal(fa, fc)


def test_stochastic_stream_same_for_graph_and_single_steps():
    """The rounding stream is keyed on the step number, so 64 steps in two
    graph launches equal 64 single-step launches bit for bit."""
    case = porous_case(64, 40, 8)
    a, b = _gpu(case, "bf16", "stochastic"), _gpu(case, "bf16", "stochastic")
    a.iteration(64)
    for _ in range(64):
        b.iteration(1)
    assert np.array_equal(a.get_populations(0), b.get_populations(0))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_batch_with_stochastic_rounding_equals_single_lattices(storage):
    """Each lattice of a batch draws the random words it draws alone (its
    own seed, step count and node numbering): batched runs of 75 steps (two
    60-step graph and shorter launches) and of 1 + 74 steps (a first step at
    odd parity) equal the lattices stepped one by one, bit for bit."""
    from paper_1202_0442_amd import lb2d
    cases = [porous_case(nx, ny, 20 + k, tau=0.6 + 0.1 * k) for k, (nx, ny) in
             enumerate([(64, 40), (131, 77), (33, 200), (256, 9)])]
    for chunks in ((75,), (1, 74)):
        singles = [_gpu(c, storage, "stochastic", seed=11 + k) for k, c in enumerate(cases)]
        members = [_gpu(c, storage, "stochastic", seed=11 + k) for k, c in enumerate(cases)]
        for s in singles:
            s.iteration(chunks[0])
        batch = lb2d.Batch(0)
        if len(chunks) > 1:
            for m in members:
                m.iteration(chunks[0])
        for m in members:
            batch.add(m)
        batch.finalize()
        for s in singles:
            for n in chunks[1:] if len(chunks) > 1 else ():
                s.iteration(n)
        batch.iteration(sum(chunks[1:]) if len(chunks) > 1 else chunks[0])
        for s, m in zip(singles, members):
            assert m.step_count() == 75
            assert np.array_equal(s.get_populations(0), m.get_populations(0))
        batch.close()


def test_batch_refuses_mixed_rounding():
    from paper_1202_0442_amd import lb2d
    a = _gpu(porous_case(32, 16, 1), "f16", "stochastic")
    b = _gpu(porous_case(32, 16, 2), "f16", "nearest")
    batch = lb2d.Batch(0)
    batch.add(a)
    with pytest.raises(lb2d.LB2DError) as e:
        batch.add(b)
    assert e.value.code == lb2d.E_INVAL
