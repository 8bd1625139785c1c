"""Permeability of the porous workload (one fluid through non-overlapping
discs r 8..24 at porosity 0.6, tau = 0.8, periodic, forced along e1):
k = nu <u_x> / a_x with <u_x> the mean over all nodes (solids read 0) and
nu = (tau - 1/2)/3, taken from a run driven to steady state.

There is no closed form for random discs.  The checks are Darcy's law
(k does not depend on the forcing at these Reynolds numbers: k(g) = k(2g)
within 1e-3) and the oracle run of the same sample for the same number of
steps (FP32 storage within 1e-5 of the oracle's k)."""
import numpy as np
import pytest

from cases import build_gpu, build_oracle

pytestmark = pytest.mark.gpu


def _case(accel, n=256, seed=7):
    from paper_1202_0442_amd import inputs
    w = inputs.porous(n=n, seed=seed)
    return dict(nx=w.nx, ny=w.ny, tau=w.tau, accel=[(1, accel, 0)], circles=w.discs), w.tau


def _k(side, accel, tau):
    _, ux, _ = side.moments(0)
    return (tau - 0.5) / 3 * float(ux.mean()) / accel


def steady_permeability(g, accel, tau, chunk=1000, rel=1e-6, max_steps=200000):
    """Steps until <u_x> changes by less than rel over `chunk` steps;
    returns (k, steps)."""
    prev = None
    while g.step_count() < max_steps:
        g.iteration(chunk)
        k = _k(g, accel, tau)
        if prev is not None and abs(k - prev) <= rel * abs(k):
            return k, g.step_count()
        prev = k
    raise AssertionError("no steady state")


def test_porous_permeability_is_darcy_and_matches_oracle():
    ks = {}
    for accel in (1e-5, 2e-5):
        case, tau = _case(accel)
        g = build_gpu(case, "f32")
        ks[accel], steps = steady_permeability(g, accel, tau)
        print(f"a_x {accel:g}: k = {ks[accel]:.6f} lu^2 after {steps} steps")
        if accel == 1e-5:
            o = build_oracle(case)
            o.iteration(steps)
            ko = _k(o, accel, tau)
            print(f"oracle k = {ko:.6f}, rel diff {abs(ks[accel] - ko) / ko:.2e}")
            assert abs(ks[accel] - ko) <= 1e-5 * ko
    assert abs(ks[2e-5] / ks[1e-5] - 1) <= 1e-3
