"""Laplace's law for two-component Shan-Chen droplets on the GPU, at radii
beyond the oracle's pin (G = 2.6, FP32 storage).

Droplets of radius 24, 40 and 64 start at the bulk densities of a
converged flat interface (computed on the oracle) and run until the
pressure jump dp stops moving (box side 4 R as in the oracle's runs: a
droplet exchanges mass with the surrounding minor phase until the
curvature shift of the bulk densities is reached; the run length grows as
R^2 from the 10^4 steps that converge R = 16).  Laplace's law with its
first curvature correction, dp R = sigma_inf + a / R (a finite interface
has a Tolman-type length), must fit the three radii to 0.5 %, with a
correction below 10 % at R = 24, and must predict the oracle's own droplet
at R = 16 (n = 64) to 1 %."""
import numpy as np
import pytest

from cases import droplet_fields, flat_coexistence, laplace_jump
from oracle import Oracle

pytestmark = pytest.mark.gpu

G = 2.6


def _oracle_droplet(hi, lo, n=64, R=16.0, steps=10000):
    o = Oracle(n, n)
    o.fluids(2, 1.0, 1.0)
    o.interforce(G)
    ra, rb = droplet_fields(n, R, hi, lo)
    o.set_fields(0, ra)
    o.set_fields(1, rb)
    o.iteration(steps)
    return laplace_jump(o.moments(0)[0], o.moments(1)[0], G)


def test_laplace_law_large_droplets_fp32():
    from paper_1202_0442_amd import lb2d
    hi, lo = flat_coexistence(G)
    r_o, dp_o = _oracle_droplet(hi, lo)
    radii, sig = [], []
    for R in (24.0, 40.0, 64.0):
        n = int(4 * R)
        steps = int(10000 * (R / 16.0) ** 2)
        g = lb2d.Lattice(0)
        g.lattice("d2q9", n, n, 1.0)
        g.fluids(1.0, 1.0)
        ra, rb = droplet_fields(n, R, hi, lo)
        g.set_fields(0, ra)
        g.set_fields(1, rb)
        g.interforce(G)
        g.bind("f32")
        jumps = []
        for k in (steps - steps // 5, steps // 5):
            g.iteration(k)
            Re, jump = laplace_jump(g.moments(0)[0], g.moments(1)[0], G)
            jumps.append(jump)
        g.close()
        print(f"R {Re:.2f}: dp {jumps[1]:.6e} (change over the last {steps // 5} steps "
              f"{jumps[1] / jumps[0] - 1:.1e}), dp R {jumps[1] * Re:.5f}")
        assert abs(jumps[1] / jumps[0] - 1.0) < 2e-3
        radii.append(Re)
        sig.append(jumps[1] * Re)
    inv = 1.0 / np.array(radii)
    a, s_inf = np.polyfit(inv, sig, 1)
    resid = np.array(sig) - (s_inf + a * inv)
    pred = s_inf + a / r_o
    print(f"sigma_inf {s_inf:.5f}, a {a:.4f}; oracle R {r_o:.2f}: dp R {dp_o * r_o:.5f}, predicted {pred:.5f}")
    assert s_inf > 0
    assert np.abs(resid).max() <= 0.005 * s_inf
    assert abs(a) / radii[0] <= 0.1 * s_inf
    assert abs(pred / (dp_o * r_o) - 1.0) <= 0.01
