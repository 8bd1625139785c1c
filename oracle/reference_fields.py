"""FP64 oracle reference fields for the precision sweep (test infrastructure).

Writes an .npz with density and velocity after a number of steps for

* ``channel``: the Poiseuille workload at n x n nodes (solid rows 0 and n-1,
  tau = 1, acceleration 1e-6 along e1).  The flow is uniform along the
  periodic x axis, so the oracle runs a 4-node-wide strip of it, which is
  exactly the n x n solution in every column;
* ``porous``: the porous workload at n x n nodes (seed 4) in full.

Only this package's oracle and the seeded input generator are used.

    python -m oracle.reference_fields OUT.npz [--n 2048] [--steps 10000]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, set_threads  # noqa: E402
from paper_1202_0442_amd import inputs  # noqa: E402


def channel(n, steps, accel=1e-6, tau=1.0):
    o = Oracle(4, n)
    o.fluids(1, tau)
    o.obstacle_rect(0, 3, 0, 0)
    o.obstacle_rect(0, 3, n - 1, n - 1)
    o.aveacceleration(1, accel)
    o.set_fields(0, 1.0)
    o.iteration(steps)
    rho, ux, uy = o.moments(0)
    return rho[:, 0].copy(), ux[:, 0].copy(), uy[:, 0].copy()


def porous(n, steps, seed=4):
    w = inputs.porous(n=n, seed=seed)
    o = Oracle(w.nx, w.ny)
    o.fluids(1, w.tau)
    for (xc, yc, r) in w.discs:
        o.obstacle_circle(xc, yc, r)
    o.aveacceleration(1, w.accel_x)
    o.set_fields(0, 1.0)
    done = 0
    while done < steps:
        k = min(500, steps - done)
        o.iteration(k)
        done += k
        print(f"porous oracle: {done}/{steps} steps", flush=True)
    rho, ux, uy = o.moments(0)
    return rho, ux, uy, o.get_mask()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    th = set_threads(a.threads)
    t0 = time.time()
    cr, cu, cv = channel(a.n, a.steps)
    print(f"channel strip done in {time.time() - t0:.1f} s ({th} threads)", flush=True)
    pr, pu, pv, pm = porous(a.n, a.steps)
    print(f"porous done in {time.time() - t0:.1f} s", flush=True)
    np.savez(a.out, n=a.n, steps=a.steps, channel_rho=cr, channel_ux=cu, channel_uy=cv,
             porous_rho=pr, porous_ux=pu, porous_uy=pv, porous_mask=pm)


if __name__ == "__main__":
    main()
