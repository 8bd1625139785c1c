"""Writes surface_growth_sweep.json: the FP64 oracle's final state of the
paper's surface-growth example (section Surface growth and its script:
200 x 200 periodic box, 11 x 11 seed, D2Q4 solute C0 = 1.5, Cs = 0.5,
b0 = 0.5, bmax = 1, tau = tau_s = 1, 20 000 steps) for Da = 4, 20, 40, 80.
Calls only the oracle; run from the repository root:
    python tests/golden/make_surface_growth_sweep.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from cases import build_oracle, surface_growth_case  # noqa: E402


def main():
    out = {"source": "FP64 oracle, tests/golden/make_surface_growth_sweep.py", "steps": 20000, "runs": {}}
    for kr in (5e-3, 0.025, 0.05, 0.1):
        o = build_oracle(surface_growth_case(kr))
        o.iteration(20000)
        m = o.get_mask()
        b = o.budgets()
        out["runs"][repr(kr)] = {"grown_nodes": int(b["grown_nodes"]), "solid_nodes": int(m.sum()),
                                 "mask_sha256": hashlib.sha256(m.astype("uint8").tobytes()).hexdigest(),
                                 "solute": b["solute"], "deposit": b["deposit"]}
        print(kr, out["runs"][repr(kr)], flush=True)
    with open(os.path.join(HERE, "surface_growth_sweep.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
