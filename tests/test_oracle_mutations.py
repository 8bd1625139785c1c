"""The oracle's pins catch plausible mistakes in it.

Each case below compiles a copy of the oracle with one deliberate mistake (a
swapped index, a dropped term, a wrong sign, a missing weight), points the
oracle wrapper at it and runs pins from ``test_oracle_pins.py`` against it:
every named pin must fail.  The unmodified oracle passes the same pins in
that file, so each pin is shown to separate the method from a near miss.
Everything runs on the CPU; the mistakes live only in temporary copies.
"""
import os

import pytest

import test_oracle_pins as pins
from oracle import oracle as orc

SRC = os.path.join(os.path.dirname(orc.__file__), "lb2d_oracle.c")

# name: (text in the oracle, replacement, pins that must fail [(name, args)])
MUTATIONS = {
    # an adiabatic wall that copies the diagonal across the wall instead of
    # its mirror (g6 <- g8, g7 <- g5 on xhi instead of g6 <- g5, g7 <- g8)
    "adiabatic_diagonals_swapped": (
        "if (axis == 0 ? (EX9[k] == -EX9[i] && EY9[k] == EY9[i])",
        "if (axis == 0 ? (EX9[k] == -EX9[i] && EY9[k] == (EX9[i] != 0 ? -EY9[i] : EY9[i]))",
        [("test_adiabatic_wall_is_a_mirror_plane", (9,)),
         ("test_adiabatic_walls_keep_tangential_equilibrium", (9,))]),
    # the equilibrium without its quadratic velocity term
    "equilibrium_drops_eu_squared": (
        "3.0 * eu + 4.5 * eu * eu - 1.5 * uu",
        "3.0 * eu - 1.5 * uu",
        [("test_equilibrium_moments_match_fluids_command", (0,)),
         ("test_equilibrium_alpha_default_is_eq_eq", ())]),
    # the cohesion of two components with the wrong sign
    "cohesion_sign_flipped": (
        "Fx += -o->G * r * sx;\n                        Fy += -o->G * r * sy;",
        "Fx += o->G * r * sx;\n                        Fy += o->G * r * sy;",
        [("test_shan_chen_force_is_gradient_of_other_component", ())]),
    # a reactive link whose rate is not shared out by the link weights
    "reaction_rate_not_weighted": (
        "double k = kr * w / solute_wall_w(q);",
        "double k = kr;",
        [("test_reactive_slab_steady_state_closed_form", (9,))]),
    # bounce-back that returns the population unreversed
    "bounce_back_not_reversed": (
        "v = o->f[c][opposite(i) * n + s];",
        "v = o->f[c][i * n + s];",
        [("test_half_way_bounce_back_reverses_at_wall", ())]),
}


@pytest.fixture(scope="module")
def mutants(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_mutants")
    src = open(SRC).read()
    out = {}
    for name, (old, new, _) in MUTATIONS.items():
        assert src.count(old) == 1, f"mutation site of {name} not unique"
        path = d / f"{name}.c"
        path.write_text(src.replace(old, new))
        out[name] = orc.load_library(orc.compile_source(str(path), str(d / f"lib{name}.so")))
    return out


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_fail_on_a_planted_mistake(name, mutants, monkeypatch):
    monkeypatch.setattr(orc, "_lib", mutants[name])
    for pin, args in MUTATIONS[name][2]:
        with pytest.raises(AssertionError):
            getattr(pins, pin)(*args)
