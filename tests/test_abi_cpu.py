"""C-ABI contract on the CPU: the library loads, exports every entry point
of include/lb2d.h, and the host state machine applies the paper's command
order rules and argument checks (no device work is done before bind)."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lb2d():
    from paper_1202_0442_amd import lb2d
    return lb2d


def test_library_exports_every_declared_symbol():
    import ctypes
    lb2d = _lb2d()
    header = open(os.path.join(ROOT, "include", "lb2d.h")).read()
    declared = set(re.findall(r"^(?:int|const char \*)\s*(lb2d_\w+)\s*\(", header, re.M))
    assert len(declared) >= 40
    lib = ctypes.CDLL(lb2d.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared <= set(lb2d.EXPORTED)


def test_lattice_must_come_first():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    for call in (lambda: L.fluids(1, 1), lambda: L.solute(1.0), lambda: L.boundary_style("noslip"),
                 lambda: L.aveforce(1, 1e-3), lambda: L.interforce(0.9)):
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_ORDER


def test_obstacle_must_follow_boundary_style():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 10, 10, 1.0)
    with pytest.raises(lb2d.LB2DError) as e:
        L.obstacle_circle(5, 5, 2.0)
    assert e.value.code == lb2d.E_ORDER
    L.boundary_style("noslip")
    L.obstacle_circle(5, 5, 2.0)
    L.obstacle_rect(0, 9, 0, 0)


def test_fluids_after_forces_is_an_order_error():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 10, 10, 1.0)
    L.aveacceleration(1, 1e-5)
    with pytest.raises(lb2d.LB2DError) as e:
        L.fluids(1.0, 1.0)
    assert e.value.code == lb2d.E_ORDER


def test_solute_commands_need_solute():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 10, 10, 1.0)
    for call in (lambda: L.solute_opening("xlo", "dirichlet", 1.0),
                 lambda: L.surface_reaction(1e-3, 0.0, "growth", 0.0, 1.0, 1),
                 lambda: L.set_concentration(np.zeros(100)),
                 lambda: L.intersolute(-5e-3, 1.0, 5e-3)):
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_ORDER
    L.solute(1.0, 4)
    for args in ((-5e-3, 1.0, 0.0), (-5e-3, 1.0, -1.0), (float("nan"), 1.0, 5e-3), (-5e-3, float("inf"), 5e-3)):
        with pytest.raises(lb2d.LB2DError) as e:
            L.intersolute(*args)
        assert e.value.code == lb2d.E_INVAL
    L.intersolute(-5e-3, 1.0, 5e-3)


def test_unsupported_forms():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 10, 10, 1.0)
    L.fluids(1, 1.0)
    for call in (lambda: L.boundary_style("mixed", 1.5), lambda: L.boundary_style("mixed", -0.1),
                 lambda: L.boundary_style("sticky")):
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_INVAL
    L.boundary_style("slip")
    with pytest.raises(lb2d.LB2DError) as e:
        L.obstacle_style(0, "slip")                 # only under the hybrid style
    assert e.value.code == lb2d.E_ORDER
    L.boundary_style("hybrid")
    for call in (lambda: L.obstacle_style(2, "slip"), lambda: L.obstacle_style(0, "mixed", 2.0),
                 lambda: L.obstacle_style(0, "hybrid")):
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_INVAL
    L.obstacle_style(0, "mixed", 0.3)
    L.solute(1.0, 9)
    with pytest.raises(lb2d.LB2DError) as e:
        L.solute_opening("xlo", "flux", 1.0)      # the whole-wall form has no velocity
    assert e.value.code == lb2d.E_INVAL
    with pytest.raises(lb2d.LB2DError) as e:
        L.lattice("d2q7", 10, 10, 1.0)


def test_bad_arguments():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    for args in (("d2q9", 2, 10, 1.0), ("d2q9", 10, 10, 0.5), ("d2q9", 10, 10, float("nan"))):
        with pytest.raises(lb2d.LB2DError) as e:
            L.lattice(*args)
        assert e.value.code == lb2d.E_INVAL
    L.lattice("d2q9", 10, 8, 1.0)
    L.boundary_style("noslip")
    for call in (lambda: L.obstacle_rect(0, 10, 0, 0), lambda: L.obstacle_rect(3, 2, 0, 0),
                 lambda: L.obstacle_circle(10, 0, 1.0), lambda: L.obstacle_circle(1, 1, -1.0),
                 lambda: L.aveforce(9, 1.0), lambda: L.aveforce(1, 1.0, 1),
                 lambda: L.set_fields(0, -np.ones(80)), lambda: L.set_fields(1, np.ones(80)),
                 lambda: L.fluids(0.4, 1.0), lambda: L.solute(1.0, 5), lambda: L.solute(0.5, 4)):
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_INVAL
    with pytest.raises(ValueError):
        L.set_fields(0, np.ones(79))


def test_sixteen_bit_storage_and_stochastic_rounding_forms():
    """16-bit storage and its stochastic rounding for every lattice;
    stochastic rounding of FP32 or FP64 storage is refused."""
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 16, 16, 1.0)
    L.fluids(1.0, 1.0)
    assert L.workspace_bytes("f16") < L.workspace_bytes("f32")
    L.rounding("stochastic", 1)
    assert L.workspace_bytes("bf16") == L.workspace_bytes("f16")
    for st in ("f32", "f64"):
        with pytest.raises(lb2d.LB2DError) as e:
            L.workspace_bytes(st)
        assert e.value.code == lb2d.E_UNSUPPORTED


def test_workspace_sizes_scale_with_storage():
    lb2d = _lb2d()
    sizes = {}
    for st in ("f64", "f32", "f16", "bf16"):
        L = lb2d.Lattice()
        L.lattice("d2q9", 512, 256, 1.0)
        sizes[st] = L.workspace_bytes(st)
    n = 512 * 256
    # two population buffers of 9 planes each dominate; the rest is fixed
    assert sizes["f64"] - sizes["f32"] == pytest.approx(2 * 9 * n * 4, rel=1e-3)
    assert sizes["f32"] - sizes["f16"] == pytest.approx(2 * 9 * n * 2, rel=1e-3)
    assert sizes["f16"] == sizes["bf16"]


def test_iteration_before_bind_and_bind_checks():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 16, 16, 1.0)
    with pytest.raises(lb2d.LB2DError) as e:
        L.iteration(1)
    assert e.value.code == lb2d.E_STATE
    import ctypes
    from paper_1202_0442_amd.lb2d import _lib
    # bind before choosing a storage format
    rc = _lib.lb2d_bind(L.handle, ctypes.c_void_p(256), 1 << 20, None)
    assert rc == lb2d.E_ORDER
    L.workspace_bytes("f32")
    assert _lib.lb2d_bind(L.handle, ctypes.c_void_p(300), 1 << 20, None) == lb2d.E_INVAL
    assert _lib.lb2d_bind(L.handle, ctypes.c_void_p(256), 10, None) == lb2d.E_SIZE


def test_opening_commands_check_their_arguments():
    """Solute and momentum openings: walls, ranges, styles, overlaps."""
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 16, 12, 1.0)
    with pytest.raises(lb2d.LB2DError) as e:
        L.solute_opening_range("xlo", 0, 11, "inlet", "dirichlet", 1.0)
    assert e.value.code == lb2d.E_ORDER                       # needs solute first
    L.solute(0.8)
    bad = [lambda: L.solute_opening_range("zlo", 0, 3, "inlet", "dirichlet", 1.0),
           lambda: L.solute_opening_range("xlo", 3, 2, "inlet", "dirichlet", 1.0),
           lambda: L.solute_opening_range("xlo", 0, 12, "inlet", "dirichlet", 1.0),
           lambda: L.solute_opening_range("ylo", 0, 3, "sideways", "dirichlet", 1.0),
           lambda: L.solute_opening_range("ylo", 0, 3, "inlet", "flux", 1.0, 0.0),
           lambda: L.momentum_opening("xlo", 0, 12, 0, "inlet", "uniform", 0.01, 1.0),
           lambda: L.momentum_opening("xlo", 0, 3, 1, "inlet", "uniform", 0.01, 1.0),
           lambda: L.momentum_opening("xlo", 0, 3, 0, "inlet", "uniform", 1.5, 1.0),
           lambda: L.momentum_opening("xlo", 0, 3, 0, "inlet", "swirl", 0.01, 1.0)]
    for call in bad:
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_INVAL
    L.solute_opening_range("xlo", 0, 5, "inlet", "flux", 1.0, 0.1)
    L.solute_opening("xhi", "adiabatic")                      # one x wall open: no pair needed
    for call in (lambda: L.solute_opening_range("xlo", 5, 9, "inlet", "dirichlet", 1.0),   # overlap
                 lambda: L.solute_opening_range("ylo", 0, 4, "inlet", "dirichlet", 1.0)):  # corner (0,0)
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_INVAL
    L.solute_opening_range("ylo", 1, 4, "inlet", "dirichlet", 1.0)
    L.momentum_opening("xlo", 1, 10, 0, "inlet", "poiseuille", 0.02, 1.0)
    with pytest.raises(lb2d.LB2DError) as e:
        L.momentum_opening("xlo", 10, 11, 0, "outlet", "dirichlet", 0.0, 1.0)
    assert e.value.code == lb2d.E_INVAL


def test_null_handles_do_not_crash():
    from paper_1202_0442_amd.lb2d import _lib
    assert _lib.lb2d_lattice(None, b"d2q9", 4, 4, 1.0) == -1
    assert _lib.lb2d_iteration(None, 1) == -1
    assert _lib.lb2d_destroy(None) == -1
    assert _lib.lb2d_last_error(None) == b"null context"


def test_rounding_command_checks():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    with pytest.raises(lb2d.LB2DError) as e:
        L.rounding("stochastic")
    assert e.value.code == lb2d.E_ORDER
    L.lattice("d2q9", 16, 16, 1.0)
    with pytest.raises(lb2d.LB2DError) as e:
        L.rounding("truncate")
    assert e.value.code == lb2d.E_INVAL
    L.rounding("stochastic", 3)
    for st in ("f32", "f64"):
        with pytest.raises(lb2d.LB2DError) as e:
            L.workspace_bytes(st)
        assert e.value.code == lb2d.E_UNSUPPORTED
    assert L.workspace_bytes("f16") > 0
    L.rounding("nearest")
    assert L.workspace_bytes("f32") > 0


def test_psi_force_forms():
    """One component: interforce / adhesiveforce take psi0 and rho0 (psi
    form); two components take neither."""
    lb2d = _lb2d()
    one = lb2d.Lattice()
    one.lattice("d2q9", 12, 10, 1.0)
    for call in (lambda: one.interforce(-120.0), lambda: one.interforce(-120.0, 4.0, 0.0),
                 lambda: one.adhesiveforce(-200.0, 0), lambda: one.adhesiveforce(-200.0, 1, 4.0, 200.0)):
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_INVAL
    one.interforce(-120.0, 4.0, 200.0)
    one.adhesiveforce(-200.0, 0, 4.0, 200.0)
    two = lb2d.Lattice()
    two.lattice("d2q9", 12, 10, 1.0)
    two.fluids(1.0, 1.0)
    for call in (lambda: two.interforce(0.9, 4.0, 200.0), lambda: two.adhesiveforce(0.3, 0, 4.0, 200.0)):
        with pytest.raises(lb2d.LB2DError) as e:
            call()
        assert e.value.code == lb2d.E_INVAL
    two.interforce(0.9)
    two.adhesiveforce(0.3, 1)


def test_initial_fields_must_be_finite():
    lb2d = _lb2d()
    L = lb2d.Lattice()
    L.lattice("d2q9", 6, 5, 1.0)
    ok = np.ones(30)
    bad = ok.copy()
    bad[7] = float("nan")
    for args in ((0, bad), (0, ok, bad), (0, ok, None, bad * float("inf")), (0, -ok)):
        with pytest.raises(lb2d.LB2DError) as e:
            L.set_fields(*args)
        assert e.value.code == lb2d.E_INVAL
    L.set_fields(0, ok, 0.01 * ok, None)
    L.solute(1.0, 9)
    for args in ((bad,), (ok, bad)):
        with pytest.raises(lb2d.LB2DError) as e:
            L.set_concentration(*args)
        assert e.value.code == lb2d.E_INVAL
    L.set_concentration(ok)
