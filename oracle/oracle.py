"""ctypes wrapper of the plain-C FP64 oracle (``lb2d_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the HIP library or its
binding.  It shares no code with the HIP path.

Arrays follow the row-major [ny][nx] layout (x fastest); populations are
[9][ny][nx].  Velocity numbering: e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0),
e4=(0,-1), e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb2d_oracle.c")
_LIB = os.path.join(_HERE, "liblb2d_oracle.so")

BUDGET_NAMES = (
    "mass0", "mass1", "mom_x", "mom_y", "solute", "deposit",
    "removed_mass0", "removed_mass1", "removed_solute", "inflow", "outflow",
    "steps", "grown_nodes", "fluid_nodes", "consumed_deposit", "reserved15",
)

STYLE = {"dirichlet": 1, "adiabatic": 2}
WALL = {"xlo": 0, "xhi": 1}


# plain -O2, no fast-math, no contraction; OpenMP over rows (results do not
# depend on the thread count)
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC"]


def compile_source(src: str, out: str, extra=()) -> str:
    """gcc build of an oracle source file into the shared library `out`."""
    subprocess.check_call(["gcc", *CFLAGS, *extra, src, "-o", out + ".tmp", "-lm"])
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


_lib = None


def load_library(path):
    """ctypes handle of an oracle library built at `path`, with the call
    signatures set.  The default library is built from ``lb2d_oracle.c``;
    tests also build deliberately broken copies of it to check that the
    pins catch plausible mistakes."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    L = ctypes.c_long
    DP = ctypes.POINTER(ctypes.c_double)
    U8P = ctypes.POINTER(ctypes.c_uint8)
    sig = {
        "orc_create": (P, [I, I]),
        "orc_destroy": (None, [P]),
        "orc_fluids": (I, [P, I, D, D, D, D]),
        "orc_aveforce": (I, [P, I, I, D]),
        "orc_aveacceleration": (I, [P, I, I, D]),
        "orc_interforce": (I, [P, D]),
        "orc_adhesiveforce": (I, [P, I, D]),
        "orc_interforce_psi": (I, [P, D, D, D]),
        "orc_momentum_opening": (I, [P, I, I, I, I, I, I, D, D]),
        "orc_adhesiveforce_psi": (I, [P, D, D, D]),
        "orc_solute": (I, [P, I, D]),
        "orc_intersolute": (I, [P, D, D, D]),
        "orc_solute_opening": (I, [P, I, I, D]),
        "orc_solute_opening_range": (I, [P, I, I, I, I, I, D, D]),
        "orc_surface_reaction": (I, [P, D, D, D, D, ctypes.c_uint64]),
        "orc_obstacle_circle": (I, [P, I, I, D]),
        "orc_obstacle_rect": (I, [P, I, I, I, I]),
        "orc_boundary_style": (I, [P, I, D]),
        "orc_obstacle_style": (I, [P, I, D]),
        "orc_set_fields": (I, [P, I, DP, DP, DP]),
        "orc_set_concentration": (I, [P, DP, DP, DP]),
        "orc_step": (I, [P, L]),
        "orc_moments": (I, [P, I, DP, DP, DP]),
        "orc_solute_state": (I, [P, DP, DP]),
        "orc_budgets": (I, [P, DP]),
        "orc_step_count": (L, [P]),
        "orc_set_step_count": (None, [P, L]),
        "orc_get_f": (I, [P, I, DP]),
        "orc_set_f": (I, [P, I, DP]),
        "orc_get_g": (I, [P, DP]),
        "orc_set_g": (I, [P, DP]),
        "orc_get_mask": (I, [P, U8P]),
        "orc_set_mask": (I, [P, U8P]),
        "orc_get_b": (I, [P, DP]),
        "orc_get_bdec": (I, [P, DP]),
        "orc_set_b": (I, [P, DP]),
        "orc_forces": (I, [P, I, DP, DP]),
        "orc_feq": (D, [I, D, D, D, D]),
        "orc_geq": (D, [I, I, D, D, D]),
        "orc_reactive_link": (D, [I, I, D, D, D, DP]),
        "orc_splitmix64": (ctypes.c_uint64, [ctypes.c_uint64]),
        "orc_pick": (I, [ctypes.c_uint64, I]),
        "orc_set_threads": (I, [I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = load_library(_LIB)
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, n):
    a = np.asarray(a, np.float64)
    if a.ndim == 0:
        a = np.full(n, float(a))
    a = np.ascontiguousarray(a.ravel())
    assert a.size == n
    return a


def feq(i, rho, ux, uy, alpha=4.0 / 9.0):
    return _load().orc_feq(i, rho, ux, uy, alpha)


def geq(q, i, C, ux, uy):
    return _load().orc_geq(q, i, C, ux, uy)


def reactive_link(q, i, kr, Cs, g_out):
    """Returns (deposit, returning population) of one reactive link."""
    gi = ctypes.c_double(0.0)
    db = _load().orc_reactive_link(q, i, kr, Cs, g_out, ctypes.byref(gi))
    return db, gi.value


def splitmix64(x):
    return _load().orc_splitmix64(x & 0xFFFFFFFFFFFFFFFF)


def pick(h, m):
    return _load().orc_pick(h, m)


def set_threads(n=0):
    """Sets the oracle's OpenMP thread count (n <= 0 keeps it); returns the
    count in use."""
    return _load().orc_set_threads(int(n))


class Oracle:
    """One lattice.  Command methods mirror the paper's commands."""

    def __init__(self, nx, ny, lib=None):
        self.lib = _load() if lib is None else lib
        self.nx, self.ny = int(nx), int(ny)
        self.n = self.nx * self.ny
        self.h = self.lib.orc_create(self.nx, self.ny)
        if not self.h:
            raise ValueError("bad lattice size")
        self.ncomp = 1
        self.q = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    def _chk(self, rc, what):
        if rc != 0:
            raise ValueError(f"oracle {what} rejected its arguments")

    # commands -----------------------------------------------------------
    def fluids(self, ncomp, tau0, tau1=1.0, alpha0=4.0 / 9.0, alpha1=4.0 / 9.0):
        self._chk(self.lib.orc_fluids(self.h, ncomp, tau0, tau1, alpha0, alpha1), "fluids")
        self.ncomp = ncomp

    def aveforce(self, mode, value, comp=0):
        self._chk(self.lib.orc_aveforce(self.h, comp, mode, value), "aveforce")

    def aveacceleration(self, mode, value, comp=0):
        self._chk(self.lib.orc_aveacceleration(self.h, comp, mode, value), "aveacceleration")

    def momentum_opening(self, wall, lo, hi, comp, kind, style, v=0.0, rho=1.0):
        """inlet/outlet + inlet_momentum/outlet_momentum: nodes lo..hi of
        wall xlo/xhi/ylo/yhi; kind inlet/outlet; style poiseuille (v =
        v_max), uniform (v), dirichlet (rho held) or gradient; rho = the
        opening nodes' initial density."""
        w = {"xlo": 0, "xhi": 1, "ylo": 2, "yhi": 3}[wall]
        st = {"poiseuille": 1, "uniform": 2, "dirichlet": 3, "gradient": 4}[style]
        self._chk(self.lib.orc_momentum_opening(self.h, w, lo, hi, comp, 1 if kind == "outlet" else 0, st,
                                                v, rho), "momentum_opening")

    def interforce(self, G, psi0=None, rho0=None):
        """Two components: interforce(G); one component: interforce(G, psi0,
        rho0) with psi = psi0 exp(-rho0 / rho)."""
        if psi0 is None:
            self._chk(self.lib.orc_interforce(self.h, G), "interforce")
        else:
            self._chk(self.lib.orc_interforce_psi(self.h, G, psi0, rho0), "interforce")

    def intersolute(self, G, psi0, C0):
        """intersolute(G, psi0, C0); after solute."""
        self._chk(self.lib.orc_intersolute(self.h, float(G), float(psi0), float(C0)), "intersolute")

    def adhesiveforce(self, G, comp=0, psi0=None, rho0=None):
        """Two components: adhesiveforce(G, comp); one component:
        adhesiveforce(G, psi0=, rho0=)."""
        if psi0 is None:
            self._chk(self.lib.orc_adhesiveforce(self.h, comp, G), "adhesiveforce")
        else:
            self._chk(self.lib.orc_adhesiveforce_psi(self.h, G, psi0, rho0), "adhesiveforce")

    def solute(self, tau_s, q=9):
        self._chk(self.lib.orc_solute(self.h, q, tau_s), "solute")
        self.q = q

    def solute_opening_range(self, wall, lo, hi, kind, style, value=0.0, v=0.0):
        """inlet_solute / outlet_solute on nodes lo..hi of wall xlo/xhi/
        ylo/yhi; style dirichlet (value = C), adiabatic, flux (value = C0,
        v = velocity of the injected solution)."""
        w = {"xlo": 0, "xhi": 1, "ylo": 2, "yhi": 3}[wall]
        st = {"dirichlet": 1, "adiabatic": 2, "flux": 3}[style]
        self._chk(self.lib.orc_solute_opening_range(self.h, w, lo, hi, 1 if kind == "outlet" else 0, st,
                                                    value, v), "solute_opening")

    def solute_opening(self, wall, style, value=0.0):
        self._chk(self.lib.orc_solute_opening(self.h, WALL[wall], STYLE[style], value),
                  "solute_opening")

    def surface_reaction(self, kr, Cs, b0, bmax, seed):
        self._chk(self.lib.orc_surface_reaction(self.h, kr, Cs, b0, bmax, seed),
                  "surface_reaction")

    def boundary_style(self, style, R=0.0):
        """noslip, slip, mixed (reflected share R) or hybrid."""
        st = {"noslip": 0, "slip": 1, "mixed": 2, "hybrid": 3}[style]
        self._chk(self.lib.orc_boundary_style(self.h, st, float(R)), "boundary_style")

    def obstacle_style(self, comp, style, R=0.0):
        """Hybrid style: style of component comp for the obstacles that
        follow (noslip, slip or mixed with share R)."""
        v = {"noslip": 0.0, "slip": 1.0}.get(style, R)
        self._chk(self.lib.orc_obstacle_style(self.h, comp, float(v)), "obstacle_style")

    def obstacle_circle(self, xc, yc, r):
        self._chk(self.lib.orc_obstacle_circle(self.h, int(xc), int(yc), float(r)), "circle")

    def obstacle_rect(self, x0, x1, y0, y1):
        self._chk(self.lib.orc_obstacle_rect(self.h, x0, x1, y0, y1), "rectangle")

    def set_fields(self, comp, rho, ux=0.0, uy=0.0):
        r, a, b = _f64(rho, self.n), _f64(ux, self.n), _f64(uy, self.n)
        self._chk(self.lib.orc_set_fields(self.h, comp, _dp(r), _dp(a), _dp(b)), "set_fields")

    def set_concentration(self, C, ux=0.0, uy=0.0):
        c, a, b = _f64(C, self.n), _f64(ux, self.n), _f64(uy, self.n)
        self._chk(self.lib.orc_set_concentration(self.h, _dp(c), _dp(a), _dp(b)),
                  "set_concentration")

    def iteration(self, nsteps):
        self._chk(self.lib.orc_step(self.h, int(nsteps)), "iteration")

    # readout ------------------------------------------------------------
    def moments(self, comp=0):
        rho = np.empty(self.n)
        ux = np.empty(self.n)
        uy = np.empty(self.n)
        self._chk(self.lib.orc_moments(self.h, comp, _dp(rho), _dp(ux), _dp(uy)), "moments")
        s = (self.ny, self.nx)
        return rho.reshape(s), ux.reshape(s), uy.reshape(s)

    def solute_state(self):
        C = np.empty(self.n)
        b = np.empty(self.n)
        self._chk(self.lib.orc_solute_state(self.h, _dp(C), _dp(b)), "solute_state")
        return C.reshape(self.ny, self.nx), b.reshape(self.ny, self.nx)

    def budgets(self):
        out = np.zeros(16)
        self.lib.orc_budgets(self.h, _dp(out))
        return dict(zip(BUDGET_NAMES, out.tolist()))

    def forces(self, comp=0):
        Fx = np.empty(self.n)
        Fy = np.empty(self.n)
        self._chk(self.lib.orc_forces(self.h, comp, _dp(Fx), _dp(Fy)), "forces")
        return Fx.reshape(self.ny, self.nx), Fy.reshape(self.ny, self.nx)

    # raw state ------------------------------------------------------------
    @property
    def t(self):
        return self.lib.orc_step_count(self.h)

    @t.setter
    def t(self, v):
        self.lib.orc_set_step_count(self.h, int(v))

    def get_f(self, comp=0):
        out = np.empty(9 * self.n)
        self.lib.orc_get_f(self.h, comp, _dp(out))
        return out.reshape(9, self.ny, self.nx)

    def set_f(self, f, comp=0):
        a = np.ascontiguousarray(f, np.float64).ravel()
        assert a.size == 9 * self.n
        self.lib.orc_set_f(self.h, comp, _dp(a))

    def get_g(self):
        out = np.empty(9 * self.n)
        self.lib.orc_get_g(self.h, _dp(out))
        return out.reshape(9, self.ny, self.nx)

    def set_g(self, g):
        a = np.ascontiguousarray(g, np.float64).ravel()
        assert a.size == 9 * self.n
        self.lib.orc_set_g(self.h, _dp(a))

    def get_mask(self):
        out = np.empty(self.n, np.uint8)
        self.lib.orc_get_mask(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return out.reshape(self.ny, self.nx)

    def set_mask(self, m):
        a = np.ascontiguousarray(m, np.uint8).ravel()
        assert a.size == self.n
        self.lib.orc_set_mask(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))

    def get_b(self):
        out = np.empty(self.n)
        self.lib.orc_get_b(self.h, _dp(out))
        return out.reshape(self.ny, self.nx)

    def get_bdec(self):
        """Deposits the growth decisions of the last step were taken from
        (after that step's deposit, before the triggering solids were reset
        to zero)."""
        out = np.empty(self.n)
        self.lib.orc_get_bdec(self.h, _dp(out))
        return out.reshape(self.ny, self.nx)

    def set_b(self, b):
        a = np.ascontiguousarray(b, np.float64).ravel()
        assert a.size == self.n
        self.lib.orc_set_b(self.h, _dp(a))
