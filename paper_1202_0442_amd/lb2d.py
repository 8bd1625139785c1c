"""Thin Python binding of the HIP library ``liblb2d_hip.so`` (C ABI in
``include/lb2d.h``).

Argument marshalling only: every step of the simulation runs in the gfx950
kernels of the library.  PyTorch provides the device workspace (one uint8
tensor per lattice) and the HIP stream.  There is no CPU fallback: if the
library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblb2d_hip.so")

OK, E_INVAL, E_ORDER, E_UNSUPPORTED, E_STATE, E_HIP, E_SIZE = 0, -1, -2, -3, -4, -5, -6
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
NBUDGET = 16
BUDGET_NAMES = (
    "mass0", "mass1", "mom_x", "mom_y", "solute", "deposit",
    "removed_mass0", "removed_mass1", "removed_solute", "inflow", "outflow",
    "steps", "grown_nodes", "fluid_nodes", "consumed_deposit", "reserved15",
)
NAN = float("nan")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -m paper_1202_0442_amd.build` "
        "(hipcc --offload-arch=gfx950) first")

# PyTorch ships its own HIP runtime (same soname as the system one).  Loading
# torch first makes the library bind to that runtime instead of starting a
# second HIP/HSA runtime in the process, which would leave torch without GPUs.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)
_P, _I, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_DP = ctypes.POINTER(ctypes.c_double)
_U8P = ctypes.POINTER(ctypes.c_uint8)
_I64 = ctypes.c_int64
_SIGS = {
    "lb2d_create": [ctypes.POINTER(_P), _I],
    "lb2d_destroy": [_P],
    "lb2d_lattice": [_P, ctypes.c_char_p, _I, _I, _D],
    "lb2d_fluids": [_P, _D, _D, _D, _D],
    "lb2d_solute": [_P, _D, _I],
    "lb2d_solute_opening": [_P, ctypes.c_char_p, ctypes.c_char_p, _D],
    "lb2d_boundary_style": [_P, ctypes.c_char_p, ctypes.c_double],
    "lb2d_intersolute": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "lb2d_obstacle_style": [_P, ctypes.c_int, ctypes.c_char_p, ctypes.c_double],
    "lb2d_rounding": [_P, ctypes.c_char_p, ctypes.c_uint64],
    "lb2d_solute_opening_range": [_P, ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p,
                                  ctypes.c_double, ctypes.c_double],
    "lb2d_momentum_opening": [_P, ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char_p,
                              ctypes.c_char_p, ctypes.c_double, ctypes.c_double],
    "lb2d_obstacle_rect": [_P, _I, _I, _I, _I],
    "lb2d_obstacle_circle": [_P, _I, _I, _D],
    "lb2d_obstacle_mask": [_P, _U8P],
    "lb2d_surface_reaction": [_P, _D, _D, ctypes.c_char_p, _D, _D, ctypes.c_uint64],
    "lb2d_set_fields": [_P, _I, _DP, _DP, _DP],
    "lb2d_set_concentration": [_P, _DP, _DP, _DP],
    "lb2d_aveforce": [_P, _I, _D, _I],
    "lb2d_aveacceleration": [_P, _I, _D, _I],
    "lb2d_interforce": [_P, _D, _D, _D],
    "lb2d_adhesiveforce": [_P, _D, _D, _D, _I],
    "lb2d_workspace_bytes": [_P, _I, ctypes.POINTER(_SZ)],
    "lb2d_bind": [_P, _P, _SZ, _P],
    "lb2d_iteration": [_P, _I64],
    "lb2d_prepare": [_P, _I64],
    "lb2d_steps_per_launch": [_P, ctypes.POINTER(_I)],
    "lb2d_batch_steps_per_launch": [_P, ctypes.POINTER(_I)],
    "lb2d_moments": [_P, _I, _DP, _DP, _DP],
    "lb2d_solute_state": [_P, _DP, _DP],
    "lb2d_mask": [_P, _U8P],
    "lb2d_budgets": [_P, _DP],
    "lb2d_budgets_noalloc": [_P, _DP],
    "lb2d_get_populations": [_P, _I, _DP],
    "lb2d_set_populations": [_P, _I, _DP],
    "lb2d_get_deposit": [_P, _DP],
    "lb2d_set_deposit": [_P, _DP],
    "lb2d_set_mask": [_P, _U8P],
    "lb2d_step_count": [_P, ctypes.POINTER(_I64)],
    "lb2d_checkpoint_bytes": [_P, ctypes.POINTER(_SZ)],
    "lb2d_checkpoint_save": [_P, _P, _SZ],
    "lb2d_checkpoint_load": [_P, _P, _SZ],
    "lb2d_set_timing": [_P, _I],
    "lb2d_kernel_time": [_P, _DP, ctypes.POINTER(_I64)],
    "lb2d_batch_create": [ctypes.POINTER(_P), _I],
    "lb2d_batch_destroy": [_P],
    "lb2d_batch_add": [_P, _P],
    "lb2d_batch_workspace_bytes": [_P, ctypes.POINTER(_SZ)],
    "lb2d_batch_finalize": [_P, _P, _SZ, _P, ctypes.c_char_p],
    "lb2d_batch_iteration": [_P, _I64],
    "lb2d_batch_config": [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                          ctypes.POINTER(_I)],
    "lb2d_batch_trials": [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                          ctypes.POINTER(_I), _DP, ctypes.POINTER(_I)],
    "lb2d_copy_bench": [_P, _P, _SZ, _I, _P, _DP],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _I
_lib.lb2d_last_error.argtypes = [_P]
_lib.lb2d_last_error.restype = ctypes.c_char_p
_lib.lb2d_batch_last_error.argtypes = [_P]
_lib.lb2d_batch_last_error.restype = ctypes.c_char_p

EXPORTED = tuple(_SIGS) + ("lb2d_last_error", "lb2d_batch_last_error")


class LB2DError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _dp(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _arr(a, n, dtype=np.float64):
    if a is None:
        return None
    a = np.asarray(a, dtype)
    if a.ndim == 0:
        a = np.full(n, a, dtype)
    a = np.ascontiguousarray(a.ravel())
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Lattice:
    """One lattice; methods carry the names of the C entry points."""

    def __init__(self, device: int = 0):
        self._h = _P()
        self.device = device
        self.workspace = None
        self.stream = None
        self._chk(_lib.lb2d_create(ctypes.byref(self._h), device))
        self.nx = self.ny = 0
        self.ncomp = 1

    def _chk(self, rc):
        if rc != OK:
            msg = _lib.lb2d_last_error(self._h) if getattr(self, "_h", None) else b""
            raise LB2DError(rc, (msg or b"").decode())
        return rc

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lb2d_destroy(self._h)
            self._h = _P()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # commands
    def lattice(self, style, nx, ny, tau):
        self._chk(_lib.lb2d_lattice(self._h, style.encode(), int(nx), int(ny), float(tau)))
        self.nx, self.ny = int(nx), int(ny)

    def fluids(self, tau1, tau2, alpha1=NAN, alpha2=NAN):
        self._chk(_lib.lb2d_fluids(self._h, tau1, tau2, alpha1, alpha2))
        self.ncomp = 2

    def solute(self, tau_s, q=9):
        self._chk(_lib.lb2d_solute(self._h, tau_s, q))

    def solute_opening(self, wall, style, value=0.0):
        self._chk(_lib.lb2d_solute_opening(self._h, wall.encode(), style.encode(), value))

    def intersolute(self, G, psi0, C0):
        self._chk(_lib.lb2d_intersolute(self._h, float(G), float(psi0), float(C0)))

    def boundary_style(self, style, R=0.0):
        self._chk(_lib.lb2d_boundary_style(self._h, style.encode(), float(R)))

    def obstacle_style(self, comp, style, R=0.0):
        self._chk(_lib.lb2d_obstacle_style(self._h, int(comp), style.encode(), float(R)))

    def momentum_opening(self, wall, lo, hi, comp, kind, style, v=0.0, rho=1.0):
        """inlet/outlet + inlet_momentum/outlet_momentum: nodes lo..hi of a
        wall; style poiseuille, uniform, dirichlet or gradient."""
        self._chk(_lib.lb2d_momentum_opening(self._h, wall.encode(), lo, hi, comp, kind.encode(), style.encode(),
                                             float(v), float(rho)))

    def solute_opening_range(self, wall, lo, hi, kind, style, value=0.0, v=0.0):
        """inlet_solute / outlet_solute on nodes lo..hi of a wall; style
        dirichlet, adiabatic or flux (value = C0, v = injection velocity)."""
        self._chk(_lib.lb2d_solute_opening_range(self._h, wall.encode(), lo, hi, kind.encode(), style.encode(),
                                                 float(value), float(v)))

    def rounding(self, mode, seed=0):
        """'nearest' or 'stochastic' rounding of 16-bit storage."""
        self._chk(_lib.lb2d_rounding(self._h, mode.encode(), int(seed)))

    def obstacle_rect(self, x0, x1, y0, y1):
        self._chk(_lib.lb2d_obstacle_rect(self._h, x0, x1, y0, y1))

    def obstacle_circle(self, xc, yc, r):
        self._chk(_lib.lb2d_obstacle_circle(self._h, int(xc), int(yc), float(r)))

    def obstacle_mask(self, m):
        a = _arr(m, self.nx * self.ny, np.uint8)
        self._chk(_lib.lb2d_obstacle_mask(self._h, a.ctypes.data_as(_U8P)))

    def surface_reaction(self, kr, Cs, style, b0, bmax, seed):
        self._chk(_lib.lb2d_surface_reaction(self._h, kr, Cs, style.encode(), b0, bmax, seed))

    def set_fields(self, comp, rho, ux=None, uy=None):
        n = self.nx * self.ny
        r, a, b = _arr(rho, n), _arr(ux, n), _arr(uy, n)
        self._chk(_lib.lb2d_set_fields(self._h, comp, _dp(r), _dp(a), _dp(b)))

    def set_concentration(self, C, ux=None, uy=None):
        n = self.nx * self.ny
        c, a, b = _arr(C, n), _arr(ux, n), _arr(uy, n)
        self._chk(_lib.lb2d_set_concentration(self._h, _dp(c), _dp(a), _dp(b)))

    def aveforce(self, mode, value, comp=0):
        self._chk(_lib.lb2d_aveforce(self._h, mode, value, comp))

    def aveacceleration(self, mode, value, comp=0):
        self._chk(_lib.lb2d_aveacceleration(self._h, mode, value, comp))

    def interforce(self, G, psi0=NAN, rho0=NAN):
        self._chk(_lib.lb2d_interforce(self._h, G, psi0, rho0))

    def adhesiveforce(self, G, comp, psi0=NAN, rho0=NAN):
        self._chk(_lib.lb2d_adhesiveforce(self._h, G, psi0, rho0, comp))

    # memory
    def workspace_bytes(self, storage="f32"):
        out = _SZ(0)
        self._chk(_lib.lb2d_workspace_bytes(self._h, STORAGE[storage], ctypes.byref(out)))
        return out.value

    def bind(self, storage="f32", stream=None, workspace=None):
        """Allocates the workspace as a torch uint8 tensor on cuda:device
        (unless one is given) and binds it with the stream."""
        import torch
        nbytes = self.workspace_bytes(storage)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        self.workspace = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._chk(_lib.lb2d_bind(self._h, ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel() * workspace.element_size(),
                                 ctypes.c_void_p(self.stream.cuda_stream)))

    # action
    def iteration(self, nsteps):
        self._chk(_lib.lb2d_iteration(self._h, int(nsteps)))

    def prepare(self, nsteps):
        """Captures the launch graphs of a later iteration(nsteps)."""
        self._chk(_lib.lb2d_prepare(self._h, int(nsteps)))

    def steps_per_launch(self):
        """lb2d_steps_per_launch: 5 where the graphs run the multi-step kernel."""
        v = _I(0)
        self._chk(_lib.lb2d_steps_per_launch(self._h, ctypes.byref(v)))
        return v.value

    # output
    def moments(self, comp=0):
        n = self.nx * self.ny
        rho, ux, uy = np.empty(n), np.empty(n), np.empty(n)
        self._chk(_lib.lb2d_moments(self._h, comp, _dp(rho), _dp(ux), _dp(uy)))
        s = (self.ny, self.nx)
        return rho.reshape(s), ux.reshape(s), uy.reshape(s)

    def solute_state(self):
        n = self.nx * self.ny
        C, b = np.empty(n), np.empty(n)
        self._chk(_lib.lb2d_solute_state(self._h, _dp(C), _dp(b)))
        return C.reshape(self.ny, self.nx), b.reshape(self.ny, self.nx)

    def mask(self):
        m = np.empty(self.nx * self.ny, np.uint8)
        self._chk(_lib.lb2d_mask(self._h, m.ctypes.data_as(_U8P)))
        return m.reshape(self.ny, self.nx)

    def budgets(self):
        out = np.zeros(NBUDGET)
        self._chk(_lib.lb2d_budgets(self._h, _dp(out)))
        return dict(zip(BUDGET_NAMES, out.tolist()))

    def budgets_noalloc(self):
        """lb2d_budgets_noalloc: the budgets with the library's static
        scratch instead of the workspace's."""
        out = np.zeros(NBUDGET)
        self._chk(_lib.lb2d_budgets_noalloc(self._h, _dp(out)))
        return dict(zip(BUDGET_NAMES, out.tolist()))

    def get_populations(self, comp=0):
        out = np.empty(9 * self.nx * self.ny)
        self._chk(_lib.lb2d_get_populations(self._h, comp, _dp(out)))
        return out.reshape(9, self.ny, self.nx)

    def set_populations(self, f, comp=0):
        a = _arr(f, 9 * self.nx * self.ny)
        self._chk(_lib.lb2d_set_populations(self._h, comp, _dp(a)))

    def get_deposit(self):
        out = np.empty(self.nx * self.ny)
        self._chk(_lib.lb2d_get_deposit(self._h, _dp(out)))
        return out.reshape(self.ny, self.nx)

    def set_deposit(self, b):
        a = _arr(b, self.nx * self.ny)
        self._chk(_lib.lb2d_set_deposit(self._h, _dp(a)))

    def set_mask(self, m):
        a = _arr(m, self.nx * self.ny, np.uint8)
        self._chk(_lib.lb2d_set_mask(self._h, a.ctypes.data_as(_U8P)))

    def step_count(self):
        t = _I64(0)
        self._chk(_lib.lb2d_step_count(self._h, ctypes.byref(t)))
        return t.value

    def checkpoint(self):
        """The lattice's device state and step count as bytes."""
        n = _SZ(0)
        self._chk(_lib.lb2d_checkpoint_bytes(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._chk(_lib.lb2d_checkpoint_save(self._h, buf, n.value))
        return buf.raw

    def restore(self, data: bytes):
        """Loads a checkpoint() of a lattice set up the same way."""
        buf = ctypes.create_string_buffer(data, len(data))
        self._chk(_lib.lb2d_checkpoint_load(self._h, buf, len(data)))

    def set_timing(self, on=True):
        self._chk(_lib.lb2d_set_timing(self._h, 1 if on else 0))

    def kernel_time(self):
        ms, k = _D(0), _I64(0)
        self._chk(_lib.lb2d_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value


class Batch:
    """Many one-fluid lattices advanced together (one launch per step)."""

    def __init__(self, device: int = 0):
        self._h = _P()
        self.device = device
        self.members = []
        self.workspace = None
        r = _lib.lb2d_batch_create(ctypes.byref(self._h), device)
        if r != OK:
            raise LB2DError(r, "batch create failed")

    def _chk(self, rc):
        if rc != OK:
            raise LB2DError(rc, (_lib.lb2d_batch_last_error(self._h) or b"").decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lb2d_batch_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, lat: Lattice):
        self._chk(_lib.lb2d_batch_add(self._h, lat.handle))
        self.members.append(lat)

    def finalize(self, stream=None, tune_cache=None):
        import torch
        n = _SZ(0)
        self._chk(_lib.lb2d_batch_workspace_bytes(self._h, ctypes.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=f"cuda:{self.device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._chk(_lib.lb2d_batch_finalize(
            self._h, ctypes.c_void_p(self.workspace.data_ptr()), n.value,
            ctypes.c_void_p(self.stream.cuda_stream),
            tune_cache.encode() if tune_cache else None))

    def iteration(self, nsteps):
        self._chk(_lib.lb2d_batch_iteration(self._h, int(nsteps)))

    def config(self):
        v = [_I(0) for _ in range(4)]
        self._chk(_lib.lb2d_batch_config(self._h, *[ctypes.byref(x) for x in v]))
        return dict(tile_w=v[0].value, tile_h=v[1].value, schedule=v[2].value,
                    blocks_per_cu=v[3].value)

    def steps_per_launch(self):
        """lb2d_batch_steps_per_launch: 5 when the multi-step tile was chosen."""
        v = _I(0)
        self._chk(_lib.lb2d_batch_steps_per_launch(self._h, ctypes.byref(v)))
        return v.value

    def trials(self):
        """The autotuner's trials: list of dicts (tile_w, tile_h, schedule,
        blocks_per_cu, ms per step); empty when a tune cache gave the
        choice."""
        cnt = _I(0)
        self._chk(_lib.lb2d_batch_trials(self._h, 0, None, None, None, None, None, ctypes.byref(cnt)))
        n = cnt.value
        if n == 0:
            return []
        ints = [(_I * n)() for _ in range(4)]
        ms = (_D * n)()
        self._chk(_lib.lb2d_batch_trials(self._h, n, *ints, ms, ctypes.byref(cnt)))
        return [dict(tile_w=ints[0][k], tile_h=ints[1][k], schedule=ints[2][k], blocks_per_cu=ints[3][k],
                     ms=ms[k]) for k in range(n)]


def copy_bench(nbytes: int, reps: int = 20, stream=None):
    """Average ms of a device copy of nbytes (read + write) on the stream."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    ms = _D(0)
    r = _lib.lb2d_copy_bench(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nbytes, reps,
                             ctypes.c_void_p(s.cuda_stream), ctypes.byref(ms))
    if r != OK:
        raise LB2DError(r, "copy bench failed")
    return ms.value


def nan():
    return math.nan
