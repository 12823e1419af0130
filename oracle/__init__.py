"""Serial FP64 CPU oracle for the Klinkenberg lattice Boltzmann model of
arXiv:1411.7051 (Chen et al.), loaded through ctypes from ``oracle/liblbo.so``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product path (``paper_1411_7051_amd``) never imports it, and the two share no
code; they meet only in the seeded input generators of
``paper_1411_7051_amd.inputs``, which hold none of the method's arithmetic.

The arithmetic lives in ``lbo.c`` (D2Q9) and ``lbo3.c`` (D3Q19), one node
at a time, FP64, phases kept apart.  This module only marshals arrays and adds the finite-difference
gradient, which is the plain definition of a derivative applied to the
oracle's own time stepping.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.environ.get("LBO_SRC", os.path.join(_HERE, "lbo.c"))
_SRC3 = os.environ.get("LBO_SRC3", os.path.join(_HERE, "lbo3.c"))
_LIB = os.environ.get("LBO_LIB", os.path.join(_HERE, "liblbo.so"))

PERIODIC, WALL, PRESSURE = 0, 1, 2

# Eq. 13 and the weights after Eq. 14, for callers that post-process states.
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def build(force: bool = True) -> str:
    """Compile ``liblbo.so`` with gcc: -O2, no FMA contraction, no fast-math."""
    srcs = [_SRC, _SRC3]
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < max(os.path.getmtime(s) for s in srcs):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-Wall", "-Wextra", "-I", _HERE, "-o", tmp, *srcs, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("f_eps", ctypes.c_double),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("rho0", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("kn_local", ctypes.c_int), ("init", ctypes.c_int),
        ("eq15_printed", ctypes.c_int),
        ("correlation", ctypes.c_int), ("slip_b", ctypes.c_double),
    ]


class _Params3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("gz", ctypes.c_double),
        ("f_eps", ctypes.c_double),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("bc_z", ctypes.c_int),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("rho0", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("kn_local", ctypes.c_int), ("init", ctypes.c_int), ("correlation", ctypes.c_int),
        ("slip_b", ctypes.c_double),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.lbo_fc.restype = ctypes.c_double
        lib.lbo_fc.argtypes = [ctypes.c_double]
        lib.lbo_fc_with.restype = ctypes.c_double
        lib.lbo_fc_with.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.lbo_feq.argtypes = [ctypes.c_double] * 4 + [_D]
        lib.lbo_guo.argtypes = [ctypes.c_double] * 7 + [ctypes.c_int, _D]
        lib.lbo_node_macro.argtypes = [ctypes.POINTER(_Params), _D] + [ctypes.c_double] * 3 + [_D] * 5
        lib.lbo_collide_node.argtypes = [ctypes.POINTER(_Params), _D] + [ctypes.c_double] * 3 + [_D]
        lib.lbo_create.restype = ctypes.c_void_p
        lib.lbo_create.argtypes = [ctypes.POINTER(_Params), _D, _D, _D]
        lib.lbo_destroy.argtypes = [ctypes.c_void_p]
        lib.lbo_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        lib.lbo_macro.argtypes = [ctypes.c_void_p, _D, _D, _D]
        lib.lbo_mass.restype = ctypes.c_double
        lib.lbo_mass.argtypes = [ctypes.c_void_p]
        lib.lbo_apparent_permeability.restype = ctypes.c_double
        lib.lbo_apparent_permeability.argtypes = [ctypes.c_void_p]
        lib.lbo_get_state.argtypes = [ctypes.c_void_p, _D]
        lib.lbo_set_state.argtypes = [ctypes.c_void_p, _D]
        lib.lbo_residual.restype = ctypes.c_double
        lib.lbo_residual.argtypes = [_D, _D, ctypes.c_size_t]
        lib.lbo_nonfinite.restype = ctypes.c_int
        lib.lbo_nonfinite.argtypes = [ctypes.c_void_p]
        P3 = ctypes.POINTER(_Params3)
        I19 = ctypes.POINTER(ctypes.c_int)
        lib.lbo3_tables.argtypes = [I19, I19, I19, _D]
        lib.lbo3_feq.argtypes = [ctypes.c_double, _D, ctypes.c_double, _D]
        lib.lbo3_guo.argtypes = [ctypes.c_double, _D, _D, ctypes.c_double, ctypes.c_double, _D]
        lib.lbo3_create.restype = ctypes.c_void_p
        lib.lbo3_create.argtypes = [P3, _D, _D, _D]
        lib.lbo3_destroy.argtypes = [ctypes.c_void_p]
        lib.lbo3_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        lib.lbo3_macro.argtypes = [ctypes.c_void_p, _D, _D, _D, _D]
        lib.lbo3_mass.restype = ctypes.c_double
        lib.lbo3_mass.argtypes = [ctypes.c_void_p]
        lib.lbo3_apparent_permeability.restype = ctypes.c_double
        lib.lbo3_apparent_permeability.argtypes = [ctypes.c_void_p]
        lib.lbo3_get_state.argtypes = [ctypes.c_void_p, _D]
        lib.lbo3_set_state.argtypes = [ctypes.c_void_p, _D]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _params(nx, ny, tau=0.8, gx=0.0, gy=0.0, f_eps=0.0, bc_x=PERIODIC,
            bc_y=PERIODIC, rho_in=1.0, rho_out=1.0, rho0=1.0, rho_ref=1.0,
            kn_local=1, init=0, eq15_printed=0, correlation=0, slip_b=-1.0) -> _Params:
    return _Params(int(nx), int(ny), float(tau), float(gx), float(gy),
                   float(f_eps), int(bc_x), int(bc_y), float(rho_in),
                   float(rho_out), float(rho0), float(rho_ref), int(kn_local),
                   int(init), int(eq15_printed), int(correlation), float(slip_b))


def fc(kn: float, correlation: int = 0, slip_b: float = -1.0) -> float:
    """Correction factor f_c(Kn): Eqs. 6-7 with slip coefficient b
    (correlation 0; b = -1 by default), Eqs. 4-5 (1: 1 + 4 Kn) or none (2);
    f_c(0) = 1."""
    if correlation == 0 and slip_b == -1.0:
        return _load().lbo_fc(float(kn))
    return _load().lbo_fc_with(int(correlation), float(slip_b), float(kn))


def feq(rho, ux, uy, eps) -> np.ndarray:
    """Eq. 14 at one node."""
    out = np.zeros(9)
    _load().lbo_feq(rho, ux, uy, eps, _ptr(out))
    return out


def guo(rho, ux, uy, fx, fy, eps, tau, printed=False) -> np.ndarray:
    """Eq. 15 at one node (printed=True: the last term exactly as printed)."""
    out = np.zeros(9)
    _load().lbo_guo(rho, ux, uy, fx, fy, eps, tau, int(printed), _ptr(out))
    return out


def node_macro(f, eps, k, kn0=0.0, **params):
    """Eqs. 16-17 at one node: (rho, ux, uy, Fx, Fy)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    p = _params(1, 1, **params)
    outs = [ctypes.c_double() for _ in range(5)]
    _load().lbo_node_macro(ctypes.byref(p), _ptr(f), eps, k, kn0,
                           *[ctypes.byref(o) for o in outs])
    return tuple(o.value for o in outs)


def collide_node(f, eps, k, kn0=0.0, **params) -> np.ndarray:
    """Eq. 12 right-hand side at one node."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    p = _params(1, 1, **params)
    _load().lbo_collide_node(ctypes.byref(p), _ptr(f), eps, k, kn0, _ptr(out))
    return out


class Lattice:
    """One oracle lattice.  Fields are [ny][nx]; ``k`` may hold +inf."""

    def __init__(self, eps, k, kn0=None, **params):
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        k = np.ascontiguousarray(k, dtype=np.float64)
        if eps.ndim != 2 or eps.shape != k.shape:
            raise ValueError("eps and k must be 2-D arrays of one shape")
        self.ny, self.nx = eps.shape
        self._kn0 = None if kn0 is None else np.ascontiguousarray(kn0, dtype=np.float64)
        self._eps, self._k = eps, k
        self.params = dict(params)
        self._p = _params(self.nx, self.ny, **params)
        lib = _load()
        h = lib.lbo_create(ctypes.byref(self._p), _ptr(eps), _ptr(k),
                           None if self._kn0 is None else _ptr(self._kn0))
        if not h:
            raise ValueError("oracle rejected the lattice description")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _load().lbo_destroy(h)
            except TypeError:  # interpreter shutdown: module globals already gone
                pass
            self._h = None

    def step(self, n: int = 1) -> "Lattice":
        _load().lbo_step(self._h, int(n))
        return self

    def macro(self):
        """(rho, ux, uy) at the current time, each [ny][nx] float64."""
        shape = (self.ny, self.nx)
        rho, ux, uy = np.zeros(shape), np.zeros(shape), np.zeros(shape)
        _load().lbo_macro(self._h, _ptr(rho), _ptr(ux), _ptr(uy))
        return rho, ux, uy

    def mass(self) -> float:
        return _load().lbo_mass(self._h)

    def apparent_permeability(self) -> float:
        return _load().lbo_apparent_permeability(self._h)

    def state(self) -> np.ndarray:
        f = np.zeros((9, self.ny, self.nx))
        _load().lbo_get_state(self._h, _ptr(f))
        return f

    def set_state(self, f) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (9, self.ny, self.nx):
            raise ValueError("state must be [9][ny][nx]")
        _load().lbo_set_state(self._h, _ptr(f))

    def nonfinite(self) -> bool:
        return bool(_load().lbo_nonfinite(self._h))


def residual(u, u_prev) -> float:
    """Steady-state residual ||u - u_prev||_2 / ||u||_2 (FP64) between two
    velocity read-outs, each a sequence of component arrays of one shape
    (ux, uy) or (ux, uy, uz); 0 when both are zero, +inf when only u_prev
    is non-zero."""
    a = np.ascontiguousarray(np.stack([np.asarray(c, dtype=np.float64) for c in u]).ravel())
    b = np.ascontiguousarray(np.stack([np.asarray(c, dtype=np.float64) for c in u_prev]).ravel())
    if a.shape != b.shape:
        raise ValueError("u and u_prev must have the same shape")
    return _load().lbo_residual(_ptr(a), _ptr(b), a.size)


def objective(lat: Lattice, name: str) -> float:
    """Scalar objectives whose gradients are checked: the global apparent
    permeability, or the outlet mass flux sum_y rho u_x on column nx-1."""
    if name == "k_app":
        return lat.apparent_permeability()
    if name == "q_out":
        rho, ux, _ = lat.macro()
        return float(np.sum(rho[:, -1] * ux[:, -1]))
    raise ValueError(name)


def fd_gradient(eps, k, kn0, steps, nodes, objective_name="k_app", h=1e-4,
                wrt="k", **params) -> np.ndarray:
    """Central finite differences of the objective after ``steps`` steps with
    respect to ln k (``wrt="k"``, kn0 held fixed) or ln kn0 (``wrt="kn0"``, k
    held fixed) at each (y, x) in ``nodes``: (J(ln p + h) - J(ln p - h)) / 2h."""
    if wrt not in ("k", "kn0"):
        raise ValueError(wrt)
    out = np.zeros(len(nodes))
    k = np.asarray(k, dtype=np.float64)
    kn0 = np.zeros_like(k) if kn0 is None else np.asarray(kn0, dtype=np.float64)
    for j, (y, x) in enumerate(nodes):
        vals = []
        for s in (+1.0, -1.0):
            kk, kn = k.copy(), kn0.copy()
            field = kk if wrt == "k" else kn
            field[y, x] = field[y, x] * math.exp(s * h)
            lat = Lattice(eps, kk, kn, **params).step(steps)
            vals.append(objective(lat, objective_name))
        out[j] = (vals[0] - vals[1]) / (2.0 * h)
    return out


# ---------------------------------------------------------------- D3Q19


def tables3():
    """(ex, ey, ez, w) of the D3Q19 set as the 3-D oracle numbers it."""
    ex, ey, ez = ((ctypes.c_int * 19)() for _ in range(3))
    w = np.zeros(19)
    _load().lbo3_tables(ex, ey, ez, _ptr(w))
    return np.array(ex), np.array(ey), np.array(ez), w


def feq3(rho, u, eps) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    _load().lbo3_feq(float(rho), _ptr(u), float(eps), _ptr(out))
    return out


def guo3(rho, u, F, eps, tau) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    _load().lbo3_guo(float(rho), _ptr(u), _ptr(F), float(eps), float(tau), _ptr(out))
    return out


class Lattice3:
    """One D3Q19 oracle lattice.  Fields are [nz][ny][nx]; ``k`` may hold
    +inf.  Parameters: tau, gx, gy, gz, f_eps, bc_x, bc_y, bc_z, rho_in,
    rho_out, rho0, rho_ref, kn_local, init, correlation, slip_b."""

    def __init__(self, eps, k, kn0=None, tau=0.8, gx=0.0, gy=0.0, gz=0.0, f_eps=0.0,
                 bc_x=PERIODIC, bc_y=PERIODIC, bc_z=PERIODIC, rho_in=1.0, rho_out=1.0,
                 rho0=1.0, rho_ref=1.0, kn_local=1, init=0, correlation=0, slip_b=-1.0):
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        k = np.ascontiguousarray(k, dtype=np.float64)
        if eps.ndim != 3 or eps.shape != k.shape:
            raise ValueError("eps and k must be 3-D arrays of one shape")
        self.nz, self.ny, self.nx = eps.shape
        self._kn0 = None if kn0 is None else np.ascontiguousarray(kn0, dtype=np.float64)
        self._eps, self._k = eps, k
        self._p = _Params3(self.nx, self.ny, self.nz, float(tau), float(gx), float(gy),
                           float(gz), float(f_eps), int(bc_x), int(bc_y), int(bc_z),
                           float(rho_in), float(rho_out), float(rho0), float(rho_ref),
                           int(kn_local), int(init), int(correlation), float(slip_b))
        h = _load().lbo3_create(ctypes.byref(self._p), _ptr(eps), _ptr(k),
                                None if self._kn0 is None else _ptr(self._kn0))
        if not h:
            raise ValueError("oracle rejected the lattice description")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _load().lbo3_destroy(h)
            except TypeError:
                pass
            self._h = None

    def step(self, n: int = 1) -> "Lattice3":
        _load().lbo3_step(self._h, int(n))
        return self

    def macro(self):
        """(rho, ux, uy, uz), each [nz][ny][nx] float64."""
        shape = (self.nz, self.ny, self.nx)
        out = [np.zeros(shape) for _ in range(4)]
        _load().lbo3_macro(self._h, *[_ptr(a) for a in out])
        return tuple(out)

    def mass(self) -> float:
        return _load().lbo3_mass(self._h)

    def apparent_permeability(self) -> float:
        return _load().lbo3_apparent_permeability(self._h)

    def state(self) -> np.ndarray:
        f = np.zeros((19, self.nz, self.ny, self.nx))
        _load().lbo3_get_state(self._h, _ptr(f))
        return f

    def set_state(self, f) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (19, self.nz, self.ny, self.nx):
            raise ValueError("state must be [19][nz][ny][nx]")
        _load().lbo3_set_state(self._h, _ptr(f))
