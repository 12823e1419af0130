"""Python face of the D3Q19 calls of the C ABI: ``Lattice3`` wraps one
``lbk_lattice3`` handle (fields [nz][ny][nx]).  Marshalling only."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import Desc3, check
from .lattice import _field

PERIODIC, WALL, PRESSURE = 0, 1, 2


def make_desc3(nx, ny, nz, tau=0.8, gx=0.0, gy=0.0, gz=0.0, f_eps=0.0, bc_x=PERIODIC,
               bc_y=PERIODIC, bc_z=PERIODIC, rho_in=1.0, rho_out=1.0, rho0=1.0, rho_ref=1.0,
               kn_local=1, init=0, storage="f32", check_every=100, correlation=0,
               slip_b=-1.0) -> Desc3:
    d = Desc3()
    check(_lib.load().lbk3_desc_default(ctypes.byref(d)))
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.tau, d.gx, d.gy, d.gz, d.f_eps = float(tau), float(gx), float(gy), float(gz), float(f_eps)
    d.bc_x, d.bc_y, d.bc_z = int(bc_x), int(bc_y), int(bc_z)
    d.rho_in, d.rho_out, d.rho0, d.rho_ref = float(rho_in), float(rho_out), float(rho0), \
        float(rho_ref)
    d.kn_local, d.init, d.check_every = int(kn_local), int(init), int(check_every)
    d.storage = _lib.STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.correlation = (_lib.CORRELATION[correlation] if isinstance(correlation, str)
                     else int(correlation))
    d.slip_b = float(slip_b)
    return d


def workspace_bytes3(desc: Desc3) -> int:
    n = ctypes.c_size_t()
    check(_lib.load().lbk3_workspace_size(ctypes.byref(desc), ctypes.byref(n)))
    return int(n.value)


class Lattice3:
    """A D3Q19 Klinkenberg lattice on one GPU: ``eps``, ``k``, ``kn0`` are
    [nz][ny][nx]; keywords are those of ``lbk_desc3``."""

    def __init__(self, eps, k, kn0=None, device: Optional[torch.device] = None, **params):
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        e, kk = _field(eps, self.device), _field(k, self.device)
        if e.dim() != 3 or e.shape != kk.shape:
            raise ValueError("eps and k must be 3-D of one shape")
        self.nz, self.ny, self.nx = e.shape
        kn = None if kn0 is None else _field(kn0, self.device)
        if kn is not None and kn.shape != e.shape:
            raise ValueError("kn0 must match eps")
        self.params = dict(params)
        self.desc = make_desc3(self.nx, self.ny, self.nz, **params)
        nbytes = workspace_bytes3(self.desc)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(_lib.load().lbk3_create(ctypes.byref(self.desc), e.data_ptr(), kk.data_ptr(),
                                          None if kn is None else kn.data_ptr(),
                                          self._ws.data_ptr(), nbytes, self.stream.cuda_stream,
                                          ctypes.byref(h)))
        self._h = h

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.load().lbk3_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if self._h is None:
            raise RuntimeError("lattice is closed")
        return self._h

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def step(self, n: int = 1) -> "Lattice3":
        check(_lib.load().lbk3_step(self._handle(), int(n)))
        return self

    @property
    def time(self) -> int:
        t = ctypes.c_int64()
        check(_lib.load().lbk3_time(self._handle(), ctypes.byref(t)))
        return int(t.value)

    @property
    def scale_exponent(self) -> int:
        """FP16: e of the storage scale 2^e (0 for FP32 and BF16)."""
        e = ctypes.c_int32()
        check(_lib.load().lbk3_scale_exponent(self._handle(), ctypes.byref(e)))
        return int(e.value)

    def macroscopic(self):
        """(rho, ux, uy, uz) as [nz][ny][nx] float32 device tensors."""
        out = [torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device=self.device)
               for _ in range(4)]
        check(_lib.load().lbk3_read_macroscopic(self._handle(), *[o.data_ptr() for o in out]))
        return tuple(out)

    def populations(self) -> torch.Tensor:
        f = torch.empty((19, self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        check(_lib.load().lbk3_read_populations(self._handle(), f.data_ptr()))
        return f

    def apparent_permeability(self) -> float:
        v = ctypes.c_double()
        check(_lib.load().lbk3_apparent_permeability(self._handle(), ctypes.byref(v)))
        return float(v.value)

    def diagnostics(self):
        """(mass, x mass flux) in FP64."""
        m, q = ctypes.c_double(), ctypes.c_double()
        check(_lib.load().lbk3_diagnostics(self._handle(), ctypes.byref(m), ctypes.byref(q)))
        return float(m.value), float(q.value)
