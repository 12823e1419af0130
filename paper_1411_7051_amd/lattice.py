"""Python face of the C ABI: ``Lattice`` wraps one ``lbk_lattice`` handle.

PyTorch supplies the device workspace and the stream (torch's current
stream of the lattice's device); all of the method runs in ``liblbk.so``.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import Desc, check

PERIODIC, WALL, PRESSURE = 0, 1, 2


def make_desc(nx, ny, tau=0.8, gx=0.0, gy=0.0, f_eps=0.0, bc_x=PERIODIC,
              bc_y=PERIODIC, rho_in=1.0, rho_out=1.0, rho0=1.0, rho_ref=1.0,
              kn_local=1, init=0, storage="f32", check_every=100, correlation=0,
              slip_b=-1.0, pass_mode=0, band=0) -> Desc:
    lib = _lib.load()
    d = Desc()
    check(lib.lbk_desc_default(ctypes.byref(d)))
    d.nx, d.ny = int(nx), int(ny)
    d.tau, d.gx, d.gy, d.f_eps = float(tau), float(gx), float(gy), float(f_eps)
    d.bc_x, d.bc_y = int(bc_x), int(bc_y)
    d.rho_in, d.rho_out, d.rho0 = float(rho_in), float(rho_out), float(rho0)
    d.rho_ref, d.kn_local, d.init = float(rho_ref), int(kn_local), int(init)
    d.storage = _lib.STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.check_every = int(check_every)
    d.correlation = (_lib.CORRELATION[correlation] if isinstance(correlation, str)
                     else int(correlation))
    d.slip_b = float(slip_b)
    d.pass_mode = (_lib.PASS_MODE[pass_mode] if isinstance(pass_mode, str)
                   else int(pass_mode))
    d.band = int(band)
    return d


def workspace_bytes(desc: Desc) -> int:
    n = ctypes.c_size_t()
    check(_lib.load().lbk_workspace_size(ctypes.byref(desc), ctypes.byref(n)))
    return int(n.value)


def _field(a, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a.detach().to(device=device, dtype=torch.float32)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return t.contiguous()


class Lattice:
    """A D2Q9 Klinkenberg lattice on one GPU.

    ``eps``, ``k``, ``kn0``: [ny][nx] arrays (numpy or torch); ``k`` may be
    +inf.  Keyword parameters are those of ``lbk_desc`` (tau, gx, gy, f_eps,
    bc_x, bc_y, rho_in, rho_out, rho0, rho_ref, kn_local, init, storage,
    check_every, correlation, slip_b, pass_mode, band)."""

    def __init__(self, eps, k, kn0=None, device: Optional[torch.device] = None,
                 **params):
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        lib = _lib.load()
        e = _field(eps, self.device)
        kk = _field(k, self.device)
        if e.dim() != 2 or e.shape != kk.shape:
            raise ValueError("eps and k must be 2-D of one shape")
        self.ny, self.nx = e.shape
        kn = None if kn0 is None else _field(kn0, self.device)
        if kn is not None and kn.shape != e.shape:
            raise ValueError("kn0 must match eps")
        self.params = dict(params)
        self.desc = make_desc(self.nx, self.ny, **params)
        nbytes = workspace_bytes(self.desc)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.lbk_create(ctypes.byref(self.desc), e.data_ptr(), kk.data_ptr(),
                                 None if kn is None else kn.data_ptr(),
                                 self._ws.data_ptr(), nbytes, self.stream.cuda_stream,
                                 ctypes.byref(h)))
        self._h = h

    # -- lifetime
    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.load().lbk_destroy(h)
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

    # -- stepping
    def step(self, n: int = 1) -> "Lattice":
        check(_lib.load().lbk_step(self._handle(), int(n)))
        return self

    @property
    def time(self) -> int:
        t = ctypes.c_int64()
        check(_lib.load().lbk_time(self._handle(), ctypes.byref(t)))
        return int(t.value)

    @property
    def steps_per_launch(self) -> int:
        """1 (single sweeps), 2 or 3 (two- or three-step passes), as
        pass_mode and the lattice's size and storage decide."""
        n = ctypes.c_int32()
        check(_lib.load().lbk_steps_per_launch(self._handle(), ctypes.byref(n)))
        return int(n.value)

    # -- read-out
    def macroscopic(self):
        """(rho, ux, uy) as [ny][nx] float32 device tensors."""
        out = [torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
               for _ in range(3)]
        check(_lib.load().lbk_read_macroscopic(self._handle(), *[o.data_ptr() for o in out]))
        return tuple(out)

    def populations(self) -> torch.Tensor:
        """Post-collision populations f*_i as a [9][ny][nx] float64 tensor."""
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        check(_lib.load().lbk_read_populations(self._handle(), f.data_ptr()))
        return f

    def apparent_permeability(self) -> float:
        v = ctypes.c_double()
        check(_lib.load().lbk_apparent_permeability(self._handle(), ctypes.byref(v)))
        return float(v.value)

    def diagnostics(self):
        """(mass, x mass flux, residual vs the previous call)."""
        m, q, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(_lib.load().lbk_diagnostics(self._handle(), ctypes.byref(m), ctypes.byref(q),
                                          ctypes.byref(r)))
        return float(m.value), float(q.value), float(r.value)

    # -- checkpoint / resume
    def state_bytes(self) -> int:
        n = ctypes.c_size_t()
        check(_lib.load().lbk_state_size(self._handle(), ctypes.byref(n)))
        return int(n.value)

    def save_state(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        check(_lib.load().lbk_save_state(self._handle(), out.data_ptr()))
        return out

    def load_state(self, src: torch.Tensor) -> None:
        if src.numel() * src.element_size() < self.state_bytes():
            raise ValueError("state buffer too small")
        check(_lib.load().lbk_load_state(self._handle(), src.contiguous().data_ptr()))

    # -- gradients
    def adjoint_workspace_bytes(self, steps: int, ckpt_every: int, hist_len: int) -> int:
        n = ctypes.c_size_t()
        check(_lib.load().lbk_adjoint_workspace_size(self._handle(), int(steps),
                                                     int(ckpt_every), int(hist_len),
                                                     ctypes.byref(n)))
        return int(n.value)

    def adjoint_plan(self, steps: int, ckpt_every: int, budget: Optional[int] = None,
                     fraction: float = 0.9, with_bytes: bool = False):
        """History length of the checkpoint plan that recomputes least within
        ``budget`` bytes (default: ``fraction`` of the device's free memory);
        with ``with_bytes`` also the workspace bytes that plan uses (more than
        the minimum when inner checkpoints of more segments fit)."""
        if budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget = int(free * fraction)
        h, n = ctypes.c_int64(), ctypes.c_size_t()
        check(_lib.load().lbk_adjoint_plan(self._handle(), int(steps), int(ckpt_every),
                                           int(budget), ctypes.byref(h), ctypes.byref(n)))
        return (int(h.value), int(n.value)) if with_bytes else int(h.value)

    def adjoint_forward(self, steps: int, objective: str = "k_app", ckpt_every: int = 500,
                        hist_len=None, workspace: Optional[torch.Tensor] = None):
        """Run ``steps`` steps keeping checkpoints; returns (J, workspace).
        ``hist_len``: steps of history recorded at a time (None: ckpt_every,
        the one-level scheme; "auto": the longest that fits in memory)."""
        ckpt_every = max(1, min(int(ckpt_every), int(steps)))
        planned = 0
        if hist_len == "auto":
            hist_len, planned = self.adjoint_plan(steps, ckpt_every, with_bytes=True)
        hist_len = ckpt_every if hist_len is None else max(1, min(int(hist_len), ckpt_every))
        nbytes = max(planned, self.adjoint_workspace_bytes(steps, ckpt_every, hist_len))
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        J = ctypes.c_double()
        check(_lib.load().lbk_adjoint_forward(self._handle(), _lib.OBJECTIVE[objective],
                                              int(steps), ckpt_every, hist_len,
                                              workspace.data_ptr(), workspace.numel(),
                                              ctypes.byref(J)))
        return float(J.value), workspace

    def adjoint_backward(self, workspace: torch.Tensor, wrt_kn0: bool = False):
        """dJ/d ln k of the last adjoint_forward, [ny][nx] float32; with
        ``wrt_kn0`` the pair (dJ/d ln k, dJ/d ln kn0)."""
        g = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        gk = torch.empty_like(g) if wrt_kn0 else None
        check(_lib.load().lbk_adjoint_backward(self._handle(), workspace.data_ptr(),
                                               workspace.numel(), g.data_ptr(),
                                               None if gk is None else gk.data_ptr()))
        return (g, gk) if wrt_kn0 else g

    def gradient(self, steps: int, objective: str = "k_app", ckpt_every: int = 500,
                 hist_len=None, wrt_kn0: bool = False):
        """(J, dJ/d ln k) after ``steps`` steps from the current state; with
        ``wrt_kn0``, (J, dJ/d ln k, dJ/d ln kn0)."""
        J, ws = self.adjoint_forward(steps, objective, ckpt_every, hist_len)
        g = self.adjoint_backward(ws, wrt_kn0)
        return (J, *g) if wrt_kn0 else (J, g)

    def run_to_steady(self, every: int = 100, tol: float = 1e-9, max_steps: int = 10**7,
                      patience: int = 10):
        """Step in blocks of ``every`` until the velocity residual
        ||u - u_prev|| / ||u|| between blocks falls below ``tol``, or stops
        decreasing for ``patience`` blocks (the FP32 floor).  Returns
        (steps, residual, reason)."""
        self.diagnostics()
        best, stall, steps = math.inf, 0, 0
        while steps < max_steps:
            self.step(every)
            steps += every
            _, _, r = self.diagnostics()
            if r < tol:
                return steps, r, "tol"
            if r < best:
                best, stall = r, 0
            else:
                stall += 1
                if stall >= patience:
                    return steps, r, "plateau"
        return steps, r, "max_steps"


class ApparentPermeability(torch.autograd.Function):
    """J(ln k) after ``steps`` steps from rest, as a differentiable function
    of the log-permeability field: forward runs the HIP sweep with
    checkpoints, backward runs the HIP adjoint sweep.

    ``ApparentPermeability.apply(log_k, eps, kn0, steps, params)`` with
    ``params`` a dict of lattice keywords (plus optional ``objective``,
    ``ckpt_every``, ``hist_len``); returns a float64 scalar tensor."""

    @staticmethod
    def forward(ctx, log_k, eps, kn0, steps, params):
        params = dict(params)
        objective = params.pop("objective", "k_app")
        ckpt = params.pop("ckpt_every", 500)
        hist = params.pop("hist_len", None)
        lat = Lattice(eps, torch.exp(log_k.detach().double()).float(), kn0,
                      device=log_k.device, **params)
        J, ws = lat.adjoint_forward(int(steps), objective, ckpt, hist)
        ctx.lat, ctx.ws = lat, ws
        return torch.tensor(J, dtype=torch.float64, device=log_k.device)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.lat.adjoint_backward(ctx.ws)
        ctx.lat.close()
        ctx.lat = ctx.ws = None
        return (grad_out.to(g.dtype) * g, None, None, None, None)
