"""Ensembles: ``Batch`` steps many ``Lattice`` samples of uneven size with one
kernel launch per step (optionally replayed from HIP graphs), wrapping one
``lbk_batch`` handle.  The launch configuration comes from the library's
tuner, remembered in an optional JSON cache keyed by the batch's shape."""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check
from .lattice import Lattice


class Batch:
    """Step ``lattices`` together.  All must share storage, boundary kinds,
    device and stream (torch's current stream when they were created)."""

    def __init__(self, lattices: Sequence[Lattice]):
        if not lattices:
            raise ValueError("a batch needs at least one lattice")
        self.lattices = list(lattices)
        self.device = self.lattices[0].device
        lib = _lib.load()
        n = len(self.lattices)
        self._arr = (ctypes.c_void_p * n)(*[l._handle().value for l in self.lattices])
        nbytes = ctypes.c_size_t()
        check(lib.lbk_batch_workspace_size(self._arr, n, ctypes.byref(nbytes)))
        self._ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.lbk_batch_create(self._arr, n, self._ws.data_ptr(), self._ws.numel(),
                                       ctypes.byref(h)))
        self._h = h

    def __len__(self) -> int:
        return len(self.lattices)

    # -- lifetime
    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.load().lbk_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if self._h is None:
            raise RuntimeError("batch is closed")
        return self._h

    # -- stepping
    def step(self, n: int = 1) -> "Batch":
        check(_lib.load().lbk_batch_step(self._handle(), int(n)))
        return self

    def set_launch(self, tile_x: int = 256, rows: int = 1, grid: int = 0,
                   graph_steps: int = 0) -> None:
        check(_lib.load().lbk_batch_set_launch(self._handle(), int(tile_x), int(rows), int(grid),
                                               int(graph_steps)))

    def set_pass_mode(self, mode: str = "auto") -> None:
        """Steps per launch: "two_step", "single" or "auto" (two-step passes
        for batches of 2^22 nodes and more until ``autotune`` keeps the
        faster); every choice gives the same states bit for bit."""
        check(_lib.load().lbk_batch_set_pass_mode(self._handle(), _lib.PASS_MODE[mode]))

    @property
    def steps_per_launch(self) -> int:
        """1 or 2: whether steps currently go through the two-step pass."""
        m, k = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().lbk_batch_get_pass_mode(self._handle(), ctypes.byref(m),
                                                  ctypes.byref(k)))
        return int(k.value)

    def set_graph_readout(self, on: bool = True) -> None:
        """Make every graph replay end with the per-sample read-out sums."""
        check(_lib.load().lbk_batch_set_graph_readout(self._handle(), int(bool(on))))

    @property
    def launch(self):
        """(tile_x, rows, grid, graph_steps)."""
        v = [ctypes.c_int32() for _ in range(4)]
        check(_lib.load().lbk_batch_get_launch(self._handle(), *[ctypes.byref(x) for x in v]))
        return tuple(int(x.value) for x in v)

    def signature(self) -> str:
        """Key of this batch's shape for the tuning cache: device, storage,
        boundary kinds and the sorted sample sizes."""
        l0 = self.lattices[0]
        sizes = sorted((l.nx, l.ny) for l in self.lattices)
        key = json.dumps([torch.cuda.get_device_name(self.device), int(l0.desc.storage),
                          int(l0.desc.bc_x), int(l0.desc.bc_y), sizes])
        return hashlib.sha1(key.encode()).hexdigest()[:16]

    def autotune(self, reps: int = 10, cache: Optional[str] = None) -> float:
        """Pick the fastest (tile_x, rows, grid) for this batch and, in the
        automatic pass mode, whether two-step passes beat it, leaving the
        samples' states untouched; returns the mean step time in
        microseconds (NaN when taken from ``cache``, a JSON file of
        signature -> [tile_x, rows, grid, steps per launch, us])."""
        sig = self.signature()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            entry = table.get(sig)
            if entry is not None and len(entry) == 5:
                tile_x, rows, grid, per_launch, _ = entry
                self.set_launch(tile_x, rows, grid, self.launch[3])
                self.set_pass_mode("two_step" if per_launch == 2 else "single")
                return float("nan")
        us = ctypes.c_double()
        check(_lib.load().lbk_batch_autotune(self._handle(), int(reps), ctypes.byref(us)))
        if cache:
            tile_x, rows, grid, _ = self.launch
            table[sig] = [tile_x, rows, grid, self.steps_per_launch, float(us.value)]
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return float(us.value)

    # -- read-out
    def apparent_permeability(self) -> np.ndarray:
        """Global permeability of every sample (float64 [n])."""
        out = np.empty(len(self), dtype=np.float64)
        check(_lib.load().lbk_batch_apparent_permeability(
            self._handle(), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    # -- gradients
    def adjoint_plan(self, steps: int, ckpt_every: int, budget: Optional[int] = None,
                     fraction: float = 0.9, with_bytes: bool = False):
        """History length of the batched checkpoint plan that recomputes
        least within ``budget`` bytes (default: ``fraction`` of the free
        device memory); with ``with_bytes`` also the workspace bytes it uses
        (more than the minimum when more segments' inner checkpoints fit)."""
        if budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget = int(free * fraction)
        h, nb = ctypes.c_int64(), ctypes.c_size_t()
        check(_lib.load().lbk_batch_adjoint_plan(self._handle(), int(steps), int(ckpt_every),
                                                 int(budget), ctypes.byref(h), ctypes.byref(nb)))
        return (int(h.value), int(nb.value)) if with_bytes else int(h.value)

    def adjoint_workspace_bytes(self, steps: int, ckpt_every: int, hist_len: int) -> int:
        n = ctypes.c_size_t()
        check(_lib.load().lbk_batch_adjoint_workspace_size(self._handle(), int(steps),
                                                           int(ckpt_every), int(hist_len),
                                                           ctypes.byref(n)))
        return int(n.value)

    def gradient(self, steps: int, objective: str = "k_app", ckpt_every: int = 500,
                 hist_len=None, wrt_kn0: bool = False, workspace_bytes: int = 0):
        """Per-sample J (float64 [n]) and dJ/d ln k planes (list of [ny][nx]
        float32 tensors) after ``steps`` steps of every sample; with
        ``wrt_kn0`` also the dJ/d ln kn0 planes.  ``hist_len``: None (one
        level), an int, or "auto" (the plan that recomputes least within the
        free memory).  ``workspace_bytes`` beyond the minimum keeps inner
        checkpoints of more segments."""
        lib = _lib.load()
        ckpt_every = max(1, min(int(ckpt_every), int(steps)))
        if hist_len == "auto":
            hist_len, planned = self.adjoint_plan(steps, ckpt_every, with_bytes=True)
            workspace_bytes = max(int(workspace_bytes), planned)
        hist_len = ckpt_every if hist_len is None else max(1, min(int(hist_len), ckpt_every))
        ws = torch.empty(max(int(workspace_bytes),
                             self.adjoint_workspace_bytes(steps, ckpt_every, hist_len)),
                         dtype=torch.uint8, device=self.device)
        n = len(self)
        J = np.empty(n, dtype=np.float64)
        check(lib.lbk_batch_adjoint_forward(self._handle(), _lib.OBJECTIVE[objective],
                                            int(steps), ckpt_every, hist_len, ws.data_ptr(),
                                            ws.numel(), J.ctypes.data_as(ctypes.c_void_p)))
        g = [torch.empty((l.ny, l.nx), dtype=torch.float32, device=self.device)
             for l in self.lattices]
        gp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in g])
        gk, gkp = None, None
        if wrt_kn0:
            gk = [torch.empty_like(t) for t in g]
            gkp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in gk])
        check(lib.lbk_batch_adjoint_backward(self._handle(), ws.data_ptr(), ws.numel(), gp,
                                             gkp))
        return (J, g, gk) if wrt_kn0 else (J, g)

    def check(self) -> None:
        """NaN/Inf check of every sample (and FP16 scale re-centring)."""
        check(_lib.load().lbk_batch_check(self._handle()))


def ensemble_lattices(cases, device=None, **overrides):
    """One ``Lattice`` per input case (``inputs.Case``), created on the
    current stream; keyword overrides apply to every case's parameters."""
    out = []
    for c in cases:
        params = dict(c.params, **overrides)
        out.append(Lattice(c.eps, c.k, c.kn0, device=device, **params))
    return out
