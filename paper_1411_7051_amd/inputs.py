"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds none of the lattice Boltzmann arithmetic.  It only draws
per-node medium fields (porosity ``eps``, intrinsic permeability ``k`` in
lattice units, reference Knudsen number ``kn0``) and the run description, so
that the HIP path and the FP64 oracle can be fed identical inputs.  Every
field is returned as float32 (``k`` may hold +inf for a node with no Darcy
drag); the oracle widens the same values to float64 exactly.

Workloads (Sec. IV of the paper; none of its images or generators are
available, so these are statistical stand-ins with the stated shapes):

* ``channel``   -- parallel plates filled with a uniform porous medium
                   (Sec. IV.A), body-force or pressure driven.
* ``discs``     -- two-component medium: overlapping circular inclusions of a
                   low-permeability solid in a permeable matrix (Sec. IV.B).
* ``shale``     -- log-normal permeability matrix with straight fractures
                   (Sec. IV.C).
* ``ensemble``  -- independent heterogeneous samples of uneven size.

Kn fields follow the pore-radius scaling of Eq. 11 (r ~ sqrt(k/eps)): a node
with permeability k and porosity eps gets
``kn0 = kn_base * sqrt((k_ref/eps_ref) / (k/eps))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

PERIODIC, WALL, PRESSURE = 0, 1, 2


@dataclasses.dataclass
class Case:
    """One lattice: medium fields ([ny][nx], float32) and run parameters."""

    eps: np.ndarray
    k: np.ndarray
    kn0: np.ndarray
    params: Dict[str, float]
    name: str = ""

    @property
    def shape(self):
        return self.eps.shape

    @property
    def nodes(self) -> int:
        return int(self.eps.size)


def run_params(tau=0.8, gx=0.0, gy=0.0, f_eps=0.0, bc_x=PERIODIC, bc_y=PERIODIC,
               rho_in=1.0, rho_out=1.0, rho0=1.0, rho_ref=1.0, kn_local=1,
               init=0, correlation=0, slip_b=-1.0) -> Dict[str, float]:
    """Run description shared by the oracle and the HIP path (lattice units).
    correlation: 0 second order (Eqs. 6-7, slip coefficient slip_b), 1 first
    order (Eqs. 4-5), 2 none."""
    return dict(tau=float(tau), gx=float(gx), gy=float(gy), f_eps=float(f_eps),
                bc_x=int(bc_x), bc_y=int(bc_y), rho_in=float(rho_in),
                rho_out=float(rho_out), rho0=float(rho0),
                rho_ref=float(rho_ref), kn_local=int(kn_local), init=int(init),
                correlation=int(correlation), slip_b=float(slip_b))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def kn_from_pore_scaling(k, eps, kn_base, k_ref, eps_ref) -> np.ndarray:
    """kn0 = kn_base * sqrt((k_ref/eps_ref)/(k/eps)) (pore radius ~ sqrt(k/eps),
    Eq. 11); zero where eps = 0 or k is infinite."""
    k = np.asarray(k, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    out = np.zeros_like(k)
    ok = (eps > 0) & np.isfinite(k)
    out[ok] = kn_base * np.sqrt((k_ref / eps_ref) / (k[ok] / eps[ok]))
    return out


def channel(nx=64, ny=32, eps=0.5, k=1.024, kn0=0.0, drive="force", gx=1e-6,
            rho_in=1.01, rho_out=1.0, tau=0.8, name="channel") -> Case:
    """Porous-filled parallel plates (Sec. IV.A): walls above and below.
    ``drive='force'``: periodic in x with body force gx.
    ``drive='pressure'``: density rho_in / rho_out on the end columns,
    starting from a linear density ramp."""
    shape = (ny, nx)
    if drive == "force":
        params = run_params(tau=tau, gx=gx, bc_x=PERIODIC, bc_y=WALL)
    elif drive == "pressure":
        params = run_params(tau=tau, bc_x=PRESSURE, bc_y=WALL, rho_in=rho_in,
                            rho_out=rho_out, init=1)
    else:
        raise ValueError(drive)
    return Case(_f32(np.full(shape, eps)), _f32(np.full(shape, k)),
                _f32(np.full(shape, kn0)), params, name)


def discs(n=4096, seed=2, n_discs=64, r_min=40.0, r_max=200.0, eps_disc=0.2,
          k_disc=1e-4, eps_matrix=0.5, k_matrix=1e-2, kn_base=0.05,
          rho_in=1.01, rho_out=1.0, tau=0.8, nx=None, ny=None,
          name="discs") -> Case:
    """Two-component medium (Sec. IV.B stand-in): ``n_discs`` overlapping
    discs, radii uniform in [r_min, r_max] scaled by n/4096, centres uniform,
    wrapped periodically in y.  Pressure-driven in x, periodic in y."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    scale = min(nx, ny) / 4096.0
    cx = rng.uniform(0, nx, n_discs)
    cy = rng.uniform(0, ny, n_discs)
    rad = rng.uniform(r_min, r_max, n_discs) * scale
    inside = np.zeros((ny, nx), dtype=bool)
    xs = np.arange(nx) + 0.5
    for j in range(n_discs):
        r = rad[j]
        y0 = int(math.floor(cy[j] - r)) - 1
        y1 = int(math.ceil(cy[j] + r)) + 1
        x0 = max(int(math.floor(cx[j] - r)) - 1, 0)
        x1 = min(int(math.ceil(cx[j] + r)) + 1, nx)
        for yy in range(y0, y1 + 1):
            dy = (yy + 0.5) - cy[j]
            if abs(dy) > r:
                continue
            row = yy % ny
            dx = xs[x0:x1] - cx[j]
            inside[row, x0:x1] |= dx * dx + dy * dy <= r * r
    eps = np.where(inside, eps_disc, eps_matrix)
    k = np.where(inside, k_disc, k_matrix)
    eps32, k32 = _f32(eps), _f32(k)
    kn0 = kn_from_pore_scaling(k32, eps32, kn_base, k_matrix, eps_matrix)
    params = run_params(tau=tau, bc_x=PRESSURE, bc_y=PERIODIC, rho_in=rho_in,
                        rho_out=rho_out, init=1)
    return Case(eps32, k32, _f32(kn0), params, name)


def gaussian_field(ny, nx, corr_len, rng) -> np.ndarray:
    """Zero-mean, unit-variance stationary Gaussian field on a periodic grid
    with covariance exp(-r^2 / (2 corr_len^2)): white noise filtered in
    Fourier space by the square root of that covariance's spectrum."""
    white = rng.standard_normal((ny, nx)).astype(np.float32)
    ky = np.fft.fftfreq(ny).astype(np.float32)[:, None]
    kx = np.fft.rfftfreq(nx).astype(np.float32)[None, :]
    filt = np.exp(-((2 * np.pi * corr_len) ** 2) * (kx * kx + ky * ky) / 4.0)
    g = np.fft.irfft2(np.fft.rfft2(white) * filt, s=(ny, nx))
    g = g - g.mean()
    sd = g.std()
    return (g / sd if sd > 0 else g).astype(np.float64)


def _draw_fractures(shape, n_frac, rng, width_choices=(2, 3, 4),
                    len_frac=(1 / 8, 1 / 2)) -> np.ndarray:
    """Straight fractures: centre uniform, angle uniform in [0, pi), width
    drawn from ``width_choices`` nodes, length uniform in ``len_frac`` times
    the domain size; wrapped periodically in y, clipped in x."""
    ny, nx = shape
    mask = np.zeros(shape, dtype=bool)
    L = min(nx, ny)
    for _ in range(n_frac):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        ang = rng.uniform(0, math.pi)
        width = int(rng.choice(width_choices))
        length = rng.uniform(len_frac[0], len_frac[1]) * L
        dx, dy = math.cos(ang), math.sin(ang)
        ts = np.arange(-length / 2, length / 2, 0.5)
        offs = np.arange(width) - (width - 1) / 2.0
        px = cx + ts[:, None] * dx - offs[None, :] * dy
        py = cy + ts[:, None] * dy + offs[None, :] * dx
        ix = np.floor(px).astype(np.int64).ravel()
        iy = np.floor(py).astype(np.int64).ravel() % ny
        ok = (ix >= 0) & (ix < nx)
        mask[iy[ok], ix[ok]] = True
    return mask


def shale(n=8192, seed=3, corr_len=32.0, sigma=1.5, k_mean=1e-5,
          eps_range=(0.05, 0.15), n_frac=24, eps_frac=0.9, k_frac=0.1,
          kn_base=0.5, rho_in=1.01, rho_out=1.0, tau=0.8, nx=None, ny=None,
          name="shale") -> Case:
    """Fractured shale matrix (Sec. IV.C stand-in): ln k Gaussian with
    correlation length ``corr_len`` and standard deviation ``sigma``,
    arithmetic mean ``k_mean``; eps i.i.d. uniform in ``eps_range``;
    ``n_frac`` straight fractures with eps_frac / k_frac.  Pressure-driven in
    x, periodic in y.  Kn reference: (k_mean, mean eps) with kn_base."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    g = gaussian_field(ny, nx, corr_len, rng)
    mu = math.log(k_mean) - 0.5 * sigma * sigma
    k = np.exp(mu + sigma * g)
    eps = rng.uniform(eps_range[0], eps_range[1], (ny, nx))
    frac = _draw_fractures((ny, nx), n_frac, rng)
    eps = np.where(frac, eps_frac, eps)
    k = np.where(frac, k_frac, k)
    eps32, k32 = _f32(eps), _f32(k)
    kn0 = kn_from_pore_scaling(k32, eps32, kn_base, k_mean,
                               0.5 * (eps_range[0] + eps_range[1]))
    params = run_params(tau=tau, bc_x=PRESSURE, bc_y=PERIODIC, rho_in=rho_in,
                        rho_out=rho_out, init=1)
    return Case(eps32, k32, _f32(kn0), params, name)


def ensemble(n_samples=192, seed=4, side=(256, 1536), sigma=1.0,
             corr=(8.0, 64.0), k_median=1e-3, eps_range=(0.1, 0.6),
             kn_range=(0.01, 2.0), rho_in=1.01, rho_out=1.0, tau=0.8,
             sides: Optional[List[int]] = None) -> List[Case]:
    """Independent heterogeneous samples of uneven size: square side uniform
    on the integers in ``side`` (or given by ``sides``), ln k Gaussian with
    standard deviation ``sigma`` and correlation length uniform in ``corr``,
    median ``k_median``; eps i.i.d. uniform in ``eps_range``; base Kn uniform
    in ``kn_range`` with the sample's (geometric-mean k, mean eps) as the
    reference pore.  Sample i is seeded with seed + i."""
    out = []
    top = np.random.default_rng(seed)
    if sides is None:
        sides = [int(s) for s in top.integers(side[0], side[1] + 1, n_samples)]
    for i, s in enumerate(sides):
        rng = np.random.default_rng(seed + i)
        ell = rng.uniform(corr[0], corr[1])
        g = gaussian_field(s, s, ell, rng)
        k = np.exp(math.log(k_median) + sigma * g)
        eps = rng.uniform(eps_range[0], eps_range[1], (s, s))
        kn_base = rng.uniform(kn_range[0], kn_range[1])
        eps32, k32 = _f32(eps), _f32(k)
        kref = float(np.exp(np.mean(np.log(k32.astype(np.float64)))))
        eref = float(np.mean(eps32.astype(np.float64)))
        kn0 = kn_from_pore_scaling(k32, eps32, kn_base, kref, eref)
        params = run_params(tau=tau, bc_x=PRESSURE, bc_y=PERIODIC,
                            rho_in=rho_in, rho_out=rho_out, init=1)
        out.append(Case(eps32, k32, _f32(kn0), params, f"sample{i}"))
    return out


def random_medium(nx, ny, seed, eps_range=(0.2, 0.9), k_range=(1e-2, 1.0),
                  kn_range=(0.0, 1.0), solid_frac=0.0, pore_frac=0.0,
                  **params) -> Case:
    """Small i.i.d. heterogeneous medium for parity and invariant tests:
    eps, ln k and kn0 uniform in their ranges, with optional fractions of
    impermeable nodes (eps = 0) and free-fluid nodes (eps = 1, k = inf)."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(eps_range[0], eps_range[1], (ny, nx))
    k = np.exp(rng.uniform(math.log(k_range[0]), math.log(k_range[1]), (ny, nx)))
    kn0 = rng.uniform(kn_range[0], kn_range[1], (ny, nx))
    u = rng.uniform(0, 1, (ny, nx))
    solid = u < solid_frac
    pore = (u >= solid_frac) & (u < solid_frac + pore_frac)
    eps = np.where(solid, 0.0, np.where(pore, 1.0, eps))
    k = np.where(pore, np.inf, k)
    kn0 = np.where(pore | solid, 0.0, kn0)
    return Case(_f32(eps), _f32(k), _f32(kn0), run_params(**params),
                f"random{nx}x{ny}s{seed}")
