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
* ``trimodal``  -- pores, impermeable and permeable solids (Sec. IV.B, Fig. 4)
                   from overlapping tolerance circles and QSGS growth.
* ``fractured_matrix`` -- nonorganic matrix with organic matter and a
                   tree-like fracture system (Sec. IV.C, Fig. 8).

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


# ------------------------------------------------------------------ geometry
#
# Stand-ins for the generators the paper names without specifying them: the
# overlapping tolerance circle method (impermeable solids, Sec. IV.B), the
# quartet structure generation set (permeable solids, Sec. IV.B) and the
# tree-like fracture generator (Sec. IV.C).  Each returns a boolean mask.


def tolerance_circles(shape, frac, r_range, tol, rng, periodic_y=True,
                      max_tries=200000, centres: Optional[list] = None) -> np.ndarray:
    """Overlapping tolerance circles: centres uniform, radii uniform in
    ``r_range``; a candidate is kept when its centre is at least
    (1 - tol)(r_i + r_j) from every kept centre (tol = 0: no overlap, 1: any
    overlap); circles are added until they cover ``frac`` of the domain.
    Wrapped in y when ``periodic_y``; the kept (x, y, r) are appended to
    ``centres`` when given."""
    ny, nx = shape
    mask = np.zeros(shape, dtype=bool)
    cs = np.zeros((0, 3))
    target = frac * nx * ny
    xs = np.arange(nx) + 0.5
    tries = 0
    while mask.sum() < target and tries < max_tries:
        tries += 1
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        r = rng.uniform(r_range[0], r_range[1])
        if len(cs):
            dy = np.abs(cs[:, 1] - cy)
            if periodic_y:
                dy = np.minimum(dy, ny - dy)
            d = np.hypot(cs[:, 0] - cx, dy)
            if np.any(d < (1.0 - tol) * (cs[:, 2] + r)):
                continue
        cs = np.vstack([cs, [cx, cy, r]])
        x0, x1 = max(int(cx - r) - 1, 0), min(int(cx + r) + 2, nx)
        for yy in range(int(math.floor(cy - r)) - 1, int(math.ceil(cy + r)) + 2):
            if not periodic_y and not 0 <= yy < ny:
                continue
            dyy = (yy + 0.5) - cy
            if abs(dyy) > r:
                continue
            dx = xs[x0:x1] - cx
            mask[yy % ny, x0:x1] |= dx * dx + dyy * dyy <= r * r
    if centres is not None:
        centres.extend(map(tuple, cs))
    return mask


_QSGS_DIRS = [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def qsgs(shape, frac, rng, core=0.005, grow_axis=0.02, grow_diag=0.005,
         allowed=None) -> np.ndarray:
    """Quartet structure generation set: cells become growth cores with
    probability ``core``; every grown cell then grows into each of its eight
    neighbours with probability ``grow_axis`` (axis directions) or
    ``grow_diag`` (diagonals), periodically, until exactly ``frac`` of all
    cells are grown (the last growth step is thinned at random).  Only cells
    in ``allowed`` (default: all) can grow."""
    ny, nx = shape
    allowed = np.ones(shape, dtype=bool) if allowed is None else np.asarray(allowed, bool)
    target = int(round(frac * nx * ny))
    if target > allowed.sum():
        raise ValueError("target fraction exceeds the allowed cells")
    grown = np.zeros(shape, dtype=bool)

    def add(cand):
        idx = np.flatnonzero(cand & allowed & ~grown)
        need = target - int(grown.sum())
        if len(idx) > need:
            idx = rng.choice(idx, need, replace=False)
        grown.flat[idx] = True

    add(rng.random(shape) < core)
    while grown.sum() < target:
        new = np.zeros(shape, dtype=bool)
        for i, (ex, ey) in enumerate(_QSGS_DIRS):
            p = grow_axis if i < 4 else grow_diag
            new |= np.roll(grown, (ey, ex), axis=(0, 1)) & (rng.random(shape) < p)
        if not (new & allowed & ~grown).any():
            new = rng.random(shape) < core  # growth stalled: seed new cores
        add(new)
    return grown


def _segment(mask, x0, y0, x1, y1, width):
    """Mark the cells within width/2 of the segment (x0, y0)-(x1, y1)."""
    ny, nx = mask.shape
    h = 0.5 * width
    xa, xb = int(max(math.floor(min(x0, x1) - h), 0)), int(min(math.ceil(max(x0, x1) + h) + 1, nx))
    ya, yb = int(max(math.floor(min(y0, y1) - h), 0)), int(min(math.ceil(max(y0, y1) + h) + 1, ny))
    if xa >= xb or ya >= yb:
        return
    X, Y = np.meshgrid(np.arange(xa, xb) + 0.5, np.arange(ya, yb) + 0.5)
    dx, dy = x1 - x0, y1 - y0
    L2 = dx * dx + dy * dy
    t = np.clip(((X - x0) * dx + (Y - y0) * dy) / L2, 0.0, 1.0) if L2 > 0 else 0.0
    d2 = (X - (x0 + t * dx)) ** 2 + (Y - (y0 + t * dy)) ** 2
    mask[ya:yb, xa:xb] |= d2 <= h * h


def tree_fractures(shape, rng, aperture=10.0, n_first=10, n_second=3,
                   angle=(20.0, 60.0)) -> np.ndarray:
    """Tree-like fracture system: a trunk of width ``aperture`` crossing the
    domain along x through its middle (wandering gently), ``n_first`` first
    branches leaving it at angles in ``angle`` (degrees) with 0.6 times the
    width, and ``n_second`` second branches on each first branch with 0.4
    times the width."""
    ny, nx = shape
    mask = np.zeros(shape, dtype=bool)
    nseg = 8
    xs = np.linspace(0.0, nx, nseg + 1)
    ys = ny / 2 + np.cumsum(rng.normal(0.0, 0.02 * ny, nseg + 1))
    ys = np.clip(ys, 0.25 * ny, 0.75 * ny)
    for j in range(nseg):
        _segment(mask, xs[j], ys[j], xs[j + 1], ys[j + 1], aperture)
    for _ in range(n_first):
        j = int(rng.integers(0, nseg))
        s = rng.uniform(0.0, 1.0)
        bx, by = xs[j] + s * (xs[j + 1] - xs[j]), ys[j] + s * (ys[j + 1] - ys[j])
        a = math.radians(rng.uniform(*angle)) * (1 if rng.random() < 0.5 else -1)
        a += 0.0 if rng.random() < 0.5 else math.pi
        L = rng.uniform(0.3, 0.5) * ny / max(abs(math.sin(a)), 0.3)
        ex, ey = bx + L * math.cos(a), by + L * math.sin(a)
        _segment(mask, bx, by, ex, ey, 0.6 * aperture)
        for _ in range(n_second):
            s2 = rng.uniform(0.3, 0.9)
            cx, cy = bx + s2 * (ex - bx), by + s2 * (ey - by)
            a2 = a + math.radians(rng.uniform(*angle)) * (1 if rng.random() < 0.5 else -1)
            L2 = 0.5 * L * rng.uniform(0.5, 1.0)
            _segment(mask, cx, cy, cx + L2 * math.cos(a2), cy + L2 * math.sin(a2), 0.4 * aperture)
    return mask


def trimodal(nx=410, ny=200, seed=5, imp_frac=0.4, perm_frac=0.3, r_range=(6.0, 20.0),
             tol=0.2, eps_ps=0.5, k_ps=0.05, kn_ps=0.5, rho_in=1.01, rho_out=1.0,
             tau=0.8, **params) -> Case:
    """Three-component medium of Sec. IV.B (Fig. 4): impermeable solid
    (eps = 0) from overlapping tolerance circles covering ``imp_frac``,
    permeable solid (eps_ps, k_ps, kn_ps in lattice units) grown by QSGS in
    the remaining space to ``perm_frac``, and pores (eps = 1, k = +inf)
    elsewhere; pressure-driven in x, periodic in y."""
    rng = np.random.default_rng(seed)
    imp = tolerance_circles((ny, nx), imp_frac, r_range, tol, rng)
    perm = qsgs((ny, nx), perm_frac, rng, allowed=~imp)
    eps = np.where(imp, 0.0, np.where(perm, eps_ps, 1.0))
    k = np.where(perm, k_ps, np.where(imp, 1.0, np.inf))
    kn0 = np.where(perm, kn_ps, 0.0)
    p = run_params(tau=tau, bc_x=PRESSURE, bc_y=PERIODIC, rho_in=rho_in, rho_out=rho_out,
                   init=1, **params)
    return Case(_f32(eps), _f32(k), _f32(kn0), p, f"trimodal{nx}x{ny}s{seed}")


def fractured_matrix(nx=1164, ny=536, seed=6, organic_frac=0.106, aperture=10.0,
                     eps_in=0.05, k_in=1e-4, kn_in=2.0, eps_org=0.2, k_org=1e-3,
                     kn_org=1.0, eps_frac=1.0, k_frac=np.inf, rho_in=1.01, rho_out=1.0,
                     tau=0.8, **params) -> Case:
    """Fractured shale matrix of Sec. IV.C (Fig. 8): a permeable nonorganic
    matrix (eps_in, k_in, kn_in) holding QSGS-grown organic matter
    (``organic_frac``; eps_org, k_org, kn_org) and a tree-like fracture
    system of width ``aperture`` nodes (free fluid by default); pressure
    driven in x, periodic in y."""
    rng = np.random.default_rng(seed)
    org = qsgs((ny, nx), organic_frac, rng)
    frac = tree_fractures((ny, nx), rng, aperture=aperture)
    eps = np.where(frac, eps_frac, np.where(org, eps_org, eps_in))
    k = np.where(frac, k_frac, np.where(org, k_org, k_in))
    kn0 = np.where(frac, 0.0 if np.isinf(k_frac) else kn_in, np.where(org, kn_org, kn_in))
    p = run_params(tau=tau, bc_x=PRESSURE, bc_y=PERIODIC, rho_in=rho_in, rho_out=rho_out,
                   init=1, **params)
    return Case(_f32(eps), _f32(k), _f32(kn0), p, f"fractured{nx}x{ny}s{seed}")


# ------------------------------------------------------------ three dims


def run_params3(tau=0.8, gx=0.0, gy=0.0, gz=0.0, f_eps=0.0, bc_x=PERIODIC, bc_y=PERIODIC,
                bc_z=PERIODIC, rho_in=1.0, rho_out=1.0, rho0=1.0, rho_ref=1.0, kn_local=1,
                init=0, correlation=0, slip_b=-1.0) -> Dict[str, float]:
    """Run description of a D3Q19 lattice shared by the oracle and the HIP
    path (lattice units)."""
    return dict(tau=float(tau), gx=float(gx), gy=float(gy), gz=float(gz), f_eps=float(f_eps),
                bc_x=int(bc_x), bc_y=int(bc_y), bc_z=int(bc_z), rho_in=float(rho_in),
                rho_out=float(rho_out), rho0=float(rho0), rho_ref=float(rho_ref),
                kn_local=int(kn_local), init=int(init), correlation=int(correlation),
                slip_b=float(slip_b))


def random_medium3(nx, ny, nz, seed, eps_range=(0.2, 0.9), k_range=(1e-2, 1.0),
                   kn_range=(0.0, 1.0), solid_frac=0.0, pore_frac=0.0, **params) -> Case:
    """Small i.i.d. heterogeneous 3-D medium ([nz][ny][nx]) with optional
    impermeable (eps = 0) and free-fluid (eps = 1, k = inf) nodes."""
    rng = np.random.default_rng(seed)
    s = (nz, ny, nx)
    eps = rng.uniform(eps_range[0], eps_range[1], s)
    k = np.exp(rng.uniform(math.log(k_range[0]), math.log(k_range[1]), s))
    kn0 = rng.uniform(kn_range[0], kn_range[1], s)
    u = rng.uniform(0, 1, s)
    solid = u < solid_frac
    pore = (u >= solid_frac) & (u < solid_frac + pore_frac)
    eps = np.where(solid, 0.0, np.where(pore, 1.0, eps))
    k = np.where(pore, np.inf, k)
    kn0 = np.where(pore | solid, 0.0, kn0)
    return Case(_f32(eps), _f32(k), _f32(kn0), run_params3(**params),
                f"random3_{nx}x{ny}x{nz}s{seed}")


def channel3(nx, ny, nz, eps=0.5, k=1.024, kn0=0.0, gx=1e-6, tau=0.8) -> Case:
    """Porous-filled plates normal to y (walls), periodic in x and z,
    driven by a body force along x (Sec. IV.A in three dimensions)."""
    s = (nz, ny, nx)
    return Case(_f32(np.full(s, eps)), _f32(np.full(s, k)), _f32(np.full(s, kn0)),
                run_params3(tau=tau, gx=gx, bc_y=WALL), f"channel3_{nx}x{ny}x{nz}")


def spheres(n=256, seed=7, n_spheres=96, r_min=8.0, r_max=40.0, eps_inc=0.2, k_inc=1e-4,
            eps_matrix=0.5, k_matrix=1e-2, kn_base=0.05, rho_in=1.01, rho_out=1.0,
            tau=0.8) -> Case:
    """Two-component 3-D medium, the disc medium of Sec. IV.B in three
    dimensions: overlapping spherical inclusions (radius uniform in [r_min,
    r_max] scaled by n/256, centres uniform, wrapped in y and z) of a
    low-permeability solid in a permeable matrix; Kn by the pore-radius
    scaling of Eq. 11; pressure-driven in x, periodic in y and z."""
    rng = np.random.default_rng(seed)
    scale = n / 256.0
    inside = np.zeros((n, n, n), dtype=bool)
    g = np.arange(n) + 0.5
    for _ in range(n_spheres):
        c = rng.uniform(0, n, 3)
        r = rng.uniform(r_min, r_max) * scale
        dz = np.minimum(np.abs(g - c[2]), n - np.abs(g - c[2]))
        dy = np.minimum(np.abs(g - c[1]), n - np.abs(g - c[1]))
        dx = np.abs(g - c[0])
        inside |= (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2) <= r * r
    eps = np.where(inside, eps_inc, eps_matrix)
    k = np.where(inside, k_inc, k_matrix)
    eps32, k32 = _f32(eps), _f32(k)
    kn0 = kn_from_pore_scaling(k32, eps32, kn_base, k_matrix, eps_matrix)
    return Case(eps32, k32, _f32(kn0),
                run_params3(tau=tau, bc_x=PRESSURE, rho_in=rho_in, rho_out=rho_out, init=1),
                f"spheres{n}")
