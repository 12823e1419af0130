"""Physical-units front end: gas, pressure, temperature and pore structure in
SI units mapped to the lattice inputs of the sweep (Secs. II.B-II.C, IV.A).

- Intrinsic permeability from porosity and grain diameter, Kozeny-Carman for
  packed spheres (Eq. 9): k_d = d^2 eps^3 / (180 (1 - eps)^2).
- Mean free path of the gas (Eq. 10): lambda = (mu / p) sqrt(pi R T / (2 M)).
- Characteristic pore radius (Eq. 11): r = 8.886e-2 sqrt(k_d / eps) with r in
  micrometres and k_d in millidarcy, i.e. the capillary-bundle radius
  sqrt(8 k_d / eps) in SI units.
- Knudsen number Kn = lambda / r (Eq. 5 with c = 1).
- Lattice inputs: k = k_d / dx^2 per node and kn0 = lambda(p_ref) / r per
  node, quoted at the lattice density rho_ref that stands for p_ref (the
  local Kn then follows the density as lambda ~ 1/p, Eq. 10).

The correction factor f_c comes from the library (``lbk_correction_factor``)
so front-end curves use the same correlations as the sweep.  Pure host code:
nothing here runs on the GPU.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import Dict, Iterable, Optional

import numpy as np

from . import _lib

R_GAS = 8.314462618         # J / (mol K)
PSI = 6894.75               # Pa per psi (Sec. IV.A)
MILLIDARCY = 9.869e-16      # m^2 per mD (Sec. II.C)
METHANE_MOLAR_MASS = 16e-3  # kg / mol (Sec. IV.A)


def kozeny_carman(eps, d):
    """Eq. 9: intrinsic permeability (m^2) of packed spheres of diameter d (m)
    at porosity eps (0 < eps < 1), with the Kozeny-Carman constant d^2/180."""
    eps = np.asarray(eps, dtype=np.float64)
    return (d * d / 180.0) * eps ** 3 / (1.0 - eps) ** 2


def mean_free_path(mu, p, T, M=METHANE_MOLAR_MASS):
    """Eq. 10: mean free path (m) for viscosity mu (Pa s), pressure p (Pa),
    temperature T (K) and molar mass M (kg/mol)."""
    return (np.asarray(mu, dtype=np.float64) / np.asarray(p, dtype=np.float64)) * \
        math.sqrt(math.pi * R_GAS * T / (2.0 * M))


def pore_radius(k_d, eps):
    """Eq. 11: characteristic pore radius (m) from the intrinsic
    permeability k_d (m^2) and porosity eps, evaluated in the units the
    equation is printed in (micrometres, millidarcy)."""
    k_md = np.asarray(k_d, dtype=np.float64) / MILLIDARCY
    return 8.886e-2 * np.sqrt(k_md / np.asarray(eps, dtype=np.float64)) * 1e-6


def knudsen(lam, r):
    """Eq. 5 with c = 1: Kn = lambda / r."""
    return np.asarray(lam, dtype=np.float64) / np.asarray(r, dtype=np.float64)


def correction_factor(kn, correlation="bkc", slip_b: float = -1.0):
    """f_c(Kn) of the selected correlation (Eqs. 6-7, 4-5 or none), FP64, from
    the library's host implementation; same shape as ``kn``."""
    kn = np.ascontiguousarray(kn, dtype=np.float64)
    out = np.empty_like(kn)
    corr = _lib.CORRELATION[correlation] if isinstance(correlation, str) else int(correlation)
    _lib.check(_lib.load().lbk_correction_factor(
        corr, float(slip_b), kn.ctypes.data_as(ctypes.c_void_p),
        out.ctypes.data_as(ctypes.c_void_p), kn.size))
    return out


@dataclass
class Gas:
    """Gas state: temperature (K), molar mass (kg/mol) and viscosity (Pa s),
    either one value or a table {pressure in Pa: viscosity}."""

    T: float = 323.0
    M: float = METHANE_MOLAR_MASS
    mu: object = 1.5e-5

    def viscosity(self, p: float) -> float:
        if isinstance(self.mu, dict):
            ps = sorted(self.mu)
            return float(np.interp(p, ps, [self.mu[q] for q in ps]))
        return float(self.mu)

    def mean_free_path(self, p: float) -> float:
        return float(mean_free_path(self.viscosity(p), p, self.T, self.M))


def lattice_fields(eps, k_d, dx: float, gas: Gas, p_ref: float, r=None):
    """Lattice inputs for the sweep from SI fields: porosity eps, intrinsic
    permeability k_d (m^2; +inf marks free fluid), node spacing dx (m), the
    gas and the pressure p_ref (Pa) that the reference density rho_ref
    stands for.  The pore radius defaults to Eq. 11.  Returns (eps, k, kn0)
    as float32 arrays: k = k_d / dx^2, kn0 = lambda(p_ref) / r (0 where the
    node is free fluid or impermeable)."""
    eps = np.asarray(eps, dtype=np.float64)
    k_d = np.asarray(k_d, dtype=np.float64)
    if r is None:
        with np.errstate(divide="ignore", invalid="ignore"):
            r = pore_radius(k_d, eps)
    lam = gas.mean_free_path(p_ref)
    porous = np.isfinite(k_d) & (eps > 0) & (np.asarray(r) > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        kn0 = np.where(porous, lam / np.where(porous, r, 1.0), 0.0)
    k = np.where(np.isfinite(k_d), k_d / (dx * dx), np.inf)
    return eps.astype(np.float32), k.astype(np.float32), kn0.astype(np.float32)


def physical_permeability(k_lattice: float, dx: float) -> float:
    """Lattice permeability (lattice units) to m^2."""
    return float(k_lattice) * dx * dx


def total_lnk_gradient(g_lnk, g_lnkn0):
    """dJ/d ln k_d for a medium whose kn0 follows from k_d by Eq. 11
    (r ~ sqrt(k_d), so kn0 ~ k_d^-1/2): dJ/d ln k - 1/2 dJ/d ln kn0."""
    return g_lnk - 0.5 * g_lnkn0


def porosity_curves(eps: Iterable[float], d: float, gas: Gas,
                    pressures_psi: Iterable[float], correlation="bkc",
                    slip_b: float = -1.0) -> Dict[str, np.ndarray]:
    """The curves of Fig. 1: pore radius (Eqs. 9, 11), Knudsen number and
    correction factor against porosity, at each pressure (psi)."""
    eps = np.asarray(list(eps), dtype=np.float64)
    r = pore_radius(kozeny_carman(eps, d), eps)
    out = {"eps": eps, "r": r}
    for p in pressures_psi:
        kn = knudsen(gas.mean_free_path(p * PSI), r)
        out[f"kn@{p:g}psi"] = kn
        out[f"fc@{p:g}psi"] = correction_factor(kn, correlation, slip_b)
    return out


def viscosity_for_mean_free_path(lam: float, p: float, T: float,
                                 M: float = METHANE_MOLAR_MASS) -> float:
    """The viscosity for which Eq. 10 gives the mean free path lam at (p, T)."""
    return lam * p / math.sqrt(math.pi * R_GAS * T / (2.0 * M))


def paper_gas() -> Gas:
    """Methane at 323 K with the viscosities that reproduce the mean free
    paths printed in Sec. IV.A at 4000, 1000 and 100 psi (the paper takes
    the viscosity from an external tool and prints only lambda)."""
    lam = {4000.0: 0.38e-9, 1000.0: 1.09e-9, 100.0: 10.26e-9}
    return Gas(T=323.0, M=METHANE_MOLAR_MASS,
               mu={p * PSI: viscosity_for_mean_free_path(l, p * PSI, 323.0)
                   for p, l in lam.items()})
