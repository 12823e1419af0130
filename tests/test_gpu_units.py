"""The physical-units front end driving the HIP sweep: a porous channel
described in SI units (grain diameter, porosity, node spacing, methane at a
pressure in psi) runs to steady state and its global permeability, in m^2,
matches the Brinkman channel closed form with the Klinkenberg factor at the
pressure's Knudsen number (Sec. IV.A); it rises as the pressure falls."""
import math

import numpy as np
import pytest
import torch

from paper_1411_7051_amd import inputs, units
from paper_1411_7051_amd.lattice import Lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda", 0)
    torch.cuda.set_device(d)
    return d


def test_physical_channel(dev):
    nx, ny, dx, eps, d = 256, 48, 10e-9, 0.2, 40e-9
    gas = units.paper_gas()
    kd = units.kozeny_carman(eps, d)
    r = units.pore_radius(kd, eps)
    out = {}
    for p in (4000.0, 1000.0, 100.0):
        e, k, kn0 = units.lattice_fields(np.full((ny, nx), eps), np.full((ny, nx), kd), dx, gas,
                                         p * units.PSI)
        params = inputs.run_params(tau=0.8, bc_x=inputs.PRESSURE, bc_y=inputs.WALL,
                                   rho_in=1.01, rho_out=1.0, init=1)
        lat = Lattice(e, k, kn0, device=dev, **params)
        steps, res, why = lat.run_to_steady(every=200, tol=1e-9, max_steps=400000)
        assert res < 1e-6, (p, steps, res, why)
        k_app = units.physical_permeability(lat.apparent_permeability(), dx)
        kn = gas.mean_free_path(p * units.PSI) / r
        fc = float(units.correction_factor([kn])[0])
        a = math.sqrt(eps / (kd * fc / (dx * dx)))  # 1 / nodes
        expect = kd * fc * (1 - math.tanh(a * ny / 2) / (a * ny / 2))
        assert abs(k_app / expect - 1) < 0.015, (p, k_app, expect)
        out[p] = k_app
    assert out[100.0] > out[1000.0] > out[4000.0] > kd * 0.9
