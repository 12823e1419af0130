"""lbk_apparent_permeability_noalloc (through the C ABI) against
lbk_apparent_permeability: two calls in a row on one GPU, the second on a
smaller lattice, so the fixed device scratch array is reused with fewer
partials; each must equal the allocating entry point's value to FP64
rounding of the regrouped sums."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1411_7051_amd import _lib, inputs
from paper_1411_7051_amd.lattice import Lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda", 0)
    torch.cuda.set_device(d)
    return d


def both(lat):
    lib = _lib.load()
    a, b = ctypes.c_double(), ctypes.c_double()
    _lib.check(lib.lbk_apparent_permeability(lat._handle(), ctypes.byref(a)))
    _lib.check(lib.lbk_apparent_permeability_noalloc(lat._handle(), ctypes.byref(b)))
    return a.value, b.value


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_noalloc_matches_allocating_entry_point(dev, storage):
    # first call: more 256-node blocks (4 x 2000 = 8000) than the fixed grid
    # of 2048 workgroups, so each walks several; second: 2 x 37 = 74 blocks
    big = inputs.random_medium(1000, 2000, seed=77, solid_frac=0.05, pore_frac=0.05,
                               bc_x=inputs.PRESSURE, bc_y=inputs.WALL, rho_in=1.01,
                               rho_out=1.0, init=1)
    small = inputs.random_medium(300, 37, seed=78, solid_frac=0.05, pore_frac=0.05,
                                 gx=2e-5, bc_y=inputs.WALL)
    seen = []
    for case, steps in ((big, 60), (small, 40)):
        lat = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, **case.params)
        lat.step(steps)
        want, got = both(lat)
        print(f"{case.name} {storage}: allocating {want:.17e}, no-alloc {got:.17e}",
              flush=True)
        assert np.isfinite(want) and want > 0
        assert abs(got - want) <= 1e-12 * abs(want)
        seen.append(got)
        lat.close()
    assert seen[0] != seen[1]


def test_noalloc_refuses_undriven(dev):
    case = inputs.random_medium(40, 8, seed=79)  # periodic, no drive
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    out = ctypes.c_double()
    st = _lib.load().lbk_apparent_permeability_noalloc(lat._handle(), ctypes.byref(out))
    assert st == -1
    lat.close()
