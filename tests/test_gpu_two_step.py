"""The two-step pass (two time steps per launch, the old and intermediate
levels in registers) against single steps, through the C ABI: a lattice
with pass_mode LBK_PASS_TWO_STEP runs lbk_step(n) as n/2 two-step passes
(and one single sweep if n is odd), so it must end bitwise where n single
sweeps (LBK_PASS_SINGLE) leave the same lattice, for FP32, FP16 and BF16
storage.  Sizes around the 60-column strips, bands of 1 to 16 rows, every
boundary combination.  A gradient whose recomputing sweeps take two-step
passes equals the single-sweep one bitwise, and the automatic mode picks
the two-step pass on large lattices only."""
import numpy as np
import pytest
import torch

from paper_1411_7051_amd import inputs
from paper_1411_7051_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

BCS = [(0, 0), (0, 1), (1, 1), (1, 0), (2, 0), (2, 1)]
SIZES = [(1, 1), (2, 3), (3, 1), (3, 5), (59, 7), (60, 13), (61, 6), (62, 33), (63, 31),
         (64, 32), (65, 1), (120, 65), (121, 40), (124, 12), (300, 37), (1030, 3)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda", 0)
    torch.cuda.set_device(d)
    return d


def pair(dev, case, storage, steps, band=0):
    """a: single sweeps (one lbk_step(1) call each); b: lbk_step(steps) with
    two-step passes requested whatever the lattice size (bands of `band`
    rows; 0: the library's choice)."""
    a = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, check_every=0,
                pass_mode="single", **case.params)
    b = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, check_every=0,
                pass_mode="two_step", band=band, **case.params)
    for _ in range(steps):
        a.step(1)
    b.step(steps)
    assert a.time == b.time == steps
    sa, sb = a.save_state(), b.save_state()
    return a, b, sa, sb


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("bcx,bcy", BCS)
def test_two_step_pass_is_bitwise_two_single_steps(dev, storage, bcx, bcy):
    for nx, ny in SIZES:
        if bcx == inputs.PRESSURE and nx < 3:
            continue
        drive = (dict(rho_in=1.03, rho_out=1.0, init=1) if bcx == inputs.PRESSURE
                 else dict(gx=1e-4, gy=-3e-5))
        case = inputs.random_medium(nx, ny, seed=nx * 31 + ny, solid_frac=0.08, pore_frac=0.08,
                                    kn_range=(0.0, 2.0), bc_x=bcx, bc_y=bcy, **drive)
        for steps in (2, 7):
            a, b, sa, sb = pair(dev, case, storage, steps)
            if not torch.equal(sa, sb):
                fa, fb = a.populations(), b.populations()
                pytest.fail(f"{nx}x{ny} {storage} bc ({bcx},{bcy}) {steps} steps: "
                            f"max |diff| {float((fa - fb).abs().max()):.3e}")
            a.close()
            b.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("band", [1, 3, 5, 8, 10, 16])
def test_two_step_pass_bands(dev, storage, band):
    """Any band gives the same state: the march unrolled over five rows with
    every remainder, bands taller than the lattice, walls at a band's
    ends."""
    for bcx, bcy in ((2, 0), (2, 1), (0, 1), (1, 1)):
        for nx, ny in ((61, 6), (63, 31), (121, 40), (300, 37)):
            drive = (dict(rho_in=1.03, rho_out=1.0, init=1) if bcx == inputs.PRESSURE
                     else dict(gx=1e-4, gy=-3e-5))
            case = inputs.random_medium(nx, ny, seed=nx * 41 + ny + band, solid_frac=0.08,
                                        pore_frac=0.08, kn_range=(0.0, 2.0), bc_x=bcx,
                                        bc_y=bcy, **drive)
            for steps in (2, 7):
                a, b, sa, sb = pair(dev, case, storage, steps, band)
                assert torch.equal(sa, sb), (nx, ny, bcx, bcy, steps)
                a.close()
                b.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_two_step_pass_forchheimer_and_correlations(dev, storage):
    for extra in (dict(f_eps=0.7), dict(correlation=1), dict(correlation=2),
                  dict(kn_local=0, rho_ref=0.5)):
        case = inputs.random_medium(200, 70, seed=91, solid_frac=0.05, pore_frac=0.05,
                                    kn_range=(0.0, 2.0), bc_x=2, bc_y=1, rho_in=1.02,
                                    rho_out=1.0, init=1, **extra)
        _, _, sa, sb = pair(dev, case, storage, 6)
        assert torch.equal(sa, sb), extra


def test_two_step_pass_discs_window(dev):
    """A 1024 x 512 cut of the benchmark's disc medium: many bands and
    strips, 40 steps."""
    case = inputs.discs(n=1024, seed=2)
    case = inputs.Case(np.ascontiguousarray(case.eps[:512]), np.ascontiguousarray(case.k[:512]),
                       np.ascontiguousarray(case.kn0[:512]), case.params, "discs-cut")
    for storage in ("f32", "f16", "bf16"):
        _, _, sa, sb = pair(dev, case, storage, 40)
        assert torch.equal(sa, sb), storage


def test_two_step_recording_sweeps_bitwise(dev):
    """The adjoint's recomputing sweeps record the history of both steps of
    a two-step pass: the gradient equals the single-sweep gradient bitwise
    (odd inner segments included)."""
    case = inputs.random_medium(300, 40, seed=92, solid_frac=0.05, pore_frac=0.05,
                                bc_x=2, bc_y=1, rho_in=1.02, rho_out=1.0, init=1)
    out = []
    for mode in ("single", "two_step"):
        lat = Lattice(case.eps, case.k, case.kn0, device=dev, pass_mode=mode, **case.params)
        J, gk, gn = lat.gradient(37, "k_app", ckpt_every=15, hist_len=7, wrt_kn0=True)
        out.append((J, gk, gn))
        lat.close()
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1]) and torch.equal(out[0][2], out[1][2])


def test_auto_mode_matches_both(dev):
    """LBK_PASS_AUTO takes two-step passes from 2^20 nodes at FP32 and from
    2^22 at FP16 (bands shortened to fill the device), single sweeps below;
    either way the state equals the other modes' bitwise."""
    for nx, ny, storage, two in ((1024, 1024, "f32", True), (1023, 1024, "f32", False),
                                 (2048, 1024, "f16", False), (2048, 2048, "f16", True)):
        case = inputs.random_medium(nx, ny, seed=94, solid_frac=0.02, pore_frac=0.02,
                                    bc_x=2, rho_in=1.01, rho_out=1.0, init=1)
        states = []
        for mode in ("auto", "single", "two_step"):
            lat = Lattice(case.eps, case.k, case.kn0, device=dev, pass_mode=mode,
                          storage=storage, **case.params)
            expect = {"auto": 2 if two else 1, "single": 1, "two_step": 2}[mode]
            assert lat.steps_per_launch == expect, (nx, ny, storage, mode)
            lat.step(4)
            states.append(lat.save_state())
            lat.close()
        assert torch.equal(states[0], states[1]) and torch.equal(states[0], states[2])
