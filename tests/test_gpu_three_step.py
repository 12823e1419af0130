"""The three-step pass (three time steps per launch, the old level and two
intermediate levels in registers) against single steps, through the C ABI:
a lattice with pass_mode LBK_PASS_THREE_STEP runs lbk_step(n) as n // 3
three-step passes and the remainder as a two-step pass or a single sweep,
so it must end bitwise where n single sweeps (LBK_PASS_SINGLE) leave the
same lattice, for FP32, FP16 and BF16 storage.  Sizes around the 58-column
strips, bands of 1 to 16 rows, every boundary combination; a gradient of
such a lattice (recording three steps per pass, reversing two) equals the
single-sweep one bitwise."""
import numpy as np
import pytest
import torch

from paper_1411_7051_amd import inputs
from paper_1411_7051_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

BCS = [(0, 0), (0, 1), (1, 1), (1, 0), (2, 0), (2, 1)]
SIZES = [(1, 1), (2, 3), (3, 1), (3, 5), (57, 7), (58, 13), (59, 6), (60, 33), (61, 31),
         (62, 4), (64, 32), (116, 9), (117, 40), (118, 12), (300, 37), (1030, 3)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda", 0)
    torch.cuda.set_device(d)
    return d


def pair(dev, case, storage, steps, band=0):
    """a: single sweeps (one lbk_step(1) call each); b: lbk_step(steps) with
    three-step passes requested whatever the lattice size."""
    a = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, check_every=0,
                pass_mode="single", **case.params)
    b = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, check_every=0,
                pass_mode="three_step", band=band, **case.params)
    assert b.steps_per_launch == 3
    for _ in range(steps):
        a.step(1)
    b.step(steps)
    assert a.time == b.time == steps
    return a, b, a.save_state(), b.save_state()


def _case(nx, ny, bcx, bcy, seed):
    drive = (dict(rho_in=1.03, rho_out=1.0, init=1) if bcx == inputs.PRESSURE
             else dict(gx=1e-4, gy=-3e-5))
    return inputs.random_medium(nx, ny, seed=seed, solid_frac=0.08, pore_frac=0.08,
                                kn_range=(0.0, 2.0), bc_x=bcx, bc_y=bcy, **drive)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("bcx,bcy", BCS)
def test_three_step_pass_is_bitwise_three_single_steps(dev, storage, bcx, bcy):
    for nx, ny in SIZES:
        if bcx == inputs.PRESSURE and nx < 3:
            continue
        case = _case(nx, ny, bcx, bcy, nx * 37 + ny)
        # 3: one pass; 7: two passes and a single sweep; 8: two passes and
        # a two-step pass
        for steps in (3, 7, 8):
            a, b, sa, sb = pair(dev, case, storage, steps)
            if not torch.equal(sa, sb):
                fa, fb = a.populations(), b.populations()
                pytest.fail(f"{nx}x{ny} {storage} bc ({bcx},{bcy}) {steps} steps: "
                            f"max |diff| {float((fa - fb).abs().max()):.3e}")
            a.close()
            b.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("band", [1, 2, 3, 5, 8, 10, 16])
def test_three_step_pass_bands(dev, storage, band):
    """Any band gives the same state: the march unrolled over five rows with
    every remainder, bands taller than the lattice, walls at a band's
    ends."""
    for bcx, bcy in ((2, 0), (2, 1), (0, 1), (1, 1)):
        for nx, ny in ((59, 6), (61, 31), (117, 40), (300, 37)):
            case = _case(nx, ny, bcx, bcy, nx * 43 + ny + band)
            for steps in (3, 9):
                a, b, sa, sb = pair(dev, case, storage, steps, band)
                assert torch.equal(sa, sb), (nx, ny, bcx, bcy, steps)
                a.close()
                b.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_three_step_pass_forchheimer_and_correlations(dev, storage):
    for extra in (dict(f_eps=0.7), dict(correlation=1), dict(correlation=2),
                  dict(kn_local=0, rho_ref=0.5)):
        case = inputs.random_medium(200, 70, seed=93, solid_frac=0.05, pore_frac=0.05,
                                    kn_range=(0.0, 2.0), bc_x=2, bc_y=1, rho_in=1.02,
                                    rho_out=1.0, init=1, **extra)
        _, _, sa, sb = pair(dev, case, storage, 9)
        assert torch.equal(sa, sb), extra


def test_three_step_pass_discs_window(dev):
    """A 1024 x 512 cut of the benchmark's disc medium: many bands and
    strips, 42 steps."""
    case = inputs.discs(n=1024, seed=2)
    case = inputs.Case(np.ascontiguousarray(case.eps[:512]), np.ascontiguousarray(case.k[:512]),
                       np.ascontiguousarray(case.kn0[:512]), case.params, "discs-cut")
    for storage in ("f32", "f16", "bf16"):
        _, _, sa, sb = pair(dev, case, storage, 42)
        assert torch.equal(sa, sb), storage


def test_three_step_lattice_gradient_bitwise(dev):
    """A gradient of a three-step lattice rebuilds and records in three-step
    passes and reverses in two-step passes: it equals the single-sweep
    gradient bitwise."""
    case = inputs.random_medium(300, 40, seed=95, solid_frac=0.05, pore_frac=0.05,
                                bc_x=2, bc_y=1, rho_in=1.02, rho_out=1.0, init=1)
    out = []
    for mode in ("single", "three_step"):
        lat = Lattice(case.eps, case.k, case.kn0, device=dev, pass_mode=mode, **case.params)
        J, gk, gn = lat.gradient(37, "k_app", ckpt_every=15, hist_len=7, wrt_kn0=True)
        out.append((J, gk, gn))
        lat.close()
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1]) and torch.equal(out[0][2], out[1][2])


def test_auto_mode_three_step_thresholds(dev):
    """LBK_PASS_AUTO takes three-step passes from 2^22 nodes at FP32 and from
    2^23 at FP16, two-step passes below (down to their own thresholds);
    either way the state equals the single sweeps' bitwise."""
    for nx, ny, storage, k in ((2048, 2048, "f32", 3), (2047, 2048, "f32", 2),
                               (4096, 2048, "f16", 3), (4095, 2048, "f16", 2)):
        case = inputs.random_medium(nx, ny, seed=96, solid_frac=0.02, pore_frac=0.02,
                                    bc_x=2, rho_in=1.01, rho_out=1.0, init=1)
        states = []
        for mode in ("auto", "single"):
            lat = Lattice(case.eps, case.k, case.kn0, device=dev, pass_mode=mode,
                          storage=storage, **case.params)
            assert lat.steps_per_launch == (k if mode == "auto" else 1), (nx, ny, storage)
            lat.step(5)
            states.append(lat.save_state())
            lat.close()
        assert torch.equal(states[0], states[1]), (nx, ny, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 1), (2, 0), (2, 1)])
def test_three_step_recording_bitwise(dev, storage, bcx, bcy):
    """The recording passes of a three-step lattice take three steps and
    record all three: J and both gradient planes equal the single-sweep
    ones bitwise, for inner segments of every length modulo 3, both
    objectives and bands that do and do not divide the lattice."""
    drive = (dict(rho_in=1.02, rho_out=1.0, init=1) if bcx == inputs.PRESSURE
             else dict(gx=1e-5, gy=-3e-6))
    case = inputs.random_medium(121, 37, seed=97 + bcx, solid_frac=0.05, pore_frac=0.05,
                                kn_range=(0.0, 2.0), bc_x=bcx, bc_y=bcy, **drive)
    for steps, ckpt, hist, objective, band in ((29, 13, 6, "k_app", 0), (31, 16, 7, "q_out", 5),
                                               (30, 15, 8, "k_app", 12)):
        if objective == "q_out" and bcx != inputs.PRESSURE:
            objective = "k_app"
        out = []
        for mode in ("single", "three_step"):
            lat = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage,
                          pass_mode=mode, band=band if mode == "three_step" else 0,
                          **case.params)
            out.append(lat.gradient(steps, objective, ckpt_every=ckpt, hist_len=hist,
                                    wrt_kn0=True))
            lat.close()
        assert out[0][0] == out[1][0], (steps, ckpt, hist)
        assert torch.equal(out[0][1], out[1][1]) and torch.equal(out[0][2], out[1][2]), \
            (steps, ckpt, hist, objective, band)


def test_batch_refuses_three_step_mode(dev):
    """Batches have no three-step pass: the mode is refused and the batch
    keeps stepping as before, bitwise its lattices' single sweeps."""
    from paper_1411_7051_amd import _lib
    from paper_1411_7051_amd.batch import Batch
    case = _case(61, 31, 2, 0, 98)
    lats = [Lattice(case.eps, case.k, case.kn0, device=dev, check_every=0, **case.params)
            for _ in range(2)]
    solo = Lattice(case.eps, case.k, case.kn0, device=dev, check_every=0, pass_mode="single",
                   **case.params)
    b = Batch(lats)
    with pytest.raises(_lib.LbkError):
        b.set_pass_mode("three_step")
    b.step(4)
    solo.step(4)
    for lat in lats:
        assert torch.equal(lat.save_state(), solo.save_state())
    b.close()
    for lat in lats + [solo]:
        lat.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_three_step_with_state_checks(dev, storage):
    """State checks (and, at FP16, the scale re-centring) fall at multiples
    of check_every in the lattice's time whatever the pass: a check interval
    of 7 cuts every chunk into two three-step passes and a single sweep,
    and the state still equals the single sweeps' bitwise."""
    case = _case(300, 37, 2, 1, 99)
    a = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, check_every=7,
                pass_mode="single", **case.params)
    b = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, check_every=7,
                pass_mode="three_step", **case.params)
    for n in (5, 13, 22):
        a.step(n)
        b.step(n)
    assert a.time == b.time == 40
    assert torch.equal(a.save_state(), b.save_state())
    a.close()
    b.close()
