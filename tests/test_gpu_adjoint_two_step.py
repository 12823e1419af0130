"""The two-step reverse pass (two reverse steps per launch, the intermediate
adjoint state in registers) against single reverse steps, through the C ABI:
a gradient taken with pass_mode LBK_PASS_TWO_STEP reverses its segments in
pairs of steps (and one single step where a segment's length is odd), so it
must equal the gradient of LBK_PASS_SINGLE bitwise.  Sizes around the
60-column strips (a pressure outlet next to a strip's edge included), bands
of 1 to 17 rows, every boundary combination, both objectives, the ln kn0
plane, the Forchheimer term and the slip correlations."""
import pytest
import torch

from paper_1411_7051_amd import inputs
from paper_1411_7051_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

BCS = [(0, 0), (0, 1), (1, 1), (1, 0), (2, 0), (2, 1)]
# nx = 63, 123, 183: the column next to the outlet would fall on the last
# lane of the second-to-last strip
SIZES = [(3, 4), (4, 1), (5, 7), (59, 7), (60, 13), (61, 6), (62, 9), (63, 31), (64, 5),
         (65, 2), (120, 8), (121, 11), (123, 12), (124, 3), (183, 7), (300, 17)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda", 0)
    torch.cuda.set_device(d)
    return d


def grads(dev, case, storage, steps, ckpt, hist, objective="k_app", band=0):
    out = []
    for mode in ("single", "two_step"):
        lat = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, check_every=0,
                      pass_mode=mode, band=band if mode == "two_step" else 0, **case.params)
        lat.step(3)
        out.append(lat.gradient(steps, objective, ckpt_every=ckpt, hist_len=hist,
                                wrt_kn0=True))
        lat.close()
    return out


def assert_same(out, what):
    (Ja, ka, na), (Jb, kb, nb) = out
    assert Ja == Jb, what
    for a, b, name in ((ka, kb, "ln k"), (na, nb, "ln kn0")):
        if not torch.equal(a, b):
            d = (a - b).abs()
            scale = float(a.abs().max())
            pytest.fail(f"{what} {name}: max |diff| {float(d.max()):.3e} (max |g| {scale:.3e}) "
                        f"at {divmod(int(d.argmax()), a.shape[1])}")


@pytest.mark.parametrize("bcx,bcy", BCS)
def test_two_step_reverse_is_bitwise_two_single_steps(dev, bcx, bcy):
    for nx, ny in SIZES:
        if bcx == inputs.PRESSURE and nx < 3:
            continue
        drive = (dict(rho_in=1.03, rho_out=1.0, init=1) if bcx == inputs.PRESSURE
                 else dict(gx=1e-4, gy=-3e-5))
        case = inputs.random_medium(nx, ny, seed=nx * 29 + ny, solid_frac=0.08, pore_frac=0.08,
                                    kn_range=(0.0, 2.0), bc_x=bcx, bc_y=bcy, **drive)
        # one segment of 9 steps (four pairs and a single step), then
        # segments of 4 and 3 steps
        for steps, ckpt, hist in ((9, 9, 9), (11, 7, 4)):
            assert_same(grads(dev, case, "f32", steps, ckpt, hist),
                        f"{nx}x{ny} bc ({bcx},{bcy}) {steps} steps ckpt {ckpt} hist {hist}")


def test_two_step_reverse_outlet_flux_and_fp16(dev):
    case = inputs.random_medium(183, 20, seed=95, solid_frac=0.05, pore_frac=0.05,
                                kn_range=(0.0, 2.0), bc_x=2, bc_y=1, rho_in=1.02, rho_out=1.0,
                                init=1)
    assert_same(grads(dev, case, "f32", 12, 12, 6, objective="q_out"), "outlet flux")
    assert_same(grads(dev, case, "f16", 10, 10, 10), "f16 storage")


@pytest.mark.parametrize("extra", [dict(f_eps=0.7), dict(correlation=1), dict(correlation=2),
                                   dict(kn_local=0, rho_ref=0.5), dict(rho_ref=2.0)])
def test_two_step_reverse_model_options(dev, extra):
    case = inputs.random_medium(250, 40, seed=96, solid_frac=0.05, pore_frac=0.05,
                                kn_range=(0.0, 2.0), bc_x=2, bc_y=0, rho_in=1.02, rho_out=1.0,
                                init=1, **extra)
    assert_same(grads(dev, case, "f32", 10, 10, 10), str(extra))


@pytest.mark.parametrize("band", [1, 3, 6, 16, 17])
def test_two_step_reverse_bands(dev, band):
    """Bands of any height reverse to the same gradient: the whole-period
    loop of 16 rows with every remainder, and bands taller than the
    lattice."""
    for bcx, bcy in ((2, 0), (2, 1), (0, 1)):
        for nx, ny in ((63, 31), (121, 40), (183, 7)):
            drive = (dict(rho_in=1.03, rho_out=1.0, init=1) if bcx == inputs.PRESSURE
                     else dict(gx=1e-4, gy=-3e-5))
            case = inputs.random_medium(nx, ny, seed=nx * 37 + ny + band, solid_frac=0.08,
                                        pore_frac=0.08, kn_range=(0.0, 2.0), bc_x=bcx,
                                        bc_y=bcy, **drive)
            assert_same(grads(dev, case, "f32", 9, 9, 9, band=band),
                        f"{nx}x{ny} bc ({bcx},{bcy}) band {band}")
