"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP32 storage: velocity relative L2 <= 1e-5 against the oracle after the same
number of steps on the same seeded inputs; populations compared element by
element.  Sizes span several 256-wide blocks with a ragged tail."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1411_7051_amd import inputs
from paper_1411_7051_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

VEL_TOL = 1e-5  # relative L2 on velocity, FP32 path vs FP64 oracle


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda", 0)
    torch.cuda.set_device(d)
    return d


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_run(dev, case, steps, **extra):
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params, **extra)
    lat.step(steps)
    return lat


def macro_np(lat):
    return [t.double().cpu().numpy() for t in lat.macroscopic()]


def oracle_run(case, steps):
    return oracle.Lattice(case.eps, case.k, case.kn0, **case.params).step(steps)


def compare(lat, ref, tol=VEL_TOL):
    rho, ux, uy = macro_np(lat)
    r_rho, r_ux, r_uy = ref.macro()
    err = rel_l2(np.stack([ux, uy]), np.stack([r_ux, r_uy]))
    assert err <= tol, f"velocity rel L2 {err:.3e}"
    assert np.max(np.abs(rho - r_rho)) < 1e-6
    f = lat.populations().cpu().numpy()
    fr = ref.state()
    # deviations from the local equilibrium scale
    scale = np.max(np.abs(fr - fr.sum(axis=0, keepdims=True) * W[:, None, None]))
    assert np.max(np.abs(f - fr)) <= 1e-4 * scale + 1e-12
    return err


W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def test_channel_workload(dev):
    """Porous-filled plates, 64x32, eps 0.5, Da 1e-3, tau 0.8, body force
    1e-6, 10,000 steps from rest (Sec. IV.A)."""
    case = inputs.channel(64, 32, eps=0.5, k=1.024, gx=1e-6)
    lat = gpu_run(dev, case, 10000)
    ref = oracle_run(case, 10000)
    compare(lat, ref)
    kg, kr = lat.apparent_permeability(), ref.apparent_permeability()
    assert abs(kg / kr - 1) < 1e-5


def test_uniform_recurrence(dev):
    """Closed form on a uniform periodic medium with Klinkenberg on:
    u_{n+1} = q u_n + eps G/(1 + A/2) (see the oracle pins)."""
    eps, k, kn0, tau, G = 0.4, 0.3, 0.5, 0.8, 1e-5
    case = inputs.Case(*(np.full((5, 70), v, np.float32) for v in (eps, k, kn0)),
                       inputs.run_params(tau=tau, gx=G))
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    nu = (tau - 0.5) / 3
    A = float(np.float32(eps)) * nu / (float(np.float32(k)) * oracle.fc(float(np.float32(kn0))))
    q, b = (1 - A / 2) / (1 + A / 2), float(np.float32(eps)) * G / (1 + A / 2)
    u = 0.5 * b
    for n in range(40):
        _, ux, uy = macro_np(lat)
        assert np.allclose(ux, u, rtol=2e-6)
        assert np.max(np.abs(uy)) < 1e-7 * u
        lat.step(1)
        u = q * u + b


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (0, 1), (1, 1), (1, 0), (2, 0), (2, 1)])
def test_random_media(dev, bcx, bcy):
    """Heterogeneous medium with free-fluid and impermeable nodes, local Kn,
    every boundary combination; 300x37 (two full blocks and a ragged tail)."""
    drive = dict(gx=3e-5, gy=-1e-5) if bcx != 2 else dict(rho_in=1.01, rho_out=1.0, init=1)
    case = inputs.random_medium(300, 37, seed=100 + 3 * bcx + bcy, solid_frac=0.08,
                                pore_frac=0.08, bc_x=bcx, bc_y=bcy, **drive)
    lat = gpu_run(dev, case, 300)
    ref = oracle_run(case, 300)
    compare(lat, ref)


def test_forchheimer(dev):
    case = inputs.random_medium(130, 20, seed=5, bc_y=1, gx=2e-4, f_eps=0.6)
    compare(gpu_run(dev, case, 400), oracle_run(case, 400))


def test_global_kn(dev):
    case = inputs.random_medium(70, 30, seed=6, kn_local=0, bc_x=2, rho_in=1.02,
                                rho_out=1.0, init=1)
    compare(gpu_run(dev, case, 300), oracle_run(case, 300))


@pytest.mark.parametrize("corr,slip_b,kn_local,rho_ref",
                         [(1, -1.0, 1, 1.0), (2, -1.0, 1, 1.0), (0, -0.4, 1, 1.0),
                          (0, 0.0, 0, 1.0), (1, -1.0, 0, 1.0), (0, -1.0, 1, 2.0),
                          (1, -1.0, 1, 0.5), (0, -1.0, 0, 0.5)])
def test_correlations(dev, corr, slip_b, kn_local, rho_ref):
    """Selectable slip correlation (Eqs. 6-7 with slip coefficient b, Eqs.
    4-5, none), a local or a fixed Kn, and kn0 quoted at a reference density
    other than 1 (Kn = kn0 rho_ref / rho; no effect with a fixed Kn), against
    the oracle on a pressure-driven heterogeneous medium with Kn up to 3."""
    case = inputs.random_medium(130, 21, seed=60 + corr, solid_frac=0.05, pore_frac=0.05,
                                kn_range=(0.0, 3.0), bc_x=2, bc_y=1, rho_in=1.02,
                                rho_out=1.0, init=1, correlation=corr, slip_b=slip_b,
                                kn_local=kn_local, rho_ref=rho_ref)
    lat = gpu_run(dev, case, 300)
    ref = oracle_run(case, 300)
    compare(lat, ref)
    assert abs(lat.apparent_permeability() / ref.apparent_permeability() - 1) < 1e-5


@pytest.mark.parametrize("nx,ny,bcx,bcy", [(1, 1, 0, 0), (1, 9, 0, 1), (7, 1, 0, 0),
                                           (3, 4, 2, 1), (3, 1, 2, 0), (257, 3, 1, 1),
                                           (64, 64, 0, 0), (513, 5, 2, 0)])
def test_edge_sizes(dev, nx, ny, bcx, bcy):
    drive = dict(gx=1e-4, gy=5e-5) if bcx != 2 else dict(rho_in=1.03, rho_out=1.0, init=1)
    case = inputs.random_medium(nx, ny, seed=nx * 7 + ny, solid_frac=0.1, pore_frac=0.1,
                                bc_x=bcx, bc_y=bcy, **drive)
    lat = gpu_run(dev, case, 60)
    ref = oracle_run(case, 60)
    rho, ux, uy = macro_np(lat)
    _, r_ux, r_uy = ref.macro()
    un = np.linalg.norm(np.stack([r_ux, r_uy]))
    if un > 0:
        assert rel_l2(np.stack([ux, uy]), np.stack([r_ux, r_uy])) <= VEL_TOL
    else:
        assert np.max(np.abs(ux)) == 0 and np.max(np.abs(uy)) == 0


def test_mass_conservation(dev):
    """Periodic x, walls in y: streaming and collision conserve mass.  The
    FP32 deviation planes round each stored value, so the FP64 total drifts
    at the level of FP32 rounding of the deviations (not of the O(1)
    populations): bounded here at 1e-8 relative over 2000 steps at flow
    speeds up to ~1e-3."""
    case = inputs.random_medium(200, 50, seed=8, solid_frac=0.1, pore_frac=0.1, bc_y=1,
                                gx=1e-4, gy=2e-5)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    m0, _, _ = lat.diagnostics()
    lat.step(2000)
    m1, _, _ = lat.diagnostics()
    assert abs(m1 - m0) / m0 < 1e-8


def test_apparent_permeability_pressure(dev):
    case = inputs.channel(48, 12, eps=0.5, k=0.05, kn0=0.4, drive="pressure")
    lat = gpu_run(dev, case, 3000)
    ref = oracle_run(case, 3000)
    assert abs(lat.apparent_permeability() / ref.apparent_permeability() - 1) < 1e-5


def test_deterministic_and_resumable(dev):
    case = inputs.random_medium(300, 40, seed=9, solid_frac=0.05, bc_x=2, rho_in=1.01,
                                rho_out=1.0, init=1)
    a = gpu_run(dev, case, 100)
    b = gpu_run(dev, case, 100)
    assert torch.equal(a.populations(), b.populations())
    snap = a.save_state()
    a.step(100)
    c = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    c.load_state(snap)
    assert c.time == 100
    c.step(100)
    assert torch.equal(a.populations(), c.populations())
    ka, kc = a.apparent_permeability(), c.apparent_permeability()
    assert ka == kc


def test_invalid_fields_rejected(dev):
    from paper_1411_7051_amd._lib import LbkError
    eps = np.full((8, 16), 0.5, np.float32)
    k = np.full((8, 16), 1.0, np.float32)
    bad = eps.copy()
    bad[3, 4] = 1.5
    with pytest.raises(LbkError):
        Lattice(bad, k, device=dev)
    badk = k.copy()
    badk[0, 0] = np.nan
    with pytest.raises(LbkError):
        Lattice(eps, badk, device=dev)


def test_nonfinite_detected(dev):
    """A tau close to 1/2 with a strong force blows up; the periodic check
    reports it instead of running on with NaNs."""
    from paper_1411_7051_amd._lib import LbkError
    case = inputs.random_medium(64, 16, seed=12, eps_range=(0.9, 1.0), k_range=(1e3, 1e4),
                                tau=0.5000001, gx=0.5)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, check_every=50, **case.params)
    with pytest.raises(LbkError) as e:
        lat.step(5000)
    assert e.value.status == -4


def test_zero_and_negative_steps(dev):
    """step(0) leaves the state and the clock untouched; a negative count is
    rejected before any device work."""
    from paper_1411_7051_amd._lib import LbkError
    case = inputs.random_medium(40, 9, seed=13, bc_x=2, rho_in=1.01, rho_out=1.0, init=1)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    lat.step(3)
    before = lat.populations().clone()
    lat.step(0)
    assert lat.time == 3 and torch.equal(lat.populations(), before)
    with pytest.raises(LbkError) as e:
        lat.step(-1)
    assert e.value.status == -1 and lat.time == 3


@pytest.mark.parametrize("storage,tol", [("f32", 2e-7), ("f16", 1e-5)])
def test_pressure_columns_hold_their_density(dev, storage, tol):
    """As in the oracle: after every step the end columns hold rho_in and
    rho_out (their populations sum to the boundary density; FP32 density
    plane plus rounded deviations)."""
    case = inputs.random_medium(70, 11, seed=17, solid_frac=0.05, bc_x=2, bc_y=1,
                                rho_in=1.03, rho_out=0.99, init=1, kn_range=(0.0, 2.0))
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, storage=storage, **case.params)
    for _ in range(3):
        lat.step(9)
        rho = lat.populations().sum(dim=0).cpu().numpy()
        assert np.allclose(rho[:, 0], 1.03, rtol=tol, atol=0)
        assert np.allclose(rho[:, -1], 0.99, rtol=tol, atol=0)


def _scale_exp(lat):
    """Exponent e of the FP16 storage scale 2^e, from the saved-state header
    (int64 words: magic, step, e, ...)."""
    return int(lat.save_state()[:64].cpu().view(torch.int64)[2])


@pytest.mark.parametrize("make,exact", [
    (lambda: inputs.channel(nx=300, ny=40, drive="force", gx=1e-5), True),
    (lambda: inputs.channel(nx=300, ny=40, drive="pressure"), False),
    (lambda: inputs.random_medium(300, 70, seed=21, gx=1e-5, bc_y=inputs.WALL), False),
], ids=["channel-force", "channel-pressure", "random"])
def test_fp16_scale_recentring_is_exact(dev, make, exact):
    """FP16 deviations are stored times 2^e; a state check moves e so that the
    largest stored magnitude sits in [2^12, 2^13).  Multiplying by a power of
    two is exact, and every later FP32 operation on values in the storage unit
    scales with it, so a run with checks matches one without bit for bit as
    long as no stored value is an FP16 subnormal at either exponent; otherwise
    the two differ by the subnormal quantum of the coarser scale, carried
    through the steps that follow.  The body-force channel keeps every stored
    value normal (measured: bit for bit); the pressure channel and the random
    medium differ in 0.03% of the values, by at most 32 quanta of 2^-44."""
    case = make()
    steps = 240
    plain = Lattice(case.eps, case.k, case.kn0, device=dev, storage="f16", check_every=0,
                    **case.params)
    checked = Lattice(case.eps, case.k, case.kn0, device=dev, storage="f16", check_every=60,
                      **case.params)
    e0 = _scale_exp(plain)
    plain.step(steps)
    checked.step(steps)
    e_plain, e_checked = _scale_exp(plain), _scale_exp(checked)
    assert e_plain == e0 and e_checked != e0, (e0, e_plain, e_checked)
    fa, fb = plain.populations(), checked.populations()
    diff = float((fa - fb).abs().max())
    same = float((fa == fb).double().mean())
    print(f"{case.name}: e {e0} -> {e_checked}, max |df| {diff:.3e}, identical {same:.6f}")
    quantum = 2.0 ** (-24 - min(e0, e_checked))
    bound = 0.0 if exact else steps * 16 * quantum
    assert diff <= bound
    # FP32 read-outs: the same bound, plus one rounding of the FP32 result
    slack = 0.0 if exact else 2.0 ** -23
    for a, b in zip(plain.macroscopic(), checked.macroscopic()):
        assert bool(torch.all((a - b).abs() <= bound + slack * a.abs()))


def test_pressure_columns_with_porosity_contrast(dev):
    """End columns whose porosity differs from their neighbours' (0.45 next
    to 0.95 at the inlet, 0.5 next to 1.0 at the outlet) in a nearly free
    fluid (k = 50), with walls: the extrapolation's equilibrium term takes
    the column's own porosity.  Taking the neighbour's there instead moves
    this velocity field by 3.8e-4 relative L2 in the oracle (measured with
    that change planted), 38 times the parity bound, so this case fixes the
    choice on the HIP path too.  Two 256-wide blocks and a ragged tail."""
    rng = np.random.default_rng(5)
    nx, ny = 300, 16
    col = rng.uniform(0.4, 1.0, nx)
    col[0], col[1], col[-2], col[-1] = 0.45, 0.95, 1.0, 0.5
    eps = np.tile(col, (ny, 1)).astype(np.float32)
    k = np.full((ny, nx), 50.0, np.float32)
    params = inputs.run_params(tau=0.8, bc_x=inputs.PRESSURE, bc_y=inputs.WALL, rho_in=1.01,
                               rho_out=1.0, init=1)
    case = inputs.Case(eps, k, np.zeros_like(eps), params, "porosity-contrast")
    compare(gpu_run(dev, case, 400), oracle_run(case, 400))


def test_diagnostics(dev):
    """lbk_diagnostics: the mass is the FP64 sum of the populations; the
    x mass flux is sum rho u_x; the residual is ||u - u_prev|| / ||u|| over
    the velocities read out at this call and the previous one (+inf on the
    first call, 0 with no step in between), and 0 for a lattice whose
    velocity stays zero (at rest, no drive)."""
    case = inputs.random_medium(300, 20, seed=31, bc_x=inputs.PRESSURE, bc_y=inputs.WALL,
                                rho_in=1.01, rho_out=1.0, init=1)
    lat = gpu_run(dev, case, 50)
    m, q, r = lat.diagnostics()
    assert math.isinf(r)
    f = lat.populations().cpu().numpy()
    assert m == pytest.approx(float(f.sum()), rel=1e-12)
    rho, ux, uy = macro_np(lat)
    assert q == pytest.approx(float((rho * ux).sum()), rel=1e-6)
    assert lat.diagnostics()[2] == 0.0
    lat.step(10)
    _, _, r2 = lat.diagnostics()
    _, ux2, uy2 = macro_np(lat)
    want = math.sqrt((((ux2 - ux) ** 2).sum() + ((uy2 - uy) ** 2).sum()) /
                     ((ux2 ** 2).sum() + (uy2 ** 2).sum()))
    assert 0 < r2 == pytest.approx(want, rel=1e-9)
    rest = Lattice(case.eps, case.k, case.kn0, device=dev)  # periodic, no drive, rest
    rest.step(5)
    rest.diagnostics()
    rest.step(5)
    assert rest.diagnostics()[2] == 0.0


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16", 2e-3)])
def test_residual_against_oracle(dev, storage, tol):
    """The steady-state residual of lbk_diagnostics against the oracle's
    (R13): ||u(200) - u(100)|| / ||u(200)|| on a heterogeneous
    pressure-driven lattice with walls, free-fluid and impermeable nodes,
    m = 100 steps apart (even, so the alternating stiff mode cancels)."""
    case = inputs.random_medium(300, 21, seed=33, solid_frac=0.05, pore_frac=0.05,
                                bc_x=inputs.PRESSURE, bc_y=inputs.WALL, rho_in=1.01,
                                rho_out=1.0, init=1)
    lat = gpu_run(dev, case, 100, storage=storage)
    lat.diagnostics()
    lat.step(100)
    _, _, r = lat.diagnostics()
    ref = oracle_run(case, 100)
    u_prev = ref.macro()[1:]
    ref.step(100)
    rr = oracle.residual(ref.macro()[1:], u_prev)
    print(f"residual {storage}: HIP {r:.9e}, oracle {rr:.9e}", flush=True)
    assert 0.0 < rr < 1.0
    assert abs(r / rr - 1) < tol


def test_permeability_needs_a_drive(dev):
    """The global permeability is normalised by the drive: without one
    (equal pressure-column densities, or no body force along x) the call is
    refused, in 2-D and 3-D, and a batch reports NaN for such a sample."""
    from paper_1411_7051_amd._lib import LbkError
    from paper_1411_7051_amd.batch import Batch
    from paper_1411_7051_amd.lattice3 import Lattice3
    eps, k = np.full((6, 40), 0.5, np.float32), np.full((6, 40), 0.1, np.float32)
    flat = Lattice(eps, k, None, device=dev, bc_x=inputs.PRESSURE, rho_in=1.0, rho_out=1.0)
    side = Lattice(eps, k, None, device=dev, gy=1e-5)
    good = Lattice(eps, k, None, device=dev, gx=1e-5)
    for lat in (flat, side):
        lat.step(3)
        with pytest.raises(LbkError) as e:
            lat.apparent_permeability()
        assert e.value.status == -1
        with pytest.raises(LbkError):
            lat.gradient(4, "k_app", ckpt_every=2)
    good.step(3)
    kb = Batch([good, side]).apparent_permeability()
    assert kb[0] == good.apparent_permeability() and math.isnan(kb[1])
    e3, k3 = np.full((3, 4, 40), 0.5, np.float32), np.full((3, 4, 40), 0.1, np.float32)
    flat3 = Lattice3(e3, k3, None, device=dev, bc_x=inputs.PRESSURE, rho_in=1.0, rho_out=1.0)
    with pytest.raises(LbkError) as e:
        flat3.apparent_permeability()
    assert e.value.status == -1
