"""The HIP adjoint sweep (through the C ABI) against finite differences of the
FP64 oracle: dJ/d ln k after N steps, for the global permeability and the
outlet flux, on heterogeneous media with free-fluid and impermeable nodes and
every boundary combination; plus properties that hold at any size."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1411_7051_amd import inputs
from paper_1411_7051_amd.lattice import ApparentPermeability, Lattice

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3  # FP32 linearisation vs FP64 FD: per node, relative to |fd|,
NODE_FLOOR = 0.1  # on every sampled node with |fd| >= NODE_FLOOR max|g|; and
                  # on every sampled node, relative to max|g|


def check_fd(gg, fd, scale, what=""):
    """The adjoint at the sampled nodes against finite differences: within
    GRAD_TOL of |fd| at each node whose |fd| is at least NODE_FLOOR of the
    largest gradient, and within GRAD_TOL of the largest gradient at every
    sampled node.  Prints the worst per-node relative error."""
    gg, fd = np.asarray(gg, dtype=np.float64), np.asarray(fd, dtype=np.float64)
    assert scale > 0
    err = np.abs(gg - fd)
    big = np.abs(fd) >= NODE_FLOOR * scale
    assert big.any()
    rel = err[big] / np.abs(fd[big])
    print(f"{what}: worst per-node relative error {rel.max():.2e} over {int(big.sum())} "
          f"nodes with |fd| >= {NODE_FLOOR} max|g|; worst error / max|g| "
          f"{err.max() / scale:.2e}", flush=True)
    assert rel.max() <= GRAD_TOL, f"{what}: per-node relative error {rel.max():.3e}"
    assert err.max() <= GRAD_TOL * scale, f"{what}: max |adjoint - fd| = {err.max():.3e}, " \
        f"scale {scale:.3e}"


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda", 0)
    torch.cuda.set_device(d)
    return d


def drive_for(bcx):
    if bcx == inputs.PRESSURE:
        return dict(rho_in=1.02, rho_out=1.0, init=1)
    return dict(gx=2e-5, gy=-5e-6)


CASES = [(0, 0, "k_app"), (0, 1, "k_app"), (1, 1, "k_app"), (2, 0, "k_app"), (2, 1, "k_app"),
         (2, 0, "q_out"), (2, 1, "q_out"), (0, 1, "q_out")]


@pytest.mark.parametrize("bcx,bcy,obj", CASES)
def test_gradient_matches_oracle_fd(dev, bcx, bcy, obj):
    nx, ny, N = 40, 12, 25
    case = inputs.random_medium(nx, ny, seed=300 + 7 * bcx + bcy, solid_frac=0.06,
                                pore_frac=0.06, bc_x=bcx, bc_y=bcy, **drive_for(bcx))
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J, g = lat.gradient(N, obj, ckpt_every=10, hist_len=4)
    g = g.double().cpu().numpy()
    ref = oracle.Lattice(case.eps, case.k, case.kn0, **case.params).step(N)
    Jr = oracle.objective(ref, obj)
    assert abs(J / Jr - 1) < 1e-5
    rng = np.random.default_rng(1)
    finite = np.isfinite(case.k) & (case.eps > 0)
    # nodes with the largest gradients plus random ones
    order = np.argsort(-np.abs(g).ravel())
    cand = [divmod(int(i), nx) for i in order[:6]]
    ys, xs = np.nonzero(finite)
    pick = rng.choice(len(ys), 6, replace=False)
    cand += [(int(ys[i]), int(xs[i])) for i in pick]
    cand = [c for c in cand if finite[c]]
    fd = oracle.fd_gradient(case.eps, case.k, case.kn0, N, cand, obj, h=1e-4, **case.params)
    gg = np.array([g[c] for c in cand])
    check_fd(gg, fd, np.max(np.abs(g)), f"d{obj}/dlnk bc ({bcx},{bcy})")
    # pores (k = inf) and impermeable nodes have no permeability to vary
    assert np.all(g[~finite] == 0.0)


@pytest.mark.parametrize("bcx,bcy,obj,kn_local,rho_ref",
                         [(2, 1, "k_app", 1, 1.0), (2, 0, "q_out", 1, 1.0),
                          (0, 1, "k_app", 1, 1.0), (2, 1, "k_app", 0, 1.0),
                          (2, 1, "k_app", 1, 2.0), (0, 0, "k_app", 1, 0.5)])
def test_kn0_gradient_matches_oracle_fd(dev, bcx, bcy, obj, kn_local, rho_ref):
    """dJ / d ln kn0 (k held fixed) against oracle finite differences in ln
    kn0; asking for it leaves dJ / d ln k bitwise unchanged.  With kn0
    quoted at rho_ref != 1 (Kn = kn0 rho_ref / rho, whose density
    derivative enters every reverse step), dJ / d ln k is checked against
    finite differences too."""
    nx, ny, N = 40, 12, 25
    case = inputs.random_medium(nx, ny, seed=330 + 7 * bcx + bcy + kn_local, solid_frac=0.05,
                                pore_frac=0.05, kn_range=(0.05, 3.0), bc_x=bcx, bc_y=bcy,
                                kn_local=kn_local, rho_ref=rho_ref, **drive_for(bcx))
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J, gk, gn = lat.gradient(N, obj, ckpt_every=10, hist_len=4, wrt_kn0=True)
    lat2 = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J2, gk2 = lat2.gradient(N, obj, ckpt_every=10, hist_len=4)
    assert J == J2 and torch.equal(gk, gk2)
    gn = gn.double().cpu().numpy()
    has = case.kn0 > 0
    assert np.all(gn[~has] == 0.0)
    order = np.argsort(-np.abs(gn).ravel())
    cand = [divmod(int(i), nx) for i in order[:6]]
    ys, xs = np.nonzero(has)
    pick = np.random.default_rng(2).choice(len(ys), 6, replace=False)
    cand += [(int(ys[i]), int(xs[i])) for i in pick]
    fd = oracle.fd_gradient(case.eps, case.k, case.kn0, N, cand, obj, h=1e-4, wrt="kn0",
                            **case.params)
    gg = np.array([gn[c] for c in cand])
    check_fd(gg, fd, np.max(np.abs(gn)), f"d{obj}/dlnkn0 rho_ref {rho_ref}")
    if rho_ref != 1.0:
        gk = gk.double().cpu().numpy()
        porous = np.isfinite(case.k) & (case.eps > 0)
        order = np.argsort(-np.abs(gk).ravel())
        cand = [c for c in (divmod(int(i), nx) for i in order[:8]) if porous[c]]
        fd = oracle.fd_gradient(case.eps, case.k, case.kn0, N, cand, obj, h=1e-4, wrt="k",
                                **case.params)
        check_fd(np.array([gk[c] for c in cand]), fd, np.max(np.abs(gk)),
                 f"d{obj}/dlnk rho_ref {rho_ref}")


@pytest.mark.parametrize("corr,slip_b", [(1, -1.0), (0, -0.3), (2, -1.0)])
def test_gradient_correlations(dev, corr, slip_b):
    """Both gradient planes with the first-order correlation, a different
    slip coefficient and no correction, against oracle finite differences
    (no correction: the ln kn0 plane is exactly zero)."""
    nx, ny, N = 36, 10, 20
    case = inputs.random_medium(nx, ny, seed=360 + corr, solid_frac=0.05, pore_frac=0.05,
                                kn_range=(0.05, 3.0), bc_x=2, bc_y=1, rho_in=1.02,
                                rho_out=1.0, init=1, correlation=corr, slip_b=slip_b)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    _, gk, gn = lat.gradient(N, "k_app", ckpt_every=8, hist_len=3, wrt_kn0=True)
    for g, wrt in ((gk, "k"), (gn, "kn0")):
        g = g.double().cpu().numpy()
        if corr == 2 and wrt == "kn0":
            assert np.all(g == 0.0)
            continue
        order = np.argsort(-np.abs(g).ravel())
        cand = [divmod(int(i), nx) for i in order[:5]]
        fd = oracle.fd_gradient(case.eps, case.k, case.kn0, N, cand, "k_app", h=1e-4, wrt=wrt,
                                **case.params)
        check_fd(np.array([g[c] for c in cand]), fd, np.max(np.abs(g)),
                 f"correlation {corr} b {slip_b} wrt ln {wrt}")


def test_whole_field_small(dev):
    """Every node of a 10x6 pressure-driven lattice against oracle FD."""
    nx, ny, N = 10, 6, 12
    case = inputs.random_medium(nx, ny, seed=41, bc_x=2, bc_y=1, rho_in=1.05, rho_out=1.0,
                                init=1)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    _, g = lat.gradient(N, "k_app", ckpt_every=5, hist_len=5)
    g = g.double().cpu().numpy()
    nodes = [(y, x) for y in range(ny) for x in range(nx)]
    fd = oracle.fd_gradient(case.eps, case.k, case.kn0, N, nodes, "k_app", h=1e-4,
                            **case.params).reshape(ny, nx)
    check_fd(g.ravel(), fd.ravel(), np.max(np.abs(g)), "whole 10x6 field")


def test_light_cone(dev):
    """The outlet flux after N steps cannot depend on k further than N + 1
    links from the outlet column: exact zeros there."""
    nx, ny, N = 64, 8, 10
    case = inputs.random_medium(nx, ny, seed=42, bc_x=2, rho_in=1.01, rho_out=1.0, init=1)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    _, g = lat.gradient(N, "q_out", ckpt_every=N)
    g = g.cpu().numpy()
    far = g[:, : nx - 1 - (N + 1)]
    assert np.all(far == 0.0)
    assert np.any(g[:, nx - 3:] != 0.0)


def test_checkpoint_schemes_agree(dev):
    """One-level, two-level and different intervals replay the same forward
    trajectory (J bitwise identical); the gradients differ only by the FP32
    rounding of the per-segment accumulation."""
    case = inputs.random_medium(300, 20, seed=43, solid_frac=0.05, bc_x=2, rho_in=1.01,
                                rho_out=1.0, init=1)
    out = []
    for ck, hl in [(60, 60), (60, 7), (13, 13), (200, 50)]:
        lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
        J, g = lat.gradient(120, "k_app", ckpt_every=ck, hist_len=hl)
        assert lat.time == 120
        out.append((J, g))
    ref = out[0][1]
    scale = float(ref.abs().max())
    for J, g in out[1:]:
        assert J == out[0][0]
        assert float((g - ref).abs().max()) <= 1e-5 * scale


def test_adjoint_plan_fits_budget(dev):
    """The planner returns a plan whose workspace fits (the one-level plan
    when it fits, since it rebuilds nothing), and the gradient with that
    plan equals the one-level gradient."""
    from paper_1411_7051_amd._lib import LbkError
    case = inputs.random_medium(200, 16, seed=47, bc_x=2, rho_in=1.01, rho_out=1.0, init=1)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    full = lat.adjoint_workspace_bytes(90, 30, 30)
    assert lat.adjoint_plan(90, 30, budget=full) == 30
    h = lat.adjoint_plan(90, 30, budget=full - 1)
    assert h < 30 and lat.adjoint_workspace_bytes(90, 30, h) <= full - 1
    with pytest.raises(LbkError) as e:
        lat.adjoint_plan(90, 30, budget=1000)
    assert e.value.status == -3
    J1, g1 = lat.gradient(90, "k_app", ckpt_every=30, hist_len=h)
    lat2 = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J2, g2 = lat2.gradient(90, "k_app", ckpt_every=30, hist_len=30)
    assert J1 == J2
    assert float((g1 - g2).abs().max()) <= 1e-5 * float(g2.abs().max())


def test_kept_inner_checkpoints(dev):
    """A workspace larger than the minimum keeps the inner checkpoints of
    more trailing segments (none rebuilt when all fit): the gradient is
    bitwise the same, since the kept states are those the backward pass
    would recompute.  The planner spends extra budget on kept segments."""
    case = inputs.random_medium(150, 12, seed=49, solid_frac=0.05, bc_x=2, rho_in=1.01,
                                rho_out=1.0, init=1)
    steps, ck, hl = 100, 25, 6
    out = []
    for extra_segments in (0, 1, 3, 10):
        lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
        base = lat.adjoint_workspace_bytes(steps, ck, hl)
        seg = lat.state_bytes() * -(-ck // hl)
        ws = torch.empty(base + extra_segments * seg, dtype=torch.uint8, device=dev)
        J, ws = lat.adjoint_forward(steps, "k_app", ck, hl, ws)
        g = lat.adjoint_backward(ws)
        out.append((J, g))
    for J, g in out[1:]:
        assert J == out[0][0]
        assert torch.equal(g, out[0][1])
    # one-level (history of 50 steps) does not fit, two-level with every
    # segment's inner checkpoints kept does: the planner finds the latter
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    budget = lat.adjoint_workspace_bytes(100, 50, 10) + 5 * lat.state_bytes()
    assert lat.adjoint_workspace_bytes(100, 50, 50) > budget
    h, nbytes = lat.adjoint_plan(100, 50, budget=budget, with_bytes=True)
    assert h < 50 and nbytes <= budget
    assert nbytes >= lat.adjoint_workspace_bytes(100, 50, h) + lat.state_bytes() * (-(-50 // h)) - 256
    J1, ws = lat.adjoint_forward(100, "k_app", 50, h, torch.empty(nbytes, dtype=torch.uint8,
                                                                  device=dev))
    g1 = lat.adjoint_backward(ws)
    lat2 = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J2, g2 = lat2.gradient(100, "k_app", ckpt_every=50, hist_len=50)
    assert J1 == J2
    assert float((g1 - g2).abs().max()) <= 1e-5 * float(g2.abs().max())


def test_taylor_remainder(dev):
    """J(ln k + h d) - J(ln k) - h <g, d> shrinks like h^2 (GPU, FP32)."""
    case = inputs.random_medium(96, 24, seed=44, bc_x=2, bc_y=1, rho_in=1.02, rho_out=1.0,
                                init=1, k_range=(0.05, 1.0))
    N = 60
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J0, g = lat.gradient(N, "k_app", ckpt_every=N)
    g = g.double().cpu().numpy()
    rng = np.random.default_rng(5)
    d = rng.standard_normal(case.k.shape)
    lnk = np.log(case.k.astype(np.float64))
    rems = []
    for h in (0.2, 0.1, 0.05):
        kk = np.exp(lnk + h * d).astype(np.float32)
        l2 = Lattice(case.eps, kk, case.kn0, device=dev, **case.params).step(N)
        Jh = l2.apparent_permeability()
        rems.append(abs(Jh - J0 - h * float(np.sum(g * d))))
    assert rems[0] / rems[1] > 3.0 and rems[1] / rems[2] > 3.0


def test_autograd_function(dev):
    case = inputs.random_medium(70, 16, seed=45, bc_x=2, rho_in=1.01, rho_out=1.0, init=1)
    log_k = torch.log(torch.from_numpy(case.k.astype(np.float64))).to(dev).requires_grad_(True)
    params = dict(case.params, ckpt_every=20, hist_len=5)
    J = ApparentPermeability.apply(log_k, torch.from_numpy(case.eps), torch.from_numpy(case.kn0),
                                   50, params)
    (gk,) = torch.autograd.grad(3.0 * J, log_k)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J2, g2 = lat.gradient(50, "k_app", ckpt_every=20, hist_len=5)
    assert float(J.detach()) == J2
    assert torch.allclose(gk.float(), 3.0 * g2, rtol=1e-6, atol=0)


@pytest.mark.parametrize("bcx,bcy,obj", [(0, 1, "k_app"), (2, 0, "k_app"), (2, 1, "q_out")])
def test_gradient_forchheimer(dev, bcx, bcy, obj):
    """With the Forchheimer term of Eq. 2 (F_eps = 0.8) on a permeable,
    fast-flowing medium (B |u| comparable to A), dJ/d ln k and dJ/d ln kn0
    through the quadratic velocity solve against oracle finite
    differences."""
    nx, ny, N = 40, 12, 25
    drive = (dict(rho_in=1.05, rho_out=1.0, init=1) if bcx == inputs.PRESSURE
             else dict(gx=4e-4, gy=-1e-4))
    case = inputs.random_medium(nx, ny, seed=470 + bcx + bcy, eps_range=(0.4, 0.9),
                                k_range=(0.5, 20.0), kn_range=(0.0, 1.0), solid_frac=0.05,
                                pore_frac=0.05, f_eps=0.8, bc_x=bcx, bc_y=bcy, **drive)
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J, gk, gn = lat.gradient(N, obj, ckpt_every=10, hist_len=4, wrt_kn0=True)
    ref = oracle.Lattice(case.eps, case.k, case.kn0, **case.params).step(N)
    assert abs(J / oracle.objective(ref, obj) - 1) < 1e-5
    # the term matters here: B |u| against A over the porous nodes
    _, ux, uy = ref.macro()
    porous = np.isfinite(case.k) & (case.eps > 0)
    nu = (case.params["tau"] - 0.5) / 3.0
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = (case.eps * 0.8 / np.sqrt(case.k)) * np.hypot(ux, uy) / (case.eps * nu / case.k)
    assert np.max(ratio[porous]) > 0.05
    for g, wrt, mask in [(gk, "k", porous), (gn, "kn0", case.kn0 > 0)]:
        g = g.double().cpu().numpy()
        order = np.argsort(-np.abs(g).ravel())
        cand = [divmod(int(i), nx) for i in order[:6]]
        ys, xs = np.nonzero(mask)
        pick = np.random.default_rng(3).choice(len(ys), 6, replace=False)
        cand += [(int(ys[i]), int(xs[i])) for i in pick]
        cand = [c for c in cand if mask[c]]
        fd = oracle.fd_gradient(case.eps, case.k, case.kn0, N, cand, obj, h=1e-4, wrt=wrt,
                                **case.params)
        gg = np.array([g[c] for c in cand])
        check_fd(gg, fd, np.max(np.abs(g)), f"Forchheimer {obj} wrt ln {wrt}")


def test_fullsize_shale_against_windowed_oracle_fd(dev, shale8192):
    """Fractured shale matrix at its full 8192 x 8192 size: the adjoint
    gradient of the outlet flux after 200 steps, at 16 seeded nodes with
    |g| > 1e-3 max|g|, against FP64 central differences of the oracle
    (h = 1e-4 in ln k), each computed on the window of the medium that the
    perturbation and the outlet rows it reaches depend on (the light cone
    of 200 steps; the rest of the flux cancels in the difference).  Bar:
    per node, |adjoint - fd| <= 1e-3 |fd|."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle_window import window_fd_outlet_flux

    case = shale8192
    steps = 200
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    _, g = lat.gradient(steps, "q_out", ckpt_every=100, hist_len=100)
    g = g.double().cpu().numpy()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    gmax = np.abs(g).max()
    cand = np.argwhere(np.abs(g) > 1e-3 * gmax)
    pick = cand[np.random.default_rng(16).choice(len(cand), 16, replace=False)]
    # the oracle runs in C through ctypes, which releases the GIL
    with ThreadPoolExecutor(max_workers=8) as ex:
        fd = np.array(list(ex.map(lambda yx: window_fd_outlet_flux(case, int(yx[0]), int(yx[1]),
                                                                    steps), pick)))
    gg = np.array([g[y, x] for y, x in pick])
    rel = np.abs(gg - fd) / np.abs(fd)
    for (y, x), a, b, e in zip(pick, gg, fd, rel):
        print(f"node ({y}, {x}): adjoint {a:.6e}, oracle fd {b:.6e}, rel {e:.2e}", flush=True)
    print(f"shale 8192^2, 200 steps: worst per-node relative error {rel.max():.2e}", flush=True)
    assert rel.max() <= GRAD_TOL


def test_fullsize_shale_20000_steps_directional(dev, shale8192):
    """The gradient run of the benchmark configuration: global permeability
    of the 8192 x 8192 shale after 20,000 steps, checkpoints every 500, the
    planner's history length and kept segments.  The whole gradient field is
    checked at once through a directional derivative: <g, d> for a smooth
    random direction d (Gaussian field, correlation length 64, scaled to
    max |d| = 1) against a central difference of the HIP forward pass along
    d (ln k +- h d, h = 0.01; truncation O(h^2) ~ 1e-4 relative).  Bar: 1e-3
    relative."""
    case = shale8192
    steps, ck, h = 20000, 500, 0.01
    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J0, g = lat.gradient(steps, "k_app", ckpt_every=ck, hist_len="auto")
    g = g.double().cpu().numpy()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ny, nx = case.k.shape
    d = inputs.gaussian_field(ny, nx, 64.0, np.random.default_rng(20000))
    d /= np.abs(d).max()
    vals = []
    for sgn in (1.0, -1.0):
        kk = (case.k.astype(np.float64) * np.exp(sgn * h * d)).astype(np.float32)
        l2 = Lattice(case.eps, kk, case.kn0, device=dev, **case.params).step(steps)
        vals.append(l2.apparent_permeability())
        l2.close()
        del l2
        torch.cuda.empty_cache()
    fd = (vals[0] - vals[1]) / (2 * h)
    dot = float((g * d).sum())
    print(f"20000-step gradient: <g, d> = {dot:.6e}, central difference = {fd:.6e}, "
          f"relative difference {abs(fd - dot) / abs(dot):.2e}", flush=True)
    assert abs(fd - dot) <= 1e-3 * abs(dot), (fd, dot, J0)


def test_backward_refuses_a_stale_forward(dev):
    """lbk_adjoint_backward differentiates the last lbk_adjoint_forward on the
    same workspace with the lattice where that forward left it: a backward
    with no forward, another workspace, or a step in between are rejected
    (status LBK_ERR_INVALID_ARG) without touching the state; the forward's
    own workspace then still gives the gradient of an undisturbed run."""
    from paper_1411_7051_amd._lib import LbkError
    case = inputs.random_medium(40, 12, seed=902, bc_x=inputs.PRESSURE, bc_y=inputs.WALL,
                                rho_in=1.02, rho_out=1.0, init=1)
    ref = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    J_ref, ws_ref = ref.adjoint_forward(30, "k_app", 10, 10)
    g_ref = ref.adjoint_backward(ws_ref)

    lat = Lattice(case.eps, case.k, case.kn0, device=dev, **case.params)
    other = torch.empty(lat.adjoint_workspace_bytes(30, 10, 10), dtype=torch.uint8,
                        device=dev)
    with pytest.raises(LbkError) as e:
        lat.adjoint_backward(other)  # no forward yet
    assert e.value.status == -1
    J, ws = lat.adjoint_forward(30, "k_app", 10, 10)
    s30 = lat.save_state().clone()
    with pytest.raises(LbkError) as e:
        lat.adjoint_backward(other)  # not the forward's workspace
    assert e.value.status == -1
    assert torch.equal(lat.save_state(), s30)
    g = lat.adjoint_backward(ws)  # still valid after the refusals
    assert J == J_ref and torch.equal(g, g_ref)
    lat.step(1)
    with pytest.raises(LbkError) as e:
        lat.adjoint_backward(ws)  # the lattice moved since the forward
    assert e.value.status == -1
    assert lat.time == 31
