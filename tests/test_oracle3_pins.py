"""Pins for the D3Q19 form of the FP64 oracle, against what the paper's
model and the lattice fix rather than the oracle's own formulas: the
isotropy conditions that define the D3Q19 set, the moment conditions of
Eqs. 14-15 with three-component vectors, the uniform-medium recurrence
(Darcy limit) for a force along an arbitrary direction, mass conservation,
the Brinkman channel of Eq. 20 and the compressible Klinkenberg-Darcy
column (CPU)."""
import itertools
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle

CS2 = 1.0 / 3.0


def _fields(nz, ny, nx, eps, k, kn0=0.0):
    s = (nz, ny, nx)
    return np.full(s, eps), np.full(s, k), np.full(s, kn0)


def test_d3q19_set_and_isotropy():
    ex, ey, ez, w = oracle.tables3()
    E = np.stack([ex, ey, ez], axis=1).astype(float)
    n2 = (E ** 2).sum(1)
    # rest, six axis links, twelve face diagonals; no cube corners
    assert sorted(n2) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(e) for e in E.astype(int)}) == 19
    assert math.isclose(w.sum(), 1.0, rel_tol=1e-15)
    d = np.eye(3)
    # odd moments vanish, second moment cs^2 delta, fourth moment cs^4 (dd + dd + dd)
    assert np.allclose(np.einsum("i,ia->a", w, E), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, E, E), CS2 * d, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, E, E, E), 0, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, E, E, E, E)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) +
                      np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(m4, iso, atol=1e-15)


@pytest.mark.parametrize("eps", [1.0, 0.6, 0.15])
def test_equilibrium_and_forcing_moments(eps):
    """Eq. 14: density, momentum, momentum flux cs^2 rho I + rho u u / eps;
    Eq. 15 (Guo): 0, (1 - 1/2tau) rho F, (1 - 1/2tau) rho (uF + Fu)/eps."""
    ex, ey, ez, _ = oracle.tables3()
    E = np.stack([ex, ey, ez], axis=1).astype(float)
    rng = np.random.default_rng(1)
    for _ in range(10):
        rho, tau = rng.uniform(0.5, 1.5), rng.uniform(0.55, 2.0)
        u = rng.uniform(-0.05, 0.05, 3)
        F = rng.uniform(-1e-3, 1e-3, 3)
        f = oracle.feq3(rho, u, eps)
        assert math.isclose(f.sum(), rho, rel_tol=1e-14)
        assert np.allclose(E.T @ f, rho * u, atol=1e-15)
        assert np.allclose(np.einsum("ia,ib,i->ab", E, E, f),
                           CS2 * rho * np.eye(3) + rho * np.outer(u, u) / eps, atol=1e-14)
        Fi = oracle.guo3(rho, u, F, eps, tau)
        c = 1 - 1 / (2 * tau)
        assert abs(Fi.sum()) < 1e-18
        assert np.allclose(E.T @ Fi, c * rho * F, atol=1e-18)
        assert np.allclose(np.einsum("ia,ib,i->ab", E, E, Fi),
                           c * rho * (np.outer(u, F) + np.outer(F, u)) / eps, atol=1e-18)


@pytest.mark.parametrize("eps,k,kn0", [(0.5, 1.0, 0.0), (0.3, 0.2, 0.4)])
def test_uniform_recurrence_and_darcy_limit(eps, k, kn0):
    """Uniform periodic medium: j_{n+1} = j_n + rho F_n exactly, so
    u_{n+1} = q u_n + eps G / (1 + A/2), q = (1 - A/2)/(1 + A/2), with the
    fixed point k_a G / nu (Darcy), for G along an arbitrary direction."""
    tau, nu = 0.8, 0.1
    G = np.array([1e-5, -4e-6, 7e-6])
    lat = oracle.Lattice3(*_fields(3, 4, 5, eps, k, kn0), tau=tau, gx=G[0], gy=G[1], gz=G[2])
    A = eps * nu / (k * oracle.fc(kn0))
    q, b = (1 - A / 2) / (1 + A / 2), eps / (1 + A / 2)
    u = 0.5 * b * G
    for _ in range(60):
        _, ux, uy, uz = lat.macro()
        assert np.allclose([ux.mean(), uy.mean(), uz.mean()], u, rtol=1e-10, atol=0)
        assert np.ptp(ux) < 1e-18
        lat.step(1)
        u = q * u + b * G
    ustar = k * oracle.fc(kn0) * G / nu
    assert np.allclose(b * G / (1 - q), ustar, rtol=1e-12)


def test_mass_conservation_with_walls():
    """Streaming, bounce-back and collision conserve mass: the FP64 total
    moves only by the round-off of the sums (about 1e-13 after 300 steps
    here, the same with and without walls)."""
    rng = np.random.default_rng(2)
    s = (6, 7, 9)
    eps = rng.uniform(0.2, 1.0, s)
    k = np.exp(rng.uniform(np.log(0.05), 0.0, s))
    kn0 = rng.uniform(0, 1, s)
    lat = oracle.Lattice3(eps, k, kn0, gx=1e-4, gy=2e-5, gz=-3e-5, bc_y=oracle.WALL,
                          bc_z=oracle.WALL)
    m0 = lat.mass()
    lat.step(300)
    assert abs(lat.mass() - m0) / m0 < 1e-12


def _brinkman(y, H, G, K, eps, nu):
    a = math.sqrt(eps / K)
    return G * K / nu * (1 - np.cosh(a * (y - H / 2)) / np.cosh(a * H / 2))


def test_brinkman_channel():
    """Plates normal to y (walls), periodic in x and z: the steady profile is
    Eq. 20, uniform in x and z; the channel permeability k (1 - tanh(aH/2)/
    (aH/2))."""
    H, eps, k, G, nu = 32, 0.5, 1.024, 1e-6, 0.1
    lat = oracle.Lattice3(*_fields(2, H, 3, eps, k), tau=0.8, gx=G, bc_y=oracle.WALL)
    lat.step(10000)
    _, ux, uy, uz = lat.macro()
    ua = _brinkman(np.arange(H) + 0.5, H, G, k, eps, nu)
    prof = ux[0, :, 0]
    assert abs(0.5 * (prof[15] + prof[16]) / _brinkman(np.array([H / 2]), H, G, k, eps, nu)[0]
               - 1) < 1e-4
    assert np.linalg.norm(prof - ua) / np.linalg.norm(ua) < 1e-2
    assert np.all(ux == ux[:1, :, :1])
    assert max(np.abs(uy).max(), np.abs(uz).max()) < 1e-9 * np.abs(ux).max()
    a = math.sqrt(eps / k)
    kg = k * (1 - math.tanh(a * H / 2) / (a * H / 2))
    assert abs(lat.apparent_permeability() / kg - 1) < 5e-3


def test_klinkenberg_darcy_column():
    """Pressure planes with a 2:1 density ratio in a uniform medium with local
    Kn: k_app = k / (rho_in - rho_out) int f_c(kn0 / rho) d rho."""
    k, kn0 = 0.01, 0.5
    lat = oracle.Lattice3(*_fields(2, 1, 40, 0.5, k, kn0), tau=0.8, bc_x=oracle.PRESSURE,
                          rho_in=2.0, rho_out=1.0, init=1).step(25000)
    integral = quad(lambda r: oracle.fc(kn0 / r), 1.0, 2.0, epsabs=1e-13)[0]
    assert abs(lat.apparent_permeability() / k / integral - 1) < 2e-3


@pytest.mark.parametrize("kn_local,rho_ref", [(0, 2.0), (1, 0.5), (1, 2.0)])
def test_klinkenberg_darcy_column_kn_reference(kn_local, rho_ref):
    """Where Kn is evaluated (Eq. 5 with Eq. 10), in three dimensions: with Kn
    held at kn0 the drag is uniform and k_app = k f_c(kn0) whatever rho_ref;
    with a local Kn quoted at rho_ref, k_app = k (1/(rho_in - rho_out))
    int f_c(kn0 rho_ref / rho) d rho.  The alternatives (local where it
    should be global, rho_ref dropped) miss by far more than the tolerance."""
    k, kn0 = 0.01, 0.5
    lat = oracle.Lattice3(*_fields(2, 1, 40, 0.5, k, kn0), tau=0.8, bc_x=oracle.PRESSURE,
                          rho_in=2.0, rho_out=1.0, init=1, kn_local=kn_local,
                          rho_ref=rho_ref).step(25000)
    ratio = lat.apparent_permeability() / k

    def column(scale):
        return quad(lambda r: oracle.fc(kn0 * scale / r), 1.0, 2.0, epsabs=1e-13)[0]

    want = oracle.fc(kn0) if kn_local == 0 else column(rho_ref)
    assert abs(ratio / want - 1) < 2e-3
    for w in ([column(1.0), column(rho_ref)] if kn_local == 0 else
              [column(1.0), oracle.fc(kn0), oracle.fc(kn0 * rho_ref)]):
        assert abs(ratio / w - 1) > 1e-2


def test_rejects_invalid():
    with pytest.raises(ValueError):
        oracle.Lattice3(*_fields(2, 2, 2, 1.5, 1.0))
    with pytest.raises(ValueError):
        oracle.Lattice3(*_fields(2, 2, 2, 0.5, 1.0), bc_z=2)


@pytest.mark.parametrize("bc_y,bc_z", [(oracle.PERIODIC, oracle.PERIODIC),
                                       (oracle.WALL, oracle.WALL)])
def test_axis_permutation_symmetry(bc_y, bc_z):
    """The D3Q19 set is closed under swapping the y and z axes, and so is the
    model: a heterogeneous medium with its y and z axes swapped, and the
    force components swapped with them, gives the swapped flow.  A velocity
    or opposite-direction table inconsistent in one direction breaks this."""
    rng = np.random.default_rng(31)
    s = (5, 7, 9)  # nz, ny, nx
    eps = rng.uniform(0.3, 1.0, s)
    k = np.exp(rng.uniform(np.log(0.05), np.log(2.0), s))
    kn0 = rng.uniform(0.0, 1.0, s)
    eps[2, 3, 4], k[2, 3, 4] = 0.0, 1.0      # an impermeable node
    eps[1, 5, 2], k[1, 5, 2] = 1.0, np.inf   # a free-fluid node
    kw = dict(gx=2e-4, gy=5e-5, gz=-3e-5, bc_y=bc_y, bc_z=bc_z)
    a = oracle.Lattice3(eps, k, kn0, **kw).step(40)
    sw = lambda f: np.ascontiguousarray(np.swapaxes(f, 0, 1))
    kw2 = dict(gx=2e-4, gy=-3e-5, gz=5e-5, bc_y=bc_z, bc_z=bc_y)
    b = oracle.Lattice3(sw(eps), sw(k), sw(kn0), **kw2).step(40)
    ra, uxa, uya, uza = a.macro()
    rb, uxb, uyb, uzb = b.macro()
    scale = np.max(np.abs(uxa))
    for p, q in [(ra, rb), (uxa, uxb), (uya, uzb), (uza, uyb)]:
        assert np.max(np.abs(sw(p) - q)) <= 1e-12 * max(scale, 1.0)


def test_impermeable_node_is_infinite_drag_limit():
    """eps = 0 nodes behave as the limit k -> 0 of a permeable node (Sec.
    III: infinite drag; R7), whatever that node's porosity: a block of
    impermeable nodes and the same block with k = 1e-13 give the same
    populations."""
    rng = np.random.default_rng(8)
    s = (6, 7, 9)
    eps = rng.uniform(0.3, 1.0, s)
    k = np.exp(rng.uniform(np.log(0.05), np.log(2.0), s))
    kn0 = rng.uniform(0.0, 1.0, s)
    e0, k0 = eps.copy(), k.copy()
    e0[2:4, 2:5, 3:6] = 0.0
    k1 = k.copy()
    k1[2:4, 2:5, 3:6] = 1e-13
    kw = dict(gx=1e-4, gy=3e-5, gz=-2e-5, bc_y=oracle.WALL)
    a = oracle.Lattice3(e0, k0, kn0, **kw).step(200).state()
    b = oracle.Lattice3(eps, k1, kn0, **kw).step(200).state()
    assert np.max(np.abs(a - b)) < 1e-12


def test_pressure_plane_next_to_equilibrium_is_own_equilibrium():
    """The inlet/outlet scheme in three dimensions: a pressure plane takes its
    own equilibrium at the imposed density and the neighbour's velocity plus
    the neighbour's non-equilibrium part, so next to a neighbour whose pulled
    populations are an equilibrium, in free fluid without a body force, it
    holds exactly its own equilibrium after the step: density rho_b,
    momentum rho_b u and momentum flux cs^2 rho_b I + rho_b u u / eps_b with
    the plane's own porosity (moment conditions of Eq. 14)."""
    ex, ey, ez, _ = oracle.tables3()
    E = np.stack([ex, ey, ez], axis=1).astype(float)
    nz, ny, nx = 1, 1, 6
    eps_col = np.array([0.5, 1.0, 1.0, 0.8, 0.8, 0.6])
    eps = np.broadcast_to(eps_col, (nz, ny, nx)).copy()
    k = np.full((nz, ny, nx), np.inf)
    rho_in, rho_out, rho_n = 1.02, 0.99, 1.003
    u = np.array([0.04, -0.03, 0.02])
    lat = oracle.Lattice3(eps, k, None, tau=0.8, bc_x=oracle.PRESSURE, rho_in=rho_in,
                          rho_out=rho_out)
    f = np.empty((19, nz, ny, nx))
    for x in range(nx):
        f[:, 0, 0, x] = oracle.feq3(rho_n, u, 1.0 if x <= 2 else 0.8)
    lat.set_state(f)
    lat.step(1)
    g = lat.state()
    for x, rho_b in ((0, rho_in), (nx - 1, rho_out)):
        fb = g[:, 0, 0, x]
        assert math.isclose(fb.sum(), rho_b, rel_tol=1e-14)
        assert np.allclose(E.T @ fb, rho_b * u, rtol=0, atol=1e-15)
        pi = np.einsum("ia,ib,i->ab", E, E, fb)
        ref = CS2 * rho_b * np.eye(3) + rho_b * np.outer(u, u) / eps_col[x]
        assert np.allclose(pi, ref, rtol=0, atol=1e-15), (x, pi - ref)


def test_forchheimer_fixed_point():
    """Eq. 2 with the Forchheimer term in three dimensions: a uniform periodic
    medium driven along an arbitrary direction settles at a velocity parallel
    to G whose magnitude solves (nu/k_a)|u| + (F_eps/sqrt(k_a))|u|^2 = |G|."""
    eps, k, kn0, f_eps, tau = 0.6, 0.5, 0.3, 0.7, 0.9
    G = 1e-3 * np.array([0.6, -0.48, 0.64])  # |G| = 1e-3
    nu = (tau - 0.5) / 3
    lat = oracle.Lattice3(*_fields(2, 2, 2, eps, k, kn0), tau=tau, gx=G[0], gy=G[1], gz=G[2],
                          f_eps=f_eps)
    lat.step(3000)
    _, ux, uy, uz = lat.macro()
    ka = k * oracle.fc(kn0)
    a, b_, c = f_eps / math.sqrt(ka), nu / ka, -np.linalg.norm(G)
    s = (-b_ + math.sqrt(b_ * b_ - 4 * a * c)) / (2 * a)
    want = s * G / np.linalg.norm(G)
    for comp, w in zip((ux, uy, uz), want):
        assert np.allclose(comp, w, rtol=1e-10)
    # the Forchheimer term matters at this flow rate
    assert abs(s - ka * np.linalg.norm(G) / nu) / s > 1e-2


def test_pressure_planes_hold_their_density():
    """The extrapolation sets the end planes to f_eq(rho_b, u_n) + f(n) -
    f_eq(rho_n, u_n), whose sum is rho_b whatever the neighbour's state, and
    the collision conserves it: after every step the density of plane 0 is
    rho_in and of plane nx-1 rho_out, on a heterogeneous medium with walls."""
    rng = np.random.default_rng(42)
    nz, ny, nx = 4, 5, 11
    eps = rng.uniform(0.3, 1.0, (nz, ny, nx))
    k = np.exp(rng.uniform(np.log(0.01), np.log(1.0), (nz, ny, nx)))
    kn0 = rng.uniform(0.0, 2.0, (nz, ny, nx))
    lat = oracle.Lattice3(eps, k, kn0, bc_x=oracle.PRESSURE, bc_y=oracle.WALL, bc_z=oracle.WALL,
                          rho_in=1.03, rho_out=0.99, init=1)
    for _ in range(3):
        lat.step(7)
        rho = lat.state().sum(axis=0)
        assert np.allclose(rho[:, :, 0], 1.03, rtol=1e-14, atol=0)
        assert np.allclose(rho[:, :, -1], 0.99, rtol=1e-14, atol=0)
        assert np.max(np.abs(rho[:, :, 1:-1] - 1.0)) > 1e-4  # the interior moves
