"""Pins of the oracle's Smagorinsky stress with Mason's wall damping (§2.2,
eqs. t-ij-1963, nu-t, smag, smag-1), on the staggered differences of §2.4.

Each pin is a closed form or a structural property that a plausible mistake
breaks:
* linear shear u = a z: S13 = a/2 on interior w nodes, so tau_xz =
  -lambda0^2 a |a| there, and a quarter of that on the bottom w node, where
  the velocity below the grid is taken as 0 (a wrong stagger, a dropped
  factor 2 in |S| = sqrt(2 S:S) or in tau = -2 nu S fails it);
* Mason's damping: the stress ratio to the undamped one is
  1 / (1 + (lambda0 / (kappa (d + z0)))^2), exactly 1/2 where
  kappa (d + z0) = lambda0, and 0 where d + z0 <= 0;
* trigonometric fields: the periodic central difference of sin(a x) is
  cos(a x) sin(a dx) / dx exactly (S11, S12, S13 each alone, so |S| is
  sqrt(2) |S11|, 2 |S12|, 2 |S13|);
* tau(s u) = s |s| tau(u) (nu_t is linear in |S|, S in u: reversing the
  flow reverses the stress);
* swapping x and y swaps the components (tau_xx <-> tau_yy, tau_xz <->
  tau_yz) on a square grid;
* the stress is dissipative: tau_xx du/dx <= 0 with du/dx from an
  independent difference.
"""
import numpy as np
import pytest

from workloads import Grid

KAPPA = 0.4
CS = 0.16


def _lambda0_sq(g, cs=CS):
    return (cs * (g.dx * g.dy * g.dz) ** (1.0 / 3.0)) ** 2


def _far(g):
    """phi far from any wall: no damping."""
    return np.full(g.shape, 1e12), np.full(g.shape, 1e12)


def _zeros(g):
    return np.zeros(g.shape)


@pytest.mark.parametrize("alpha", [0.7, -1.3])
def test_linear_shear_closed_form(ora, alpha):
    g = Grid(8, 6, 12, 0.7, 1.3, 0.9)
    zu = (np.arange(g.nz)[:, None, None] + 0.5) * g.dz
    u = np.broadcast_to(alpha * zu, g.shape).copy()
    pu, pw = _far(g)
    tau = ora.smagorinsky(g, pu, pw, u, _zeros(g), _zeros(g), z0=1e-3, cs=CS, kappa=KAPPA)
    l2 = _lambda0_sq(g)
    for c in (0, 1, 2, 3, 5):
        assert np.abs(tau[c]).max() == 0.0, c
    exp = -l2 * alpha * abs(alpha)
    np.testing.assert_allclose(tau[4][1:], exp, rtol=1e-13)
    # bottom w node: du/dz = (u_0 - 0) / dz = a / 2, so S13 = a / 4 and |S| = |a| / 2
    np.testing.assert_allclose(tau[4][0], exp / 4.0, rtol=1e-13)


def test_mason_damping_ratio(ora):
    g = Grid(7, 4, 10, 1.0, 1.0, 1.0)
    alpha, z0 = 0.9, 2e-3
    zu = (np.arange(g.nz)[:, None, None] + 0.5) * g.dz
    u = np.broadcast_to(alpha * zu, g.shape).copy()
    l2 = _lambda0_sq(g)
    lam0 = np.sqrt(l2)
    d_half = lam0 / KAPPA - z0                     # kappa (d + z0) = lambda0
    ds = np.array([d_half, 0.05, 0.5, 3.0, 40.0, -z0, -1.0])
    pu, pw = _far(g)
    pw = np.broadcast_to(ds[None, None, :], g.shape).copy()   # one wall distance per column
    tau = ora.smagorinsky(g, pu, pw, u, _zeros(g), _zeros(g), z0=z0, cs=CS, kappa=KAPPA)
    undamped = -l2 * alpha * abs(alpha)
    for i, d in enumerate(ds):
        ratio = 0.0 if d + z0 <= 0 else 1.0 / (1.0 + (lam0 / (KAPPA * (d + z0))) ** 2)
        np.testing.assert_allclose(tau[4][1:, :, i], undamped * ratio, rtol=1e-13, atol=0.0)
    np.testing.assert_allclose(tau[4][1:, :, 0], undamped / 2.0, rtol=1e-13)


def test_per_node_log_z0_matches_scalar(ora):
    g = Grid(6, 5, 7)
    rng = np.random.default_rng(3)
    vel = [rng.standard_normal(g.shape) for _ in range(3)]
    pu, pw = rng.uniform(0.2, 3.0, g.shape), rng.uniform(0.2, 3.0, g.shape)
    a = ora.smagorinsky(g, pu, pw, *vel, z0=3e-3)
    b = ora.smagorinsky(g, pu, pw, *vel, log_z0=np.full(g.shape, np.log(3e-3)))
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=1e-14, atol=0.0)


def test_trigonometric_fields(ora):
    g = Grid(16, 12, 6, 0.8, 1.3, 0.6)
    ax, ay = 2 * np.pi * 3 / g.lx, 2 * np.pi * 2 / g.ly
    x = np.arange(g.nx)[None, None, :] * g.dx
    y = np.arange(g.ny)[None, :, None] * g.dy
    pu, pw = _far(g)
    l2 = _lambda0_sq(g)
    z = _zeros(g)
    inner = slice(1, g.nz - 1)      # uv nodes whose w neighbours k, k+1 are interior
    # u = A sin(ax x): S11 alone on interior uv nodes
    A = 1.7
    u = np.broadcast_to(A * np.sin(ax * x), g.shape).copy()
    tau = ora.smagorinsky(g, pu, pw, u, z, z, z0=1e-3)
    s11 = A * np.cos(ax * x) * np.sin(ax * g.dx) / g.dx
    exp = -2 * l2 * np.sqrt(2.0) * np.abs(s11) * s11
    np.testing.assert_allclose(tau[0][inner], np.broadcast_to(exp, g.shape)[inner], rtol=1e-12,
                               atol=1e-15)
    assert np.abs(tau[1]).max() == 0.0 and np.abs(tau[3][inner]).max() == 0.0
    # u = A sin(ay y): S12 = (du/dy) / 2 alone
    u = np.broadcast_to(A * np.sin(ay * y), g.shape).copy()
    tau = ora.smagorinsky(g, pu, pw, u, z, z, z0=1e-3)
    s12 = 0.5 * A * np.cos(ay * y) * np.sin(ay * g.dy) / g.dy
    exp = -2 * l2 * 2.0 * np.abs(s12) * s12
    np.testing.assert_allclose(tau[3][inner], np.broadcast_to(exp, g.shape)[inner], rtol=1e-12,
                               atol=1e-15)
    assert np.abs(tau[0]).max() == 0.0
    # w = C sin(ax x): S13 = (dw/dx) / 2 on w nodes whose uv neighbours have S33 = 0
    C = -0.9
    w = np.broadcast_to(C * np.sin(ax * x), g.shape).copy()
    tau = ora.smagorinsky(g, pu, pw, z, z, w, z0=1e-3)
    s13 = 0.5 * C * np.cos(ax * x) * np.sin(ax * g.dx) / g.dx
    exp = -2 * l2 * 2.0 * np.abs(s13) * s13
    np.testing.assert_allclose(tau[4][1:g.nz - 1], np.broadcast_to(exp, g.shape)[1:g.nz - 1],
                               rtol=1e-12, atol=1e-15)
    assert np.abs(tau[5]).max() == 0.0


def test_quadratic_homogeneity_and_sign(ora):
    g = Grid(9, 7, 8, 1.1, 0.9, 1.2)
    rng = np.random.default_rng(11)
    vel = [rng.standard_normal(g.shape) for _ in range(3)]
    pu, pw = rng.uniform(-0.5, 4.0, g.shape), rng.uniform(-0.5, 4.0, g.shape)
    base = ora.smagorinsky(g, pu, pw, *vel, z0=1e-3)
    for s in (2.5, -0.5):
        sc = ora.smagorinsky(g, pu, pw, *[s * a for a in vel], z0=1e-3)
        for a, b in zip(sc, base):
            np.testing.assert_allclose(a, s * abs(s) * b, rtol=1e-12, atol=1e-15)
    # dissipative: tau_xx has the sign opposite to du/dx (independent difference)
    dudx = (np.roll(vel[0], -1, axis=2) - np.roll(vel[0], 1, axis=2)) / (2 * g.dx)
    assert (base[0] * dudx <= 0.0).all()
    dvdy = (np.roll(vel[1], -1, axis=1) - np.roll(vel[1], 1, axis=1)) / (2 * g.dy)
    assert (base[1] * dvdy <= 0.0).all()
    # no damping length at nodes with phi + z0 <= 0
    assert (base[0][pu + 1e-3 <= 0] == 0.0).all() and (base[4][pw + 1e-3 <= 0] == 0.0).all()


def test_xy_swap_covariance(ora):
    g = Grid(10, 10, 7)
    rng = np.random.default_rng(5)
    u, v, w = (rng.standard_normal(g.shape) for _ in range(3))
    pu, pw = rng.uniform(0.1, 5.0, g.shape), rng.uniform(0.1, 5.0, g.shape)
    t = ora.smagorinsky(g, pu, pw, u, v, w, z0=1e-3)
    T = lambda a: np.ascontiguousarray(np.swapaxes(a, 1, 2))
    ts = ora.smagorinsky(g, T(pu), T(pw), T(v), T(u), T(w), z0=1e-3)
    pairs = [(0, 1), (1, 0), (2, 2), (3, 3), (4, 5), (5, 4)]
    for a, b in pairs:
        np.testing.assert_allclose(ts[a], T(t[b]), rtol=1e-13, atol=1e-16)


def test_quadratic_profiles_average_between_node_sets(ora):
    """u = A sin(ax x) + b z^2 on uv nodes and w = c z^2 on w nodes: the
    staggered differences of the quadratics are exact and linear in z (S13 =
    b z on w nodes, S33 = 2 c z on uv nodes), so the averages that carry
    them to the other node set land exactly on that node's height."""
    g = Grid(12, 5, 9, 0.9, 1.1, 0.7)
    A, b, c = 1.3, 0.4, -0.6
    ax = 2 * np.pi * 2 / g.lx
    x = np.arange(g.nx)[None, None, :] * g.dx
    zu = (np.arange(g.nz)[:, None, None] + 0.5) * g.dz
    zw = np.arange(g.nz)[:, None, None] * g.dz
    u = np.broadcast_to(A * np.sin(ax * x) + b * zu ** 2, g.shape).copy()
    w = np.broadcast_to(c * zw ** 2, g.shape).copy()
    pu, pw = _far(g)
    tau = ora.smagorinsky(g, pu, pw, u, _zeros(g), w, z0=1e-3)
    l2 = _lambda0_sq(g)
    s11 = A * np.cos(ax * x) * np.sin(ax * g.dx) / g.dx
    k = slice(1, g.nz - 1)          # interior: no zero padding enters
    # uv nodes: S13 averaged from w nodes k, k+1 is b z_uv
    mag = np.sqrt(2 * (s11 ** 2 + (2 * c * zu) ** 2 + 2 * (b * zu) ** 2))
    np.testing.assert_allclose(tau[0][k], np.broadcast_to(-2 * l2 * mag * s11, g.shape)[k],
                               rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(tau[2][k], np.broadcast_to(-2 * l2 * mag * 2 * c * zu, g.shape)[k],
                               rtol=1e-12, atol=1e-15)
    # w nodes: S33 averaged from uv nodes k-1, k is 2 c z_w
    mag_w = np.sqrt(2 * (s11 ** 2 + (2 * c * zw) ** 2 + 2 * (b * zw) ** 2))
    np.testing.assert_allclose(tau[4][k], np.broadcast_to(-2 * l2 * mag_w * b * zw, g.shape)[k],
                               rtol=1e-12, atol=1e-15)
