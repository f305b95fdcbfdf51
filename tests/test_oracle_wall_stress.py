"""Pins of the oracle's wall model (§3.3, eq. bc-bottom-immersed and the tensor rotation).

* Flat walls with a pure log profile at the §4.1 offsets: closed-form
  stresses; for z_w = 1 and phi_c = 1.5 the sample lands on a uv node and
  tau_w = -u_*^2 exactly, which is the flat-wall condition of eq.
  bc-bottom-1 (tau_xz = tau_w u/U_r, tau_yz = tau_w v/U_r, other components 0).
* Tilted planes with uniform velocity: tau = tau_w (t n^T + n t^T).
* Rotation covariance: tau(R plane, R U0) = R tau(plane, U0) R^T.
* Discrete x<->y swap and x reflection permute every output.
* Symmetry and zero trace of the rotated tensor; U_r = 0 gives zero stress.
* Band statistics (sums of tau_w per node set, max |U_r| over all records,
  record count) in closed form with the two node sets' bands on flat walls
  at different heights.
"""
import numpy as np
import pytest

from workloads import Grid, configs, terrain

KAPPA = 0.4


def _ln(phi_c, z0):
    return np.log(phi_c / z0)


@pytest.mark.parametrize("zw", [1.0, 1.25, 1.5, 1.75])
@pytest.mark.parametrize("theta", [0.0, 0.7, -2.2])
@pytest.mark.parametrize("b,phi_c", [(1.5, 1.5), (1.0, 1.0), (1.0, 1.5), (1.25, 2.0)])
def test_flat_wall_log_profile_closed_form(ora, zw, theta, b, phi_c):
    g = Grid(6, 5, 10)
    z0 = 8e-4
    ustar = 1.3
    wl = configs.flat(g, zw, theta=theta, z0=z0, band_width=b, phi_c=phi_c)
    wl.u *= ustar
    wl.v *= ustar
    tau_in = [np.full(g.shape, 7.0) for _ in range(6)]       # a marker for "untouched"
    tau, stats = ora.wall_stress(g, b, phi_c, KAPPA, wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w, z0,
                                 None, tau_in)
    # every band node samples the height z_w + phi_c; uv index coordinate zeta
    zs = zw + phi_c
    zeta = zs - 0.5
    k0 = int(np.floor(zeta))
    a = zeta - k0
    U = lambda k: ustar / KAPPA * np.log((k + 0.5 - zw) / z0)
    Ubar = (1 - a) * U(k0) + a * U(k0 + 1)
    tau_w = -(KAPPA * Ubar / _ln(phi_c, z0)) ** 2
    if zw == 1.0 and phi_c == 1.5:
        assert abs(tau_w + ustar ** 2) < 1e-13          # the equilibrium log-law stress
    mask = ora.classify(g, b, wl.phi_uv, wl.phi_w)
    uvc, wc = mask & 3, (mask >> 2) & 3
    # w band: tau_xz, tau_yz from eq. bc-bottom-1; uv band: the four other components vanish
    np.testing.assert_allclose(tau[4][wc == 1], tau_w * np.cos(theta), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(tau[5][wc == 1], tau_w * np.sin(theta), rtol=1e-13, atol=1e-15)
    for c in range(4):
        assert np.abs(tau[c][uvc == 1]).max() < 1e-14
    # solid nodes zeroed on their own grid's components, fluid untouched
    for c in range(4):
        assert (tau[c][uvc == 2] == 0).all() and (tau[c][uvc == 0] == 7.0).all()
    for c in (4, 5):
        assert (tau[c][wc == 2] == 0).all() and (tau[c][wc == 0] == 7.0).all()
    nb = (uvc == 1).sum() + (wc == 1).sum()
    assert stats[3] == nb
    np.testing.assert_allclose(stats[0], tau_w * (uvc == 1).sum(), rtol=1e-12)
    np.testing.assert_allclose(stats[1], tau_w * (wc == 1).sum(), rtol=1e-12)


def _tilted_setup(n_hat, U0, g=Grid(20, 18, 16), point=(10.0, 9.0, 7.0)):
    pu, pw = terrain.plane(g, point, n_hat)
    vel = [np.full(g.shape, U0[c]) for c in range(3)]
    return g, pu, pw, vel


def _interior_band(g, phi, b, kind, margin=4):
    if kind == 0:
        sel = (phi >= 0) & (phi <= b)
    else:
        sel = np.abs(phi) <= b / 2
    idx = np.argwhere(sel)
    keep = ((idx[:, 2] >= margin) & (idx[:, 2] < g.nx - margin) & (idx[:, 1] >= margin)
            & (idx[:, 1] < g.ny - margin) & (idx[:, 0] >= 1) & (idx[:, 0] < g.nz - 3))
    return idx[keep]


def _rand_unit(rng, zmin=0.25):
    while True:
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        if v[2] > zmin:
            return v


def test_tilted_planes_closed_form(ora):
    rng = np.random.default_rng(5)
    b, phi_c, z0 = 1.5, 1.5, 1e-3
    lnr = _ln(phi_c, z0)
    for _ in range(12):
        n_hat = _rand_unit(rng)
        U0 = rng.standard_normal(3) * 3
        g, pu, pw, vel = _tilted_setup(n_hat, U0)
        ur = U0 - U0.dot(n_hat) * n_hat
        t = ur / np.linalg.norm(ur)
        tw = -(KAPPA * np.linalg.norm(ur) / lnr) ** 2
        expect = tw * (np.outer(t, n_hat) + np.outer(n_hat, t))
        tau, _ = ora.wall_stress(g, b, phi_c, KAPPA, pu, pw, *vel, z0, None,
                                 [np.zeros(g.shape)] * 6)
        ok = 0
        for kind, phi, comps in ((0, pu, [(0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 0, 1)]),
                                 (1, pw, [(4, 0, 2), (5, 1, 2)])):
            for (k, j, i) in _interior_band(g, phi, b, kind):
                for c, a_, b_ in comps:
                    assert abs(tau[c][k, j, i] - expect[a_, b_]) < 1e-14 * (1 + abs(tw))
                ok += 1
        assert ok > 50


def test_tilted_plane_linear_velocity(ora):
    """Each velocity component is linear in the position of its own node set,
    so the interpolated sample is exact and the stress has a closed form; a
    sample taken on the wrong staggered grid or at the wrong point fails."""
    rng = np.random.default_rng(13)
    b, phi_c, z0 = 1.5, 1.5, 1e-3
    lnr = _ln(phi_c, z0)
    g = Grid(22, 20, 16, 1.0, 0.9, 1.1)
    for _ in range(8):
        n_hat = _rand_unit(rng, 0.4)
        pu, pw = terrain.plane(g, (11.0, 9.0, 8.0), n_hat)
        A = rng.standard_normal(3)
        B = rng.standard_normal((3, 3)) * 0.3
        x = (np.arange(g.nx) * g.dx)[None, None, :]
        y = (np.arange(g.ny) * g.dy)[None, :, None]
        vel = []
        for c, zoff in ((0, 0.5), (1, 0.5), (2, 0.0)):
            z = ((np.arange(g.nz) + zoff) * g.dz)[:, None, None]
            vel.append(np.ascontiguousarray(np.broadcast_to(
                A[c] + B[c, 0] * x + B[c, 1] * y + B[c, 2] * z, g.shape)))
        tau, _ = ora.wall_stress(g, b, phi_c, KAPPA, pu, pw, *vel, z0, None,
                                 [np.zeros(g.shape)] * 6)
        n_ok = 0
        for kind, phi, zoff, comps in ((0, pu, 0.5, [(0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 0, 1)]),
                                       (1, pw, 0.0, [(4, 0, 2), (5, 1, 2)])):
            for (k, j, i) in _interior_band(g, phi, b, kind):
                xn = np.array([i * g.dx, j * g.dy, (k + zoff) * g.dz])
                p = xn + (phi_c - phi[k, j, i]) * n_hat
                if not (0.5 * g.dz < p[2] < (g.nz - 1) * g.dz):
                    continue
                us = A + B @ p
                ur = us - us.dot(n_hat) * n_hat
                U = np.linalg.norm(ur)
                tw = -(KAPPA * U / lnr) ** 2
                ex = tw / U * (np.outer(ur, n_hat) + np.outer(n_hat, ur))
                for c, a_, b_ in comps:
                    assert abs(tau[c][k, j, i] - ex[a_, b_]) < 1e-12 * (1 + abs(tw))
                n_ok += 1
        assert n_ok > 40


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _tau_at_some_band_node(ora, n_hat, U0, b=1.5, phi_c=1.5, z0=1e-3):
    g, pu, pw, vel = _tilted_setup(n_hat, U0)
    k, j, i = _interior_band(g, pu, b, 0)[0]
    t, tw, U = ora.local_stress(g, b, phi_c, KAPPA, pu, 0, i, j, k, *vel, _ln(phi_c, z0))
    return t


def test_rotation_covariance(ora):
    rng = np.random.default_rng(9)
    done = 0
    while done < 12:
        n_hat = _rand_unit(rng)
        R = _rotation(rng)
        if (R @ n_hat)[2] < 0.25:      # keep the rotated surface a graph over the floor
            continue
        U0 = rng.standard_normal(3) * 2
        t1 = _tau_at_some_band_node(ora, n_hat, U0)
        t2 = _tau_at_some_band_node(ora, R @ n_hat, R @ U0)
        np.testing.assert_allclose(t2, R @ t1 @ R.T, atol=1e-14 * np.abs(t1).max())
        done += 1


def test_symmetric_traceless_and_zero_slip(ora):
    rng = np.random.default_rng(2)
    for _ in range(10):
        n_hat = _rand_unit(rng)
        U0 = rng.standard_normal(3)
        t = _tau_at_some_band_node(ora, n_hat, U0)
        assert (t == t.T).all()                      # bit-exact symmetry
        assert abs(np.trace(t)) < 1e-15 * (1 + np.abs(t).max())
    # velocity along the normal: no tangential part, no stress
    n_hat = _rand_unit(rng)
    t = _tau_at_some_band_node(ora, n_hat, 2.5 * n_hat)
    assert np.abs(t).max() < 1e-15


def _square_cube():
    g = Grid(24, 24, 14)
    pu, pw = terrain.cube_on_floor(g, 1.0, 7.0, 13.0, 9.0, 16.0, 7.0)
    rng = np.random.default_rng(21)
    f = lambda s=1.0: s * rng.standard_normal(g.shape)
    return g, pu, pw, f(), f(), f(), [f(0.01) for _ in range(6)]


def _run(ora, g, pu, pw, u, v, w, tau):
    t, st = ora.wall_stress(g, 1.5, 1.5, KAPPA, pu, pw, u, v, w, 1e-3, None, tau)
    d = ora.divergence(g, t)
    return ora.classify(g, 1.5, pu, pw), t, d


def test_xy_swap_permutes_outputs(ora):
    g, pu, pw, u, v, w, tau = _square_cube()
    T = lambda a: np.ascontiguousarray(a.transpose(0, 2, 1))
    m1, t1, d1 = _run(ora, g, pu, pw, u, v, w, tau)
    m2, t2, d2 = _run(ora, g, T(pu), T(pw), T(v), T(u), T(w),
                      [T(tau[1]), T(tau[0]), T(tau[2]), T(tau[3]), T(tau[5]), T(tau[4])])
    assert (T(m1) == m2).all()
    perm = [1, 0, 2, 3, 5, 4]
    for c in range(6):
        np.testing.assert_allclose(t2[c], T(t1[perm[c]]), rtol=0, atol=1e-15)
    for c, pc in enumerate([1, 0, 2]):
        np.testing.assert_allclose(d2[c], T(d1[pc]), rtol=0, atol=1e-14)


def test_x_reflection_permutes_outputs(ora):
    g, pu, pw, u, v, w, tau = _square_cube()
    idx = (-np.arange(g.nx)) % g.nx
    Rf = lambda a: np.ascontiguousarray(a[:, :, idx])
    m1, t1, d1 = _run(ora, g, pu, pw, u, v, w, tau)
    sgn_t = [1, 1, 1, -1, -1, 1]
    m2, t2, d2 = _run(ora, g, Rf(pu), Rf(pw), -Rf(u), Rf(v), Rf(w),
                      [s * Rf(a) for s, a in zip(sgn_t, tau)])
    assert (Rf(m1) == m2).all()
    for c in range(6):
        np.testing.assert_allclose(t2[c], sgn_t[c] * Rf(t1[c]), rtol=0, atol=1e-15)
    for c, s in enumerate([-1, 1, 1]):
        np.testing.assert_allclose(d2[c], s * Rf(d1[c]), rtol=0, atol=1e-14)


def test_per_node_log_z0_matches_scalar(ora):
    wl = configs.cube(32, 16, 16)
    g = wl.grid
    z0 = 3e-4
    a, sa = ora.wall_stress(g, 1.5, 1.5, KAPPA, wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w, z0, None,
                            wl.tau)
    b, sb = ora.wall_stress(g, 1.5, 1.5, KAPPA, wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w, 99.0,
                            np.full(g.shape, np.log(z0)), wl.tau)
    for c in range(6):
        np.testing.assert_allclose(a[c], b[c], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("za,zb,a,c", [(1.0, 3.25, -2.0, 1.5), (3.25, 1.0, -2.0, 1.5),
                                       (1.5, 2.75, -10.0, 1.0), (2.75, 1.5, 0.5, 2.0)])
def test_band_statistics_two_walls(ora, za, zb, a, c):
    """All four band statistics in closed form, with the uv band and the w
    band drawn from flat walls at different heights (the caller supplies phi
    on each node set): every uv record samples z_a + phi_c and every w record
    z_b + phi_c, where the velocity (a + c z)(cos t, sin t, .) is linear in z,
    so |U_r| is |a + c (z + phi_c)| per set.  stats = [sum of tau_w over uv
    records, the same over w records, max |U_r| over all records, record
    count]: a maximum over one set only, or without the other set's value,
    fails one of the four cases."""
    g = Grid(6, 5, 12)
    b, phi_c, z0, theta = 1.5, 1.5, 1e-3, 0.6
    pu = terrain.flat(g, za)[0]
    pw = terrain.flat(g, zb)[1]
    zuv = (np.arange(g.nz) + 0.5)[:, None, None] * np.ones(g.shape)
    prof = a + c * zuv
    u, v = prof * np.cos(theta), prof * np.sin(theta)
    w = np.random.default_rng(3).standard_normal(g.shape)       # removed by n = e_z
    tau, stats = ora.wall_stress(g, b, phi_c, KAPPA, pu, pw, u, v, w, z0, None,
                                 [np.zeros(g.shape)] * 6)
    Ua, Ub = abs(a + c * (za + phi_c)), abs(a + c * (zb + phi_c))
    tw = lambda U: -(KAPPA * U / _ln(phi_c, z0)) ** 2
    nuv = int(((pu >= 0) & (pu <= b)).sum())
    nw = int((np.abs(pw) <= b / 2).sum())
    assert nuv > 0 and nw > 0
    np.testing.assert_allclose(stats[0], nuv * tw(Ua), rtol=1e-12)
    np.testing.assert_allclose(stats[1], nw * tw(Ub), rtol=1e-12)
    np.testing.assert_allclose(stats[2], max(Ua, Ub), rtol=1e-13)
    assert stats[3] == nuv + nw
