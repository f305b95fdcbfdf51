"""Property-based pins of the oracle (hypothesis, derandomized): the closed
forms of the tilted-plane and flat-wall pins under random plane tilts and
offsets, band widths 2 phi_b in [dz, 1.5 dz], phi_c in [2 phi_b, 4 phi_b] and
anisotropic spacings.

* Tilted plane, uniform velocity U0: every band node away from the seams and
  the top has tau = tau_w (t n^T + n t^T) with t the unit tangential part of
  U0 and tau_w = -(kappa |U_r| / ln(phi_c / z0))^2 (§3.3: the interpolated
  velocity of a uniform field is the field, the local frame is (t, n x t,
  n)).
* Flat wall at z_w: per column, the uv band nodes are those with 0 <=
  (k + 1/2) dz - z_w <= b, the w band nodes those with |k dz - z_w| <= b/2,
  solid below (§3.3 class lists), counted in closed form.
"""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

from workloads import Grid, terrain

KAPPA = 0.4
SETTINGS = settings(max_examples=30, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.function_scoped_fixture])


@SETTINGS
@given(polar=st.floats(0.0, 1.1), azim=st.floats(0.0, 2 * math.pi),
       off=st.floats(0.0, 1.0), beta=st.floats(1.0, 1.5), gamma=st.floats(1.0, 2.0),
       dx=st.floats(0.6, 1.6), dy=st.floats(0.6, 1.6), dz=st.floats(0.6, 1.6),
       u0=st.tuples(st.floats(-3, 3), st.floats(-3, 3), st.floats(-3, 3)))
def test_tilted_plane_uniform_velocity(ora, polar, azim, off, beta, gamma, dx, dy, dz, u0):
    n_hat = np.array([math.sin(polar) * math.cos(azim), math.sin(polar) * math.sin(azim),
                      math.cos(polar)])
    U0 = np.array(u0)
    ur = U0 - U0.dot(n_hat) * n_hat
    if np.linalg.norm(ur) < 1e-3:
        return
    g = Grid(32, 32, 26, dx, dy, dz)
    b = beta * dz
    phi_c = gamma * b
    z0 = 1e-3 * dz
    pu, pw = terrain.plane(g, (16 * dx, 16 * dy, (6 + off) * dz), n_hat)
    vel = [np.full(g.shape, U0[c]) for c in range(3)]
    tau, _ = ora.wall_stress(g, b, phi_c, KAPPA, pu, pw, *vel, z0, None,
                             [np.zeros(g.shape)] * 6)
    t = ur / np.linalg.norm(ur)
    tw = -(KAPPA * np.linalg.norm(ur) / math.log(phi_c / z0)) ** 2
    expect = tw * (np.outer(t, n_hat) + np.outer(n_hat, t))
    reach = phi_c + b                                   # the sample shift and more
    mx = math.ceil(reach / dx) + 2
    my = math.ceil(reach / dy) + 2
    kmax = g.nz - 3 - math.ceil(reach / dz)
    checked = 0
    for kind, phi, comps in ((0, pu, [(0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 0, 1)]),
                             (1, pw, [(4, 0, 2), (5, 1, 2)])):
        sel = (phi >= 0) & (phi <= b) if kind == 0 else np.abs(phi) <= b / 2
        for k, j, i in np.argwhere(sel):
            if not (mx <= i < g.nx - mx and my <= j < g.ny - my and k <= kmax):
                continue
            for c, a, bb in comps:
                assert abs(tau[c][k, j, i] - expect[a, bb]) <= 1e-13 * (1 + abs(tw))
            checked += 1
    assert checked > 0


@SETTINGS
@given(zw_cells=st.floats(0.3, 3.0), beta=st.floats(1.0, 1.5), dz=st.floats(0.6, 1.6),
       dx=st.floats(0.6, 1.6))
def test_flat_wall_class_counts(ora, zw_cells, beta, dz, dx):
    g = Grid(5, 4, 9, dx, 1.0, dz)
    zw = zw_cells * dz
    b = beta * dz
    pu, pw = terrain.flat(g, zw)
    mask = ora.classify(g, b, pu, pw)
    uvc, wc = mask & 3, (mask >> 2) & 3
    k = np.arange(g.nz)
    huv = (k + 0.5) * dz - zw
    hw = k * dz - zw
    # every column alike
    exp_uv_band = int(((huv >= 0) & (huv <= b)).sum())
    exp_uv_solid = int((huv < 0).sum())
    exp_w_band = int((np.abs(hw) <= b / 2).sum())
    exp_w_solid = int((hw < -b / 2).sum())
    cols = g.nx * g.ny
    assert int((uvc == 1).sum()) == exp_uv_band * cols
    assert int((uvc == 2).sum()) == exp_uv_solid * cols
    assert int((wc == 1).sum()) == exp_w_band * cols
    assert int((wc == 2).sum()) == exp_w_solid * cols
