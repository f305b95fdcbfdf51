"""Pins of the oracle's stress divergence, forcing and drag.

* Trigonometric stresses: a periodic central difference of sin(a x) is
  cos(a x) sin(a dx)/dx exactly; linear vertical profiles have exact
  staggered differences, with the zero-padding rule at k = -1 and k = nz.
* Telescoping: summed over every node the horizontal terms cancel and the
  vertical ones leave the first and last planes.
* Flat-wall drag: for any SGS stress, the fluid-side drag of a flat wall
  equals -nx ny dx dy tau_w cos(theta) (the w node below the first fluid uv
  node is always a band node, §3.3).
* Forcing, eq. u-*-IBM: forced nodes carry (3 dt / 2) grad p, others keep u*.
* D^T is the transpose of D (dot-product test).
"""
import numpy as np
import pytest

from workloads import Grid, configs

KAPPA = 0.4


def test_divergence_trigonometric_closed_form(ora):
    g = Grid(16, 12, 9, 0.8, 1.3, 0.6)
    x = np.arange(g.nx)[None, None, :] * g.dx
    y = np.arange(g.ny)[None, :, None] * g.dy
    zu = (np.arange(g.nz)[:, None, None] + 0.5) * g.dz
    zw = np.arange(g.nz)[:, None, None] * g.dz
    k = np.arange(g.nz)[:, None, None]
    ax, ay = 2 * np.pi * 3 / g.lx, 2 * np.pi * 2 / g.ly
    c = [0.3, -1.1, 0.7, 1.9, -0.4, 0.8]
    s = [0.2, 0.5, -1.3, 0.6, 1.4, -0.9]
    Lz = lambda m, z: c[m] + s[m] * z
    sx, cx, sy, cy = np.sin(ax * x), np.cos(ax * x), np.sin(ay * y), np.cos(ay * y)
    full = lambda a: np.ascontiguousarray(np.broadcast_to(a, g.shape))
    tau = [full(sx * cy * Lz(0, zu)), full(cx * sy * Lz(1, zu)), full(np.sin(ax * x + ay * y) * Lz(2, zu)),
           full(cx * cy * Lz(3, zu)), full(sx * sy * Lz(4, zw)), full(cx * sy * Lz(5, zw))]
    div = ora.divergence(g, tau)
    # exact periodic central differences: d sin = cos * f, d cos = -sin * f
    fx, fy = np.sin(ax * g.dx) / g.dx, np.sin(ay * g.dy) / g.dy
    top, bot = k == g.nz - 1, k == 0
    # (A(k+1) - A(k)) / dz for A linear on w nodes with A(nz) = 0
    v4 = np.where(top, -Lz(4, zw) / g.dz, s[4])
    v5 = np.where(top, -Lz(5, zw) / g.dz, s[5])
    # (B(k) - B(k-1)) / dz for B linear on uv nodes with B(-1) = 0
    v2 = np.where(bot, Lz(2, zu) / g.dz, s[2])
    ex = [cx * fx * cy * Lz(0, zu) + cx * (-sy * fy) * Lz(3, zu) + sx * sy * v4,
          (-sx * fx) * cy * Lz(3, zu) + cx * cy * fy * Lz(1, zu) + cx * sy * v5,
          cx * fx * sy * Lz(4, zw) + cx * cy * fy * Lz(5, zw) + np.sin(ax * x + ay * y) * v2]
    for c_ in range(3):
        np.testing.assert_allclose(div[c_], full(ex[c_]), rtol=0, atol=1e-13)


def test_divergence_telescopes(ora):
    g = Grid(9, 7, 6, 1.1, 0.9, 0.5)
    rng = np.random.default_rng(4)
    tau = [rng.standard_normal(g.shape) for _ in range(6)]
    div = ora.divergence(g, tau)
    dv = g.dv
    # sum of (A(k+1)-A(k))/dz over k with A(nz)=0 is -A(0)/dz; (B(k)-B(k-1)) gives B(nz-1)/dz
    np.testing.assert_allclose(div[0].sum() * dv, -tau[4][0].sum() * g.dx * g.dy, atol=1e-12)
    np.testing.assert_allclose(div[1].sum() * dv, -tau[5][0].sum() * g.dx * g.dy, atol=1e-12)
    np.testing.assert_allclose(div[2].sum() * dv, tau[2][-1].sum() * g.dx * g.dy, atol=1e-12)


@pytest.mark.parametrize("zw", [1.0, 1.25, 1.5, 1.75])
@pytest.mark.parametrize("b", [1.0, 1.25, 1.5])
def test_flat_wall_drag_closed_form(ora, zw, b):
    g = Grid(8, 6, 10)
    theta = 0.6
    wl = configs.flat(g, zw, theta=theta, z0=8e-4, tau_std=0.05, band_width=b, phi_c=1.5,
                      seed=int(zw * 100 + b * 10))
    tau, st = ora.wall_stress(g, b, 1.5, KAPPA, wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w, wl.z0,
                              None, wl.tau)
    div = ora.divergence(g, tau)
    D = ora.drag(g, wl.phi_uv, wl.phi_w, div)
    # closed-form tau_w: every band node samples the height z_w + phi_c of the log profile
    zeta = zw + 1.5 - 0.5
    k0 = int(np.floor(zeta))
    a = zeta - k0
    U = lambda k: np.log((k + 0.5 - zw) / wl.z0) / KAPPA
    tau_w = -(KAPPA * ((1 - a) * U(k0) + a * U(k0 + 1)) / np.log(1.5 / wl.z0)) ** 2
    expect_x = -g.nx * g.ny * g.dx * g.dy * tau_w * np.cos(theta)
    expect_y = -g.nx * g.ny * g.dx * g.dy * tau_w * np.sin(theta)
    assert abs(D[0] - expect_x) < 1e-12 * abs(expect_x)
    assert abs(D[1] - expect_y) < 1e-12 * abs(expect_x)


def test_divergence_transpose_dot_product(ora):
    g = Grid(7, 6, 5, 0.9, 1.2, 0.8)
    rng = np.random.default_rng(8)
    tau = [rng.standard_normal(g.shape) for _ in range(6)]
    gd = [rng.standard_normal(g.shape) for _ in range(3)]
    div = ora.divergence(g, tau)
    gt = ora.divergence_transpose(g, gd)
    lhs = sum((a * b).sum() for a, b in zip(div, gd))
    rhs = sum((a * b).sum() for a, b in zip(tau, gt))
    assert abs(lhs - rhs) < 1e-13 * sum(np.abs(a).sum() for a in div)


def test_forcing(ora):
    wl = configs.cube(32, 16, 12)
    g = wl.grid
    us = ora.forcing(g, wl.phi_uv, wl.phi_w, (wl.u, wl.v, wl.w), None, wl.dt)
    fu, fw = wl.phi_uv <= 0, wl.phi_w <= 0
    assert (us[0][fu] == 0).all() and (us[1][fu] == 0).all() and (us[2][fw] == 0).all()
    assert (us[0][~fu] == wl.u[~fu]).all() and (us[2][~fw] == wl.w[~fw]).all()
    us = ora.forcing(g, wl.phi_uv, wl.phi_w, (wl.u, wl.v, wl.w), wl.gradp, wl.dt)
    for c, f in ((0, fu), (1, fu), (2, fw)):
        np.testing.assert_allclose(us[c][f], 1.5 * wl.dt * wl.gradp[c][f], rtol=2e-16, atol=0)
    assert fu.sum() > 0 and fw.sum() > fu.sum()
