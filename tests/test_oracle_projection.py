"""Pins of the oracle's AB2 update and pressure projection (§2.4, eqs.
u-inter, u-t+1, p-Poisson, p-Poisson-Fourier).

* a pure discrete gradient u* = (3 dt / 2) G p_true is removed entirely and
  p_true is recovered: the solver's vertical operator is the vertical part of
  D G (a wrong stencil, end row, wavenumber or factor 2/(3 dt) fails it);
* any u* with w = 0 on the bottom plane (which satisfies the solvability
  condition of the singular modes without horizontal wavenumber: the mean
  and the Nyquist modes) is projected to a discretely divergence-free field,
  D u = 0 at every node;
* projecting a divergence-free field changes nothing (p is a constant);
* AB2 with constant right-hand sides: u* = u + dt rhs.
"""
import numpy as np
import pytest

from workloads import Grid


def _grid_coords(g):
    x = np.arange(g.nx)[None, None, :] * g.dx
    y = np.arange(g.ny)[None, :, None] * g.dy
    k = np.arange(g.nz)[:, None, None]
    return x, y, k


@pytest.mark.parametrize("shape,sp", [((8, 6, 7), (1.0, 1.0, 1.0)), ((12, 8, 5), (0.7, 1.3, 0.9))])
def test_pure_gradient_removed(ora, shape, sp):
    g = Grid(*shape, *sp)
    x, y, k = _grid_coords(g)
    rng = np.random.default_rng(1)
    ax, ay = 2 * np.pi / g.lx, 2 * np.pi / g.ly
    # horizontal modes with arbitrary vertical profiles, plus a (0,0) part zero at k = 0
    p_true = (np.cos(2 * ax * x) * np.sin(ay * y) * rng.standard_normal((g.nz, 1, 1))
              + np.sin(ax * x + 0.3) * rng.standard_normal((g.nz, 1, 1))
              + np.cos(ay * y) * rng.standard_normal((g.nz, 1, 1)))
    h = rng.standard_normal((g.nz, 1, 1))
    h[0] = 0.0
    p_true = p_true + h
    dt = 0.013
    ustar = [1.5 * dt * c for c in ora.gradient_pressure(g, p_true)]
    u, v, w, p = ora.pressure_project(g, ustar, dt)
    np.testing.assert_allclose(p, p_true, atol=1e-10)
    for c in (u, v, w):
        assert np.abs(c).max() < 1e-11


def test_projected_field_is_divergence_free(ora):
    g = Grid(10, 8, 9, 1.1, 0.8, 0.7)
    rng = np.random.default_rng(2)
    u, v, w = rng.standard_normal((3,) + g.shape)
    w[0] = 0.0                                # a wall: the singular modes are solvable
    d0 = np.abs(ora.divergence_velocity(g, u, v, w)).max()
    uo, vo, wo, p = ora.pressure_project(g, [u, v, w], 0.02)
    d1 = np.abs(ora.divergence_velocity(g, uo, vo, wo)).max()
    assert d0 > 1.0 and d1 < 1e-11 * d0
    # the bottom w node carries no correction
    np.testing.assert_array_equal(wo[0], w[0])


def test_divergence_free_field_unchanged(ora):
    g = Grid(8, 8, 6)
    rng = np.random.default_rng(3)
    u, v, w = rng.standard_normal((3,) + g.shape)
    w[0] = 0.0
    uo, vo, wo, _ = ora.pressure_project(g, [u, v, w], 0.05)
    u2, v2, w2, p2 = ora.pressure_project(g, [uo, vo, wo], 0.05)
    for a, b in ((u2, uo), (v2, vo), (w2, wo)):
        np.testing.assert_allclose(a, b, atol=1e-11)
    assert np.abs(p2).max() < 1e-9


def test_ab2_constant_rhs(ora):
    rng = np.random.default_rng(4)
    u = [rng.standard_normal((3, 4, 5)) for _ in range(3)]
    r = [rng.standard_normal((3, 4, 5)) for _ in range(3)]
    out = ora.ab2_predict(u, r, r, 0.1)
    for a, b, c in zip(out, u, r):
        np.testing.assert_allclose(a, b + 0.1 * c, rtol=0, atol=1e-14)
    out = ora.ab2_predict(u, r, [2 * c for c in r], 0.1)     # 3/2 r - 1/2 (2 r) = r / 2
    for a, b, c in zip(out, u, r):
        np.testing.assert_allclose(a, b + 0.05 * c, rtol=0, atol=1e-14)
