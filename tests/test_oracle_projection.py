"""Pins of the oracle's AB2 update and pressure projection (§2.4, eqs.
u-inter, u-t+1, p-Poisson, p-Poisson-Fourier, p-bc; walls of eqs.
bc-bottom-u3 and bc-top).

By eq. dxdydz (dz = Lz / (nz - 1)) the w node nz-1 sits on the lid z = Lz and
the w node 0 on the floor; the uv layers 0 .. nz-2 are the cells between
them and the uv layer nz-1 lies above the lid.  Each pin below would fail on
a plausible mistake in that geometry or in the solve:

* a pure discrete gradient u* = (3 dt / 2) G p_true is removed entirely and
  p_true is recovered: the solver's vertical operator is the vertical part of
  D G (a wrong stencil, end row, wavenumber or factor 2/(3 dt) fails it);
* any u* is projected to a field with D u = 0 in every cell and w = 0 on both
  wall nodes (eq. p-bc's wall gradient), also when w* is not 0 there;
* with w* = 0 on both walls the lid's w stays exactly 0 (eq. bc-top);
* the wall values of w* enter neither the pressure nor the interior
  velocities (they are taken up by the wall gradient alone);
* the projection commutes with the reflection z -> Lz - z (w -> -w), which
  only holds if floor and lid are treated alike;
* the correction is orthogonal to the result over the domain's unknowns
  (G = -D^T there: the projection is an orthogonal projection);
* the layer above the lid keeps u*, v* and gets p = 0;
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


def _random(g, seed):
    rng = np.random.default_rng(seed)
    return list(rng.standard_normal((3,) + g.shape))


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
    p_true[-1] = 0.0                          # the layer above the lid carries no pressure
    dt = 0.013
    ustar = [1.5 * dt * c for c in ora.gradient_pressure(g, p_true)]
    assert np.abs(ustar[2][0]).max() == 0.0 and np.abs(ustar[2][-1]).max() == 0.0
    u, v, w, p = ora.pressure_project(g, ustar, dt)
    np.testing.assert_allclose(p, p_true, atol=1e-10)
    for c in (u, v, w):
        assert np.abs(c).max() < 1e-11


@pytest.mark.parametrize("shape,sp", [((10, 8, 9), (1.1, 0.8, 0.7)), ((8, 8, 2), (1.0, 1.0, 1.0))])
def test_projected_field_is_divergence_free(ora, shape, sp):
    g = Grid(*shape, *sp)
    u, v, w = _random(g, 2)                   # w* is not 0 on the walls
    d0 = np.abs(ora.divergence_velocity(g, u, v, w)).max()
    uo, vo, wo, p = ora.pressure_project(g, [u, v, w], 0.02)
    d1 = np.abs(ora.divergence_velocity(g, uo, vo, wo)).max()
    assert d0 > 1.0 and d1 < 1e-11 * d0
    # both wall w nodes end at 0 (eqs. bc-bottom-u3, bc-top)
    assert np.abs(wo[0]).max() < 1e-15 * np.abs(w).max()
    assert np.abs(wo[-1]).max() < 1e-15 * np.abs(w).max()


def test_lid_stays_zero(ora):
    g = Grid(8, 8, 9)
    u, v, w = _random(g, 13)
    w[0] = 0.0
    w[-1] = 0.0
    uo, vo, wo, _ = ora.pressure_project(g, [u, v, w], 0.01)
    assert np.abs(wo[-1]).max() == 0.0 and np.abs(wo[0]).max() == 0.0
    assert np.abs(ora.divergence_velocity(g, uo, vo, wo)).max() < 1e-11 * np.abs(u).max()


def test_wall_values_do_not_enter_interior(ora):
    g = Grid(8, 6, 7, 1.0, 1.2, 0.8)
    u, v, w = _random(g, 14)
    w0 = w.copy()
    w0[0] = 0.0
    w0[-1] = 0.0
    a = ora.pressure_project(g, [u, v, w], 0.03)
    b = ora.pressure_project(g, [u, v, w0], 0.03)
    for x, y in zip(a[:2] + (a[3],), b[:2] + (b[3],)):        # u, v, p
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a[2][1:-1], b[2][1:-1])


def _reflect(g, u, v, w):
    """z -> Lz - z: uv layer k <-> nz-2-k (the layer above the lid stays),
    w node k <-> nz-1-k with w -> -w."""
    def uv(a):
        out = a.copy()
        out[:-1] = a[:-1][::-1]
        return out
    return uv(u), uv(v), -w[::-1].copy()


@pytest.mark.parametrize("shape,sp", [((8, 8, 9), (1.0, 1.0, 1.0)), ((12, 6, 6), (0.9, 1.1, 0.6))])
def test_vertical_reflection(ora, shape, sp):
    g = Grid(*shape, *sp)
    u, v, w = _random(g, 15)
    w[0] = 0.0
    w[-1] = 0.0
    dt = 0.02
    out = ora.pressure_project(g, [u, v, w], dt)[:3]
    ref = ora.pressure_project(g, list(_reflect(g, u, v, w)), dt)[:3]
    for a, b in zip(_reflect(g, *out), ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_correction_orthogonal_to_result(ora):
    g = Grid(8, 8, 7, 0.9, 1.1, 0.7)
    u, v, w = _random(g, 16)
    w[0] = 0.0
    w[-1] = 0.0
    out = ora.pressure_project(g, [u, v, w], 0.02)[:3]
    # the domain's unknowns: u, v on the cells, w on the interior w nodes
    sl = (slice(0, -1), slice(0, -1), slice(1, -1))
    dot = sum(float(np.sum(o[s] * (a - o)[s])) for o, a, s in zip(out, (u, v, w), sl))
    scale = sum(float(np.sum(a[s] ** 2)) for a, s in zip((u, v, w), sl))
    corr = sum(float(np.sum((a - o)[s] ** 2)) for o, a, s in zip(out, (u, v, w), sl))
    assert corr > 0.1 * scale
    assert abs(dot) < 1e-12 * scale


def test_layer_above_lid(ora):
    g = Grid(8, 4, 6)
    u, v, w = _random(g, 17)
    uo, vo, wo, p = ora.pressure_project(g, [u, v, w], 0.02)
    np.testing.assert_array_equal(uo[-1], u[-1])
    np.testing.assert_array_equal(vo[-1], v[-1])
    assert np.abs(p[-1]).max() == 0.0
    assert np.abs(p[:-1]).max() > 0.0


def test_divergence_free_field_unchanged(ora):
    g = Grid(8, 8, 6)
    u, v, w = _random(g, 3)
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
