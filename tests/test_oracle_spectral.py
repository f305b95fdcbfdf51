"""Pins of the oracle's pseudo-spectral horizontal derivative (§2.4,
eq. dudx) and of the divergence built on it.

* trigonometric modes below the Nyquist number are differentiated exactly:
  d/dx sin(k x) = k cos(k x) (this is what separates it from the central
  difference, whose factor is sin(k dx) / dx);
* the Nyquist mode of an even node count, (-1)^i, has no derivative;
* a brute-force DFT (explicit sums of exponentials, no library FFT) on small
  rows gives the same derivative;
* the operator is skew: sum a db/dx = -sum b da/dx;
* the spectral divergence of trigonometric stresses in closed form, with the
  staggered vertical differences and zero padding of the central-difference
  divergence.
"""
import numpy as np
import pytest

from workloads import Grid


@pytest.mark.parametrize("n,length", [(16, 5.0), (32, 11.3), (12, 2.0)])
def test_trigonometric_modes_exact(ora, n, length):
    x = np.arange(n) * length / n
    for m in range(1, (n - 1) // 2 + 1):
        k = 2 * np.pi * m / length
        for f, df in ((np.sin(k * x), k * np.cos(k * x)), (np.cos(k * x), -k * np.sin(k * x))):
            got = ora.spectral_derivative(f, 0, length)
            np.testing.assert_allclose(got, df, rtol=0, atol=1e-11 * k)


def test_nyquist_mode_dropped(ora):
    n = 16
    f = (-1.0) ** np.arange(n)
    assert np.abs(ora.spectral_derivative(f, 0, 3.0)).max() < 1e-13
    # with a mode below it, only the lower mode survives
    x = np.arange(n) * 3.0 / n
    k = 2 * np.pi * 5 / 3.0
    got = ora.spectral_derivative(np.sin(k * x) + 0.7 * f, 0, 3.0)
    np.testing.assert_allclose(got, k * np.cos(k * x), atol=1e-12)


@pytest.mark.parametrize("n", [8, 9, 10])
def test_brute_force_dft(ora, n):
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n)
    length = 1.7
    x = np.arange(n) * length / n
    ms = [m for m in range(-(n // 2), n // 2 + 1) if abs(m) < n / 2]    # Nyquist excluded
    d = np.zeros(n)
    for m in ms:
        k = 2 * np.pi * m / length
        a = sum(f[l] * np.exp(-1j * k * x[l]) for l in range(n)) / n
        d += np.real(1j * k * a * np.exp(1j * k * x))
    np.testing.assert_allclose(ora.spectral_derivative(f, 0, length), d, atol=1e-12)


def test_skew_symmetry_and_axes(ora):
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal((2, 5, 8, 16))
    for axis, length in ((2, 3.0), (1, 7.0)):
        lhs = (a * ora.spectral_derivative(b, axis, length)).sum()
        rhs = -(b * ora.spectral_derivative(a, axis, length)).sum()
        assert abs(lhs - rhs) < 1e-11 * np.abs(a).sum()
    # along y only: a field constant in y has no y derivative
    c = np.broadcast_to(rng.standard_normal((5, 1, 16)), (5, 8, 16))
    assert np.abs(ora.spectral_derivative(c, 1, 7.0)).max() < 1e-13


def test_spectral_divergence_closed_form(ora):
    g = Grid(16, 12, 7, 0.8, 1.3, 0.6)
    x = np.arange(g.nx)[None, None, :] * g.dx
    y = np.arange(g.ny)[None, :, None] * g.dy
    zu = (np.arange(g.nz)[:, None, None] + 0.5) * g.dz
    zw = np.arange(g.nz)[:, None, None] * g.dz
    ax, ay = 2 * np.pi * 3 / g.lx, 2 * np.pi * 2 / g.ly
    c = [0.3, -1.1, 0.7, 1.9, -0.4, 0.8]
    one = np.ones(g.shape)
    # tau_c = c_c * (trig in x and y) * (linear in z on its own node set)
    txx = c[0] * np.sin(ax * x) * (1 + zu) * one
    tyy = c[1] * np.cos(ay * y) * (2 - zu) * one
    tzz = c[2] * np.sin(ax * x) * np.cos(ay * y) * (1 + 2 * zu) * one
    txy = c[3] * np.cos(ax * x) * np.sin(ay * y) * zu * one
    txz = c[4] * np.cos(ax * x) * (1 + zw) * one
    tyz = c[5] * np.sin(ay * y) * (3 - zw) * one
    div = ora.divergence_spectral(g, [txx, tyy, tzz, txy, txz, tyz])
    k = np.arange(g.nz)[:, None, None]
    top = (k == g.nz - 1)
    bot = (k == 0)
    # x momentum: exact horizontal derivatives, staggered z with zero above the top
    dz_txz = np.where(top, -c[4] * np.cos(ax * x) * (1 + zw), c[4] * np.cos(ax * x) * g.dz) / g.dz
    ex = (c[0] * ax * np.cos(ax * x) * (1 + zu) + c[3] * ay * np.cos(ax * x) * np.cos(ay * y) * zu
          + dz_txz)
    np.testing.assert_allclose(div[0], ex * one, atol=1e-11)
    dz_tyz = np.where(top, -c[5] * np.sin(ay * y) * (3 - zw), -c[5] * np.sin(ay * y) * g.dz) / g.dz
    ey = (-c[3] * ax * np.sin(ax * x) * np.sin(ay * y) * zu - c[1] * ay * np.sin(ay * y) * (2 - zu)
          + dz_tyz)
    np.testing.assert_allclose(div[1], ey * one, atol=1e-11)
    tzz_below = np.where(bot, 0.0, c[2] * np.sin(ax * x) * np.cos(ay * y) * (1 + 2 * (zu - g.dz)))
    ez = (-c[4] * ax * np.sin(ax * x) * (1 + zw) + c[5] * ay * np.cos(ay * y) * (3 - zw)
          + (tzz - tzz_below) / g.dz)
    np.testing.assert_allclose(div[2], ez * one, atol=1e-11)
