"""Pins of the oracle's version of Chester et al.'s original method (§1: a
near-wall model in the fluid band, linear extrapolation of the stresses into a
solid band, SOR smoothing of the stress inside the body; §3.3's closing
paragraphs).

The steps' stencils are readings (the paper names the steps only); each pin
checks the oracle against a fact fixed independently of its code:

* classes: the hand-derived layer table of
  ``tests/golden/chester_flat_wall_layers.txt`` and the interval end points;
* step 1: on a flat wall with a log profile the fluid-band stresses follow the
  flat-wall closed form of eq. bc-bottom-1 on both node sets, the body is 0;
* step 2: a stress field linear in position is reproduced exactly on the solid
  band of tilted planes (samples at phi_c and 2 phi_c along the normal, on the
  component's own node set); on a flat wall a stress quadratic in z gives the
  straight line through its vertically interpolated samples;
* step 3: one red-black sweep equals the matrix form of SOR built from a
  dense Laplacian; many sweeps converge to the dense harmonic extension
  (numpy solve) of the fixed values; a field linear in z is a fixed point.
"""
import os

import numpy as np
import pytest

from workloads import Grid, configs, terrain

GOLD = os.path.join(os.path.dirname(__file__), "golden", "chester_flat_wall_layers.txt")
KAPPA = 0.4


def _rows():
    out = []
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if line:
            v = line.split()
            out.append((float(v[0]), float(v[1]), *map(int, v[2:])))
    return out


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"b{r[0]}-zw{r[1]}")
def test_flat_wall_layer_table(ora, row):
    b, zw, uvb, uvs, uvi, wb, ws, wi = row
    g = Grid(6, 5, 9)
    pu, pw = terrain.flat(g, zw)
    cols = g.nx * g.ny
    cnt = ora.chester_counts(g, b, pu, pw)
    assert list(cnt) == [(g.nz - uvb - uvs - uvi) * cols, uvb * cols, uvs * cols, uvi * cols,
                         (g.nz - wb - ws - wi) * cols, wb * cols, ws * cols, wi * cols]


@pytest.mark.parametrize("phi,cls", [(1.5, 1), (np.nextafter(1.5, 2), 0), (0.0, 1), (-0.0, 1),
                                     (np.nextafter(0.0, -1), 2), (-1.5, 2),
                                     (np.nextafter(-1.5, -2), 3), (-1e300, 3), (1e300, 0)])
def test_interval_ends(ora, phi, cls):
    assert ora.chester_class(phi, 1.5) == cls


@pytest.mark.parametrize("zw", [1.0, 1.25, 1.5, 1.75])
def test_step1_flat_wall_closed_form(ora, zw):
    g = Grid(6, 5, 10)
    b = phi_c = 1.5
    z0, theta, us = 8e-4, 0.7, 1.2
    wl = configs.flat(g, zw, theta=theta, z0=z0)
    wl.u *= us
    wl.v *= us
    tau, stats = ora.chester_wall_stress(g, b, phi_c, KAPPA, wl.phi_uv, wl.phi_w, wl.u, wl.v,
                                         wl.w, z0, None, [np.full(g.shape, 7.0)] * 6)
    zeta = zw + phi_c - 0.5                      # uv index coordinate of every sample
    k0 = int(np.floor(zeta))
    a = zeta - k0
    U = lambda k: us / KAPPA * np.log((k + 0.5 - zw) / z0)
    tw = -(KAPPA * ((1 - a) * U(k0) + a * U(k0 + 1)) / np.log(phi_c / z0)) ** 2
    cls = lambda phi: np.where(phi > b, 0, np.where(phi >= 0, 1, np.where(phi >= -b, 2, 3)))
    cu, cw = cls(wl.phi_uv), cls(wl.phi_w)
    np.testing.assert_allclose(tau[4][cw == 1], tw * np.cos(theta), rtol=1e-13)
    np.testing.assert_allclose(tau[5][cw == 1], tw * np.sin(theta), rtol=1e-13)
    for c in range(4):
        assert np.abs(tau[c][cu == 1]).max() < 1e-14
        assert (tau[c][cu >= 2] == 0).all() and (tau[c][cu == 0] == 7.0).all()
    for c in (4, 5):
        assert (tau[c][cw >= 2] == 0).all() and (tau[c][cw == 0] == 7.0).all()
    assert stats[3] == (cu == 1).sum() + (cw == 1).sum()
    np.testing.assert_allclose(stats[1], tw * (cw == 1).sum(), rtol=1e-12)


def _positions(g, kind):
    x = np.arange(g.nx)[None, None, :] * g.dx
    y = np.arange(g.ny)[None, :, None] * g.dy
    z = (np.arange(g.nz)[:, None, None] + (0.5 if kind == 0 else 0.0)) * g.dz
    return x + 0 * y + 0 * z, y + 0 * x + 0 * z, z + 0 * x + 0 * y


def _unit(rng, zmin=0.6):
    while True:
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        if v[2] > zmin:
            return v


def test_step2_linear_field_reproduced(ora):
    """Tilted planes: every component linear in the position of its own node
    set; phi_c = 2 keeps both samples' stencils outside the body (a 1-Lipschitz
    phi drops by at most sqrt(3) over a stencil), so the extrapolated solid
    band equals the linear field; body nodes hold a marker that must not leak."""
    rng = np.random.default_rng(21)
    g = Grid(24, 22, 16)
    b, phi_c = 1.5, 2.0
    checked = 0
    for _ in range(6):
        n_hat = _unit(rng)
        pu, pw = terrain.plane(g, (12.0, 11.0, 6.0), n_hat)
        tau, expect = [], []
        for c in range(6):
            kind = 0 if c < 4 else 1
            X, Y, Z = _positions(g, kind)
            cf = rng.standard_normal(4)
            lin = cf[0] + cf[1] * X + cf[2] * Y + cf[3] * Z
            phi = pu if kind == 0 else pw
            tau.append(np.where(phi >= 0, lin, 1e6))
            expect.append(lin)
        out = ora.chester_extrapolate(g, b, phi_c, pu, pw, tau)
        for c in range(6):
            phi = pu if c < 4 else pw
            sb = (phi < 0) & (phi >= -b)
            # nodes whose samples reach the periodic seam of the (non-periodic) plane
            kk, jj, ii = np.nonzero(sb)
            keep = (ii >= 6) & (ii < g.nx - 6) & (jj >= 6) & (jj < g.ny - 6)
            got = out[c][kk[keep], jj[keep], ii[keep]]
            ref = expect[c][kk[keep], jj[keep], ii[keep]]
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10 * (1 + np.abs(ref).max()))
            checked += keep.sum()
            # every other node is unchanged
            np.testing.assert_array_equal(out[c][~sb], tau[c][~sb])
    assert checked > 1000


@pytest.mark.parametrize("zw,b,phi_c", [(3.0, 1.5, 1.5), (3.25, 1.5, 2.0), (2.75, 1.0, 1.25)])
def test_step2_flat_wall_quadratic(ora, zw, b, phi_c):
    """On a flat wall (n = e_z) a stress a + c z^2 on uv nodes and on w nodes
    is sampled at z_w + phi_c and z_w + 2 phi_c by vertical linear
    interpolation between node heights; the solid band gets the straight
    line through the two samples evaluated at its own height."""
    g = Grid(5, 4, 14)
    pu, pw = terrain.flat(g, zw)
    a_, c_ = 0.3, -0.7
    tau = []
    for c in range(6):
        kind = 0 if c < 4 else 1
        Z = _positions(g, kind)[2]
        phi = pu if kind == 0 else pw
        tau.append(np.where(phi >= 0, a_ + (c + 1) * c_ * Z ** 2, 0.0))
    out = ora.chester_extrapolate(g, b, phi_c, pu, pw, tau)
    for c in range(6):
        kind = 0 if c < 4 else 1
        off = 0.5 if kind == 0 else 0.0
        f = lambda z: a_ + (c + 1) * c_ * z ** 2 if z - zw >= 0 else 0.0

        def sample(z):                      # linear between the node heights around z
            t = z / g.dz - off
            k0 = int(np.floor(t))
            s = t - k0
            return (1 - s) * f((k0 + off) * g.dz) + s * f((k0 + 1 + off) * g.dz)

        t1, t2 = sample(zw + phi_c), sample(zw + 2 * phi_c)
        phi = pu if kind == 0 else pw
        for k in range(g.nz):
            ph = phi[k, 0, 0]
            if -b <= ph < 0:
                exp = t1 + (ph - phi_c) * (t2 - t1) / phi_c
                np.testing.assert_allclose(out[c][k], exp, rtol=1e-13, atol=1e-14)


def _laplacian_parts(g):
    """Dense neighbour-sum matrix M (7-point, weights 1/d^2, periodic in x
    and y, nothing outside 0 <= k < nz) and the diagonal 2 (1/dx^2 + 1/dy^2 +
    1/dz^2), for the discrete Laplacian (M - diag I)."""
    n = g.n
    M = np.zeros((n, n))
    lin = lambda i, j, k: (k * g.ny + j) * g.nx + i
    for k in range(g.nz):
        for j in range(g.ny):
            for i in range(g.nx):
                q = lin(i, j, k)
                for (di, dj, dk, wgt) in ((1, 0, 0, 1 / g.dx ** 2), (-1, 0, 0, 1 / g.dx ** 2),
                                          (0, 1, 0, 1 / g.dy ** 2), (0, -1, 0, 1 / g.dy ** 2),
                                          (0, 0, 1, 1 / g.dz ** 2), (0, 0, -1, 1 / g.dz ** 2)):
                    kk = k + dk
                    if 0 <= kk < g.nz:
                        M[q, lin((i + di) % g.nx, (j + dj) % g.ny, kk)] += wgt
    return M, 2 * (1 / g.dx ** 2 + 1 / g.dy ** 2 + 1 / g.dz ** 2)


def _random_body(g, rng, b):
    """phi drawn so that the interior (phi < -b) is a random set of nodes."""
    phi = rng.uniform(-2.5 * b, 2.0 * b, g.shape)
    return phi


def test_step3_one_sweep_matrix_form(ora):
    g = Grid(6, 4, 5, 1.0, 1.3, 0.8)
    rng = np.random.default_rng(31)
    b, omega = 1.5, 1.3
    pu, pw = _random_body(g, rng, b), _random_body(g, rng, b)
    tau = [rng.standard_normal(g.shape) for _ in range(6)]
    out = ora.chester_sor(g, b, pu, pw, omega, 1, tau)
    M, diag = _laplacian_parts(g)
    k, j, i = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    red = ((i + j + k) % 2 == 0).ravel()
    for c in range(6):
        phi = (pu if c < 4 else pw).ravel()
        inner = phi < -b
        x = tau[c].ravel().copy()
        for colour in (red, ~red):
            sel = inner & colour
            new = (1 - omega) * x + omega * (M @ x) / diag
            x[sel] = new[sel]
        np.testing.assert_allclose(out[c].ravel(), x, rtol=0, atol=1e-13)
        assert inner.sum() > 10


def test_step3_converges_to_harmonic_extension(ora):
    """8^3 with a sphere: SOR sweeps converge to the dense solve of the
    Laplace equation over the interior with every other node fixed."""
    g = Grid(8, 8, 8)
    b = 1.0
    pu, pw = terrain.sphere(g, (4.0, 4.0, 4.0), 3.2)
    rng = np.random.default_rng(32)
    tau = [rng.standard_normal(g.shape) for _ in range(6)]
    out = ora.chester_sor(g, b, pu, pw, 1.5, 400, tau)
    M, diag = _laplacian_parts(g)
    A = M - diag * np.eye(g.n)
    for c in range(6):
        phi = (pu if c < 4 else pw).ravel()
        I = phi < -b
        B = ~I
        assert I.sum() > 20
        x = tau[c].ravel().copy()
        x[I] = np.linalg.solve(A[np.ix_(I, I)], -A[np.ix_(I, B)] @ x[B])
        np.testing.assert_allclose(out[c].ravel(), x, rtol=0, atol=1e-11)


def test_step3_linear_field_fixed(ora):
    g = Grid(8, 6, 12)
    b = 1.0
    pu, pw = terrain.sphere(g, (4.0, 3.0, 6.0), 2.8)
    tau = []
    for c in range(6):
        Z = _positions(g, 0 if c < 4 else 1)[2]
        tau.append(0.4 - 0.9 * Z)
    out = ora.chester_sor(g, b, pu, pw, 1.7, 5, tau)
    for c in range(6):
        np.testing.assert_allclose(out[c], tau[c], rtol=0, atol=1e-13)
