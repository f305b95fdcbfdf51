"""Pins of the oracle's normals (§3.1) and its second-order interpolation (§3.3).

Normals: a linear phi must give its exact unit gradient (central and
one-sided differences are exact on linear data); on a sphere the error must
fall as the second power of the resolution.  Interpolation: linear fields
are reproduced exactly, and values equal a brute-force hat-function sum over
all nodes with periodic images in x and y and a clamped vertical coordinate.
"""
import itertools

import numpy as np
import pytest

from workloads import Grid, terrain

TILTS = [(0.0, 0.0, 1.0), (0.3, 0.1, 1.0), (-0.5, 0.4, 0.8), (0.9, -0.7, 0.4), (0.0, 1.0, 1.0),
         (1.0, 0.0, 0.2)]


@pytest.mark.parametrize("nrm", TILTS)
def test_plane_normals_exact(ora, nrm):
    g = Grid(16, 14, 12, 1.0, 0.7, 1.3)
    n_hat = np.array(nrm) / np.linalg.norm(nrm)
    pu, pw = terrain.plane(g, (8.0, 6.0, 7.0), n_hat)
    for phi in (pu, pw):
        for (i, j, k) in [(5, 5, 0), (7, 6, 5), (9, 8, 11), (3, 4, 1), (12, 10, 10)]:
            n = ora.normal(g, phi, i, j, k)
            assert np.allclose(n, n_hat, atol=2e-15, rtol=0)


def test_constant_phi_gives_ez(ora):
    g = Grid(4, 4, 4)
    n = ora.normal(g, np.full(g.shape, 3.0), 1, 2, 1)
    assert list(n) == [0.0, 0.0, 1.0]


def test_sphere_normal_second_order(ora):
    errs = []
    for R in (4.0, 8.0, 16.0):
        N = int(2 * R + 12)
        g = Grid(N, N, N)
        c = (N / 2 + 0.31, N / 2 - 0.17, N / 2 + 0.23)
        pu, _ = terrain.sphere(g, c, R)
        err = 0.0
        band = np.argwhere(np.abs(pu) <= 1.0)
        for (k, j, i) in band[:: max(1, len(band) // 200)]:
            x = np.array([i, j, k + 0.5]) - c
            exact = x / np.linalg.norm(x)
            err = max(err, np.linalg.norm(ora.normal(g, pu, i, j, k) - exact))
        errs.append(err)
    # each doubling of R (in cells) cuts the error by about 4 (second order)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    assert errs[0] < 0.05


def _hat_sum(g, f, kind, p):
    """Brute force: sum over every node of f * prod(max(0, 1 - |xi - node|)),
    x/y over periodic images, z index coordinate clamped to [0, nz-1]."""
    xi = p[0] / g.dx
    yi = p[1] / g.dy
    zi = p[2] / g.dz - (0.5 if kind == 0 else 0.0)
    zi = min(max(zi, 0.0), g.nz - 1)
    tot = 0.0
    for k in range(g.nz):
        wz = max(0.0, 1 - abs(zi - k))
        if wz == 0:
            continue
        for j in range(g.ny):
            wy = sum(max(0.0, 1 - abs(yi - (j + m * g.ny))) for m in (-2, -1, 0, 1, 2))
            if wy == 0:
                continue
            for i in range(g.nx):
                wx = sum(max(0.0, 1 - abs(xi - (i + m * g.nx))) for m in (-2, -1, 0, 1, 2))
                tot += f[k, j, i] * wx * wy * wz
    return tot


def test_interp_matches_hat_function_sum(ora):
    g = Grid(7, 6, 5, 1.0, 0.8, 1.2)
    rng = np.random.default_rng(7)
    f = rng.standard_normal(g.shape)
    pts = rng.uniform([-3, -3, -2], [g.lx + 3, g.ly + 3, g.nz * g.dz + 2], size=(40, 3))
    pts = np.vstack([pts, [[0, 0, 0], [g.lx - 1e-12, 0.0, 0.6], [2.0, 1.6, 4.8]]])
    for kind in (0, 1):
        for p in pts:
            assert abs(ora.interp(g, f, kind, p) - _hat_sum(g, f, kind, p)) < 1e-13


def test_interp_reproduces_linear_fields(ora):
    g = Grid(12, 10, 9, 0.9, 1.1, 0.7)
    rng = np.random.default_rng(3)
    a, b, c, d = rng.standard_normal(4)
    x = np.arange(g.nx) * g.dx
    y = np.arange(g.ny) * g.dy
    for kind, zoff in ((0, 0.5), (1, 0.0)):
        z = (np.arange(g.nz) + zoff) * g.dz
        f = a + b * x[None, None, :] + c * y[None, :, None] + d * z[:, None, None]
        f = np.ascontiguousarray(np.broadcast_to(f, g.shape))
        for _ in range(30):
            # keep off the periodic seam and inside the vertical node range
            p = rng.uniform([1.0, 1.0, (zoff + 0.1) * g.dz],
                            [(g.nx - 2) * g.dx, (g.ny - 2) * g.dy, (g.nz - 1 + zoff - 0.1) * g.dz])
            exact = a + b * p[0] + c * p[1] + d * p[2]
            assert abs(ora.interp(g, f, kind, p) - exact) < 1e-12


def test_interp_scatter_is_adjoint(ora):
    g = Grid(5, 4, 6)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(g.shape)
    for kind in (0, 1):
        for _ in range(10):
            p = rng.uniform([-2, -2, -1], [7, 6, 7])
            s = np.zeros(g.shape)
            ora.interp_scatter(g, s, kind, p, 1.7)
            assert abs(1.7 * ora.interp(g, f, kind, p) - float((s * f).sum())) < 1e-13
            assert abs(s.sum() - 1.7) < 1e-14
