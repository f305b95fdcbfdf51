"""Pins of the oracle's node classes and forcing flags (§3.3 class lists, eq. u-*-IBM).

The expected values are the hand-derived layer table in
``tests/golden/flat_wall_layers.txt`` and the interval end points written in
§3.3, not a re-evaluation of the oracle's own comparisons.
"""
import os

import numpy as np
import pytest

from workloads import Grid, terrain

GOLD = os.path.join(os.path.dirname(__file__), "golden", "flat_wall_layers.txt")


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
    b, zw, uvb, uvs, uvf, wb, ws, wf = row
    g = Grid(6, 5, 9)
    pu, pw = terrain.flat(g, zw)
    mask = ora.classify(g, b, pu, pw)
    cols = g.nx * g.ny
    uvc = mask & 3
    wc = (mask >> 2) & 3
    assert (uvc == 1).sum() == uvb * cols
    assert (uvc == 2).sum() == uvs * cols
    assert ((mask >> 4) & 1).sum() == uvf * cols
    assert (wc == 1).sum() == wb * cols
    assert (wc == 2).sum() == ws * cols
    assert ((mask >> 5) & 1).sum() == wf * cols
    cnt = ora.counts(g, b, pu, pw)
    assert list(cnt) == [(g.nz - uvb - uvs) * cols, uvb * cols, uvs * cols,
                         (g.nz - wb - ws) * cols, wb * cols, ws * cols]


# (phi, expected class) at the interval end points of §3.3, band width 1.5 (phi_b = 0.75)
UV_ENDS = [(-1e-300, 2), (-0.0, 1), (0.0, 1), (1.5, 1), (np.nextafter(1.5, 2), 0), (1e300, 0),
           (-1e300, 2), (0.7, 1)]
W_ENDS = [(np.nextafter(-0.75, -1), 2), (-0.75, 1), (0.0, 1), (0.75, 1),
          (np.nextafter(0.75, 1), 0), (-5.0, 2), (5.0, 0)]


@pytest.mark.parametrize("phi,cls", UV_ENDS)
def test_uv_interval_ends(ora, phi, cls):
    assert ora.uv_class(phi, 1.5) == cls


@pytest.mark.parametrize("phi,cls", W_ENDS)
def test_w_interval_ends(ora, phi, cls):
    assert ora.w_class(phi, 1.5) == cls


def test_forcing_flag_includes_zero(ora):
    """phi <= 0 is forced (eq. f-IB uses the closed bound) on each grid separately."""
    g = Grid(2, 1, 1)
    pu = np.array([0.0, 1e-300]).reshape(1, 1, 2)
    pw = np.array([-0.0, 1e-300]).reshape(1, 1, 2)
    m = ora.classify(g, 1.5, pu, pw).ravel()
    assert [(x >> 4) & 1 for x in m] == [1, 0]
    assert [(x >> 5) & 1 for x in m] == [1, 0]


def test_cube_counts_closed_form(ora):
    """Side-8 cube on a floor at z_f = 1 (grid spacing 1, band width 1.5).

    Solid uv nodes: the floor layer k=0 everywhere, plus the cube's interior
    uv nodes strictly inside the box: x, y on the 9x9 closed footprint nodes
    with phi < 0 (faces give phi = 0, which is band), z = k + 1/2 in (1, 9)
    -> k = 1..8.  Interior nodes: 7x7 in x, y (faces excluded) x 8 layers.
    """
    from workloads import configs
    wl = configs.cube()
    g = wl.grid
    cnt = ora.counts(g, 1.5, wl.phi_uv, wl.phi_w)
    assert cnt[2] == g.nx * g.ny + 7 * 7 * 8
    # w grid: solid phi_w < -0.75.  Floor: k=0 (phi=-1) everywhere outside the footprint;
    # below the footprint, k=0 nodes have depth min(9, sqrt(dh^2 + 1)) >= 1 -> solid.
    # Inside the box, w nodes at z = k in [1, 8]: depth min(9 - k, dh) with dh the
    # distance to the nearest side face; dh >= 1 for the 7x7 interior footprint nodes
    # and 9 - k >= 1 for k <= 8, so all 7x7 x 8 interior nodes are solid.
    assert cnt[5] == g.nx * g.ny + 7 * 7 * 8
