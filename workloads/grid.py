"""Staggered uniform grid (paper §2.4, eq. dxdydz and the vertical staggering).

Fields are stored C-order ``[nz][ny][nx]`` (x fastest).  A ``uv`` node
(i, j, k) sits at (i*dx, j*dy, (k+1/2)*dz); a ``w`` node (i, j, k) sits at
(i*dx, j*dy, k*dz), half a cell below the ``uv`` node of the same index.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    @property
    def lx(self):
        return self.nx * self.dx

    @property
    def ly(self):
        return self.ny * self.dy

    @property
    def dv(self):
        return self.dx * self.dy * self.dz


def node_xy(g: Grid):
    """x (shape (nx,)) and y (shape (ny,)) node coordinates, shared by both grids."""
    return np.arange(g.nx, dtype=np.float64) * g.dx, np.arange(g.ny, dtype=np.float64) * g.dy


def node_z(g: Grid, which: str):
    """z coordinates (shape (nz,)) of the ``uv`` or ``w`` node set."""
    k = np.arange(g.nz, dtype=np.float64)
    if which == "uv":
        return (k + 0.5) * g.dz
    if which == "w":
        return k * g.dz
    raise ValueError(which)


def wrap(d, length):
    """Minimum-image displacement in a periodic direction: result in [-L/2, L/2)."""
    return d - length * np.floor(d / length + 0.5)
