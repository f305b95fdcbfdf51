"""Seeded flow fields: log-profile velocity with noise, SGS stress, pressure gradient.

The mean velocity follows the equilibrium log law of §4.1 (eq. log-law-u),
u / u_* = ln(eta / z0) / kappa with eta the height above the local surface,
and is zero where eta <= z0.  Gaussian noise is added to every node of u, v
and w.  Draw order from the generator is fixed: u, v, w noise, then the six
stress components, then the three pressure-gradient components.
"""
import numpy as np

from .grid import Grid, node_z


def log_profile(eta, z0, kappa=0.4, ustar=1.0):
    eta = np.asarray(eta, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = (ustar / kappa) * np.log(eta / z0)
    return np.where(eta > z0, u, 0.0)


def velocity(g: Grid, rng, surface, z0, kappa=0.4, noise=0.1, theta=0.0, ustar=1.0):
    """u, v on uv nodes and w on w nodes.  ``surface`` is the surface height,
    a scalar or a (ny, nx) array of column heights."""
    zs = np.broadcast_to(np.asarray(surface, dtype=np.float64), (g.ny, g.nx))
    eta = node_z(g, "uv")[:, None, None] - zs[None]
    mean = log_profile(eta, z0, kappa, ustar)
    u = mean * np.cos(theta)
    v = mean * np.sin(theta)
    w = np.zeros(g.shape)
    if noise:
        u = u + noise * rng.standard_normal(g.shape)
        v = v + noise * rng.standard_normal(g.shape)
        w = w + noise * rng.standard_normal(g.shape)
    return (np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(w))


def sgs_stress(g: Grid, rng, std=0.01):
    """Six independent N(0, std^2) fields in the order xx, yy, zz, xy, xz, yz."""
    return [std * rng.standard_normal(g.shape) for _ in range(6)]


def pressure_gradient(g: Grid, rng, std=0.1):
    """dp/dx, dp/dy (uv nodes) and dp/dz (w nodes), N(0, std^2)."""
    return [std * rng.standard_normal(g.shape) for _ in range(3)]
