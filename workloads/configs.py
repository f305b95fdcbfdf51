"""The five synthetic workloads, plus the flat-wall family used by the pins.

Grid spacing is 1 cell in every direction, the floor is at z_f = 1 (a wall on
the w grid, case 1 of §4.1), kappa = 0.4 (§2.2), band width 2 phi_b = 1.5 and
sample distance phi_c = 1.5.  Generators are ``numpy.random.Generator(
PCG64(200603343 + cfg))`` with cfg = 1..5 in the order below.

=====  ==================  ===============================================
cfg    shape (nx,ny,nz)    terrain
=====  ==================  ===============================================
1      64 x 32 x 32        cube [16,24] x [12,20] x [1,9] on the floor
2      256 x 128 x 128     cos^2 ridge, H=16, L=40, centre x0=64
3      512 x 256 x 256     cos^2 hill, H=32, L=80, centre (128, 128)
4      64 cases            1-6 periodic Gaussian bumps on uneven grids
5      256 x 128 x 128     fractal surface (slope -2, RMS 8), per-cell log z0
=====  ==================  ===============================================

Every builder takes smaller shapes too, so the same recipe drives the
small parity cases.
"""
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

from . import fields, terrain
from .grid import Grid

SEED = 200603343
KAPPA = 0.4
ZF = 1.0
BAND = 1.5
PHI_C = 1.5
DT = 0.01


@dataclass
class Workload:
    name: str
    grid: Grid
    phi_uv: np.ndarray
    phi_w: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    tau: List[np.ndarray]
    gradp: Optional[List[np.ndarray]]
    band_width: float = BAND
    phi_c: float = PHI_C
    kappa: float = KAPPA
    z0: float = 1e-4
    log_z0: Optional[np.ndarray] = None
    dt: float = DT
    meta: dict = field(default_factory=dict)

    def cast(self, dtype):
        """Round every field to ``dtype`` (the stored values both sides read)."""
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=dtype)
        return replace(self, phi_uv=c(self.phi_uv), phi_w=c(self.phi_w), u=c(self.u),
                       v=c(self.v), w=c(self.w), tau=[c(t) for t in self.tau],
                       gradp=None if self.gradp is None else [c(t) for t in self.gradp],
                       log_z0=c(self.log_z0))


def _rng(cfg, offset=0):
    return np.random.Generator(np.random.PCG64(SEED + cfg + offset))


def _finish(name, g, phi, rng, surface, z0, noise=0.1, tau_std=0.01, gp_std=0.1,
            log_z0=None, theta=0.0, meta=None):
    u, v, w = fields.velocity(g, rng, surface, z0, KAPPA, noise, theta)
    tau = fields.sgs_stress(g, rng, tau_std) if tau_std else [np.zeros(g.shape) for _ in range(6)]
    gp = fields.pressure_gradient(g, rng, gp_std) if gp_std else None
    return Workload(name, g, phi[0], phi[1], u, v, w, tau, gp, z0=z0, log_z0=log_z0,
                    meta=meta or {})


def cube(nx=64, ny=32, nz=32, seed_offset=0):
    """cfg 1: a side-8 cube on the floor (the wall-mounted cube of §4.2)."""
    g = Grid(nx, ny, nz)
    phi = terrain.cube_on_floor(g, ZF, 16.0, 24.0, 12.0, 20.0, 9.0)
    z0 = 1e-4 * 8.0
    return _finish("cube", g, phi, _rng(1, seed_offset), ZF, z0)


def ridge(nx=256, ny=128, nz=128, H=16.0, L=40.0, x0=64.0, seed_offset=0):
    """cfg 2: 2-D cos^2 ridge (§4.3), z0/H = 1e-4."""
    g = Grid(nx, ny, nz)
    phi = terrain.ridge(g, H, L, x0, ZF)
    zs = terrain.ridge_surface(g, H, L, x0, ZF)
    return _finish("ridge", g, phi, _rng(2, seed_offset), zs, 1e-4 * H)


def hill(nx=512, ny=256, nz=256, H=32.0, L=80.0, x0=128.0, y0=128.0, seed_offset=0):
    """cfg 3: axisymmetric cos^2 hill (§4.4), z0 = 2e-4 H."""
    g = Grid(nx, ny, nz)
    phi = terrain.hill(g, H, L, x0, y0, ZF)
    zs = terrain.hill_surface(g, H, L, x0, y0, ZF)
    return _finish("hill", g, phi, _rng(3, seed_offset), zs, 2e-4 * H)


ENSEMBLE_SHAPES = ((64, 64, 64), (128, 64, 64), (256, 128, 64), (256, 128, 128))


def ensemble_shapes(ncases=64, shapes=ENSEMBLE_SHAPES):
    rng = _rng(4)
    pick = rng.integers(0, len(shapes), ncases)
    return [shapes[p] for p in pick]


def bumps_case(case, shape, with_gradp=True):
    """cfg 4, one member: 1-6 Gaussian bumps, heights 4-24, widths 8-40,
    clipped at nz/2; z0 = H 10^U[-5,-3] with H the case's maximum height."""
    rng = _rng(4, 1000 + case)
    g = Grid(*shape)
    h, hx, hy = terrain.gaussian_bumps(g, rng, clip=0.5 * g.nz * g.dz)
    phi = terrain.heightfield(g, h, hx, hy, ZF)
    z0 = float(h.max()) * 10.0 ** rng.uniform(-5.0, -3.0)
    return _finish(f"bumps{case}", g, phi, rng, ZF + h, z0, gp_std=0.1 if with_gradp else 0)


def ensemble(ncases=64, shapes=ENSEMBLE_SHAPES):
    return [bumps_case(c, s) for c, s in enumerate(ensemble_shapes(ncases, shapes))]


def fractal(nx=256, ny=128, nz=128, rms=8.0, seed_offset=0):
    """cfg 5: fractal terrain with a per-cell log z0 ~ N(ln 1e-4, 0.5^2)."""
    g = Grid(nx, ny, nz)
    rng = _rng(5, seed_offset)
    h, hx, hy = terrain.fractal(g, rng, rms)
    phi = terrain.heightfield(g, h, hx, hy, ZF)
    log_z0 = np.log(1e-4) + 0.5 * rng.standard_normal(g.shape)
    return _finish("fractal", g, phi, rng, ZF + h, 1e-4, log_z0=log_z0)


def flat(g: Grid, zw, theta=0.0, z0=8e-4, noise=0.0, tau_std=0.0, gp_std=0.0,
         band_width=BAND, phi_c=PHI_C, seed=0):
    """A flat wall at zw with a pure log profile (the §4.1 offsets)."""
    phi = terrain.flat(g, zw)
    wl = _finish(f"flat{zw}", g, phi, _rng(10, seed), zw, z0, noise, tau_std, gp_std,
                 theta=theta)
    wl.band_width = band_width
    wl.phi_c = phi_c
    return wl
