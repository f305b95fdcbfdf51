"""Signed-distance fields of the paper's terrain shapes, sampled on both node sets.

phi > 0 in the fluid, phi < 0 in the solid and phi = 0 on the immersed
boundary (paper §3.1).  Every function returns ``(phi_uv, phi_w)``, two
float64 arrays of shape ``(nz, ny, nx)``.

* flat walls, tilted planes and spheres: closed forms;
* the wall-mounted cube on a floor (§4.2): exact distance to the union of the
  floor slab and the box, with periodic minimum image;
* the cos^2 ridge (§4.3, eq. hill-2d) and the axisymmetric cos^2 hill (§4.4,
  eq. hill-3d) on a floor: exact distance to the profile curve in the
  vertical (x, z) or meridional (r, z) half-plane, found by a coarse sweep of
  the curve and a safeguarded Newton refinement;
* heightfield terrains (Gaussian bumps, fractal surfaces): the first-order
  signed distance (z - z_s) / sqrt(1 + |grad z_s|^2), which is exact for
  planes, zero on the surface, has the right sign everywhere and is
  accurate to second order in the distance near the surface.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .grid import Grid, node_xy, node_z, wrap


def _full(g, arr):
    return np.ascontiguousarray(np.broadcast_to(arr, g.shape), dtype=np.float64)


# --------------------------------------------------------------------- planes
def flat(g: Grid, zw: float):
    """Horizontal wall at height zw (the flat-terrain cases of §4.1)."""
    out = []
    for which in ("uv", "w"):
        z = node_z(g, which)
        out.append(_full(g, (z - zw)[:, None, None]))
    return tuple(out)


def plane(g: Grid, point, normal):
    """Tilted plane through ``point`` with unit ``normal`` pointing into the fluid.

    Not periodic: values near the x/y seams are not a distance to one plane.
    """
    nrm = np.asarray(normal, dtype=np.float64)
    nrm = nrm / np.linalg.norm(nrm)
    x, y = node_xy(g)
    out = []
    for which in ("uv", "w"):
        z = node_z(g, which)
        phi = ((x[None, None, :] - point[0]) * nrm[0]
               + (y[None, :, None] - point[1]) * nrm[1]
               + (z[:, None, None] - point[2]) * nrm[2])
        out.append(_full(g, phi))
    return tuple(out)


def sphere(g: Grid, center, radius, solid_inside=True):
    """Sphere of ``radius`` about ``center`` (periodic minimum image in x and y)."""
    x, y = node_xy(g)
    dx = wrap(x - center[0], g.lx)[None, None, :]
    dy = wrap(y - center[1], g.ly)[None, :, None]
    out = []
    for which in ("uv", "w"):
        dz = (node_z(g, which) - center[2])[:, None, None]
        d = np.sqrt(dx * dx + dy * dy + dz * dz) - radius
        out.append(_full(g, d if solid_inside else -d))
    return tuple(out)


# ------------------------------------------------------------ cube on a floor
def cube_on_floor(g: Grid, zf, x0, x1, y0, y1, ztop):
    """Floor z < zf united with the box [x0,x1] x [y0,y1] x (-inf, ztop]."""
    x, y = node_xy(g)
    cx, cy = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
    hx, hy = 0.5 * (x1 - x0), 0.5 * (y1 - y0)
    qx = (np.abs(wrap(x - cx, g.lx)) - hx)[None, None, :]   # > 0 outside the footprint in x
    qy = (np.abs(wrap(y - cy, g.ly)) - hy)[None, :, None]
    in_foot = (qx <= 0) & (qy <= 0)
    out = []
    for which in ("uv", "w"):
        z = node_z(g, which)[:, None, None]
        # outside: distance to the floor plane and to the box
        d_box = np.sqrt(np.maximum(qx, 0) ** 2 + np.maximum(qy, 0) ** 2
                        + np.maximum(z - ztop, 0) ** 2)
        d_out = np.minimum(z - zf, d_box)
        # inside the box column: through the top, or sideways out of the footprint
        dh = np.minimum(-qx, -qy)
        d_side = np.sqrt(dh * dh + np.maximum(zf - z, 0) ** 2)
        d_in_box = np.minimum(ztop - z, d_side)
        solid = (z < zf) | (in_foot & (z < ztop))
        phi = np.where(solid, -np.where(in_foot, d_in_box, zf - z), d_out)
        out.append(_full(g, phi + 0.0))
    return tuple(out)


# ------------------------------------------------------ cos^2 ridge and hill
def cos2_height(rho, H, L):
    """H cos^2(pi rho / 2L) for |rho| < L, else 0 (eq. hill-2d / hill-3d)."""
    return np.where(np.abs(rho) < L, H * np.cos(np.pi * rho / (2.0 * L)) ** 2, 0.0)


def _cos2_d1(rho, H, L):
    return np.where(np.abs(rho) < L, -H * np.pi / (2.0 * L) * np.sin(np.pi * rho / L), 0.0)


def _cos2_d2(rho, H, L):
    return np.where(np.abs(rho) < L, -H * np.pi ** 2 / (2.0 * L * L) * np.cos(np.pi * rho / L), 0.0)


def _profile_chunk(r, z, rs, zs, H, L, zf):
    ns = rs.size
    f = (rs[None, :] - r[:, None]) ** 2 + (zs[None, :] - z[:, None]) ** 2
    jb = np.argmin(f, axis=1)
    fmin = f[np.arange(r.size), jb]
    del f
    lo = rs[np.maximum(jb - 1, 0)]
    hi = rs[np.minimum(jb + 1, ns - 1)]
    x = rs[jb].copy()
    act = np.arange(r.size)
    for _ in range(80):
        xa, ra, za, la, ha = x[act], r[act], z[act], lo[act], hi[act]
        h0 = zf + cos2_height(xa, H, L) - za
        h1 = _cos2_d1(xa, H, L)
        h2 = _cos2_d2(xa, H, L)
        fp = 2.0 * (xa - ra) + 2.0 * h0 * h1
        fpp = 2.0 + 2.0 * h1 * h1 + 2.0 * h0 * h2
        la = np.where(fp < 0, xa, la)
        ha = np.where(fp > 0, xa, ha)
        with np.errstate(divide="ignore", invalid="ignore"):
            xn = xa - fp / fpp
        ok = (fpp > 0) & (xn > la) & (xn < ha)
        xn = np.where(ok, xn, 0.5 * (la + ha))
        done = (np.abs(xn - xa) <= 1e-15 * (1.0 + np.abs(xa))) | (fp == 0)
        x[act], lo[act], hi[act] = xn, la, ha
        act = act[~done]
        if act.size == 0:
            break
    farc = (x - r) ** 2 + (zf + cos2_height(x, H, L) - z) ** 2
    d_arc = np.sqrt(np.minimum(fmin, farc))
    a = np.abs(r)
    d_floor = np.where(a >= L, np.abs(z - zf), np.hypot(L - a, z - zf))
    d = np.minimum(d_arc, d_floor)
    surf = zf + cos2_height(r, H, L)
    return np.where(z >= surf, d, -d)


def profile_signed_distance(rho0, z0, H, L, zf, step=1.0, chunk=1 << 15):
    """Signed distance from half-plane points (rho0, z0) to the curve
    z = zf + H cos^2(pi rho / 2L) (|rho| <= L), z = zf elsewhere.

    A sweep over curve samples ``step`` apart picks the basin; a safeguarded
    Newton iteration on the squared distance, kept inside the bracket of the
    neighbouring samples, converges to the closest point.
    """
    rho0 = np.asarray(rho0, dtype=np.float64).ravel()
    z0 = np.asarray(z0, dtype=np.float64).ravel()
    out = np.empty_like(rho0)
    ns = int(np.ceil(2.0 * L / step)) + 1
    rs = np.linspace(-L, L, ns)
    zs = zf + cos2_height(rs, H, L)

    def work(s):
        out[s:s + chunk] = _profile_chunk(rho0[s:s + chunk], z0[s:s + chunk], rs, zs, H, L, zf)

    starts = range(0, rho0.size, chunk)
    workers = max(1, min(16, os.cpu_count() or 1))
    if rho0.size <= chunk or workers == 1:
        for s in starts:
            work(s)
    else:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(work, starts))
    return out


def ridge(g: Grid, H, L, x0, zf):
    """2-D cos^2 ridge centred at x0 on a floor at zf, uniform in y (§4.3)."""
    x, _ = node_xy(g)
    rho = wrap(x - x0, g.lx)
    out = []
    for which in ("uv", "w"):
        z = node_z(g, which)
        R, Z = np.meshgrid(rho, z)                     # (nz, nx)
        phi = profile_signed_distance(R, Z, H, L, zf).reshape(g.nz, 1, g.nx)
        out.append(_full(g, phi))
    return tuple(out)


def ridge_surface(g: Grid, H, L, x0, zf):
    x, _ = node_xy(g)
    zs = zf + cos2_height(wrap(x - x0, g.lx), H, L)
    return np.broadcast_to(zs[None, :], (g.ny, g.nx)).copy()


def hill(g: Grid, H, L, x0, y0, zf):
    """Axisymmetric cos^2 hill centred at (x0, y0) on a floor at zf (§4.4).

    The closest point of a surface of revolution lies in the meridional
    half-plane of the query point, so phi depends on (r, z) only; distinct
    radii are solved once.
    """
    x, y = node_xy(g)
    dx = wrap(x - x0, g.lx)[None, :]
    dy = wrap(y - y0, g.ly)[:, None]
    r2 = dx * dx + dy * dy                            # (ny, nx)
    ur2, inv = np.unique(r2.ravel(), return_inverse=True)
    ur = np.sqrt(ur2)
    out = []
    for which in ("uv", "w"):
        z = node_z(g, which)
        R, Z = np.meshgrid(ur, z)                      # (nz, nr)
        table = profile_signed_distance(R, Z, H, L, zf).reshape(g.nz, ur.size)
        out.append(np.ascontiguousarray(table[:, inv].reshape(g.shape)))
    return tuple(out)


def hill_surface(g: Grid, H, L, x0, y0, zf):
    x, y = node_xy(g)
    dx = wrap(x - x0, g.lx)[None, :]
    dy = wrap(y - y0, g.ly)[:, None]
    return zf + cos2_height(np.sqrt(dx * dx + dy * dy), H, L)


# ------------------------------------------------------ heightfield terrains
def gaussian_bumps(g: Grid, rng, nb_range=(1, 6), amp_range=(4.0, 24.0),
                   sigma_range=(8.0, 40.0), clip=None, images=4):
    """Periodic sum of Gaussian bumps; returns (h, dh/dx, dh/dy) on the (ny, nx) columns."""
    nb = int(rng.integers(nb_range[0], nb_range[1] + 1))
    amp = rng.uniform(amp_range[0], amp_range[1], nb)
    sig = rng.uniform(sigma_range[0], sigma_range[1], nb)
    cx = rng.uniform(0.0, g.lx, nb)
    cy = rng.uniform(0.0, g.ly, nb)
    x, y = node_xy(g)
    h = np.zeros((g.ny, g.nx))
    hx = np.zeros_like(h)
    hy = np.zeros_like(h)
    for b in range(nb):
        for mx in range(-images, images + 1):
            ddx = (x - cx[b] - mx * g.lx)[None, :]
            for my in range(-images, images + 1):
                ddy = (y - cy[b] - my * g.ly)[:, None]
                e = amp[b] * np.exp(-(ddx * ddx + ddy * ddy) / (2.0 * sig[b] ** 2))
                h += e
                hx += -ddx / sig[b] ** 2 * e
                hy += -ddy / sig[b] ** 2 * e
    if clip is not None:
        top = h > clip
        h = np.where(top, clip, h)
        hx = np.where(top, 0.0, hx)
        hy = np.where(top, 0.0, hy)
    return h, hx, hy


def fractal(g: Grid, rng, rms=8.0):
    """Periodic random surface with |h_hat(k)| ~ |k|^-1 (2-D spectrum slope -2),
    scaled to the given RMS and shifted so that its minimum is 0."""
    kx = 2.0 * np.pi * np.fft.fftfreq(g.nx, g.dx)[None, :]
    ky = 2.0 * np.pi * np.fft.fftfreq(g.ny, g.dy)[:, None]
    kk = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(kk)
    amp[kk > 0] = 1.0 / kk[kk > 0]
    if g.nx % 2 == 0:
        amp[:, g.nx // 2] = 0.0
    if g.ny % 2 == 0:
        amp[g.ny // 2, :] = 0.0
    coef = amp * (rng.standard_normal((g.ny, g.nx)) + 1j * rng.standard_normal((g.ny, g.nx)))
    h = np.real(np.fft.ifft2(coef))
    hx = np.real(np.fft.ifft2(1j * kx * coef))
    hy = np.real(np.fft.ifft2(1j * ky * coef))
    s = rms / np.sqrt(np.mean((h - h.mean()) ** 2))
    h, hx, hy = h * s, hx * s, hy * s
    return h - h.min(), hx, hy


def heightfield(g: Grid, h, hx, hy, zf):
    """First-order signed distance to the surface z = zf + h(x, y)."""
    scale = 1.0 / np.sqrt(1.0 + hx * hx + hy * hy)
    out = []
    for which in ("uv", "w"):
        z = node_z(g, which)[:, None, None]
        out.append(_full(g, (z - zf - h[None]) * scale[None]))
    return tuple(out)
