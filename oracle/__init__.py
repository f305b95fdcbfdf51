"""ctypes front end of the FP64 CPU oracle (``oracle/ibm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library neither imports nor
links it.  Inputs are widened to float64 before the call, so an FP32 GPU run
is compared against the oracle fed with exactly the stored FP32 values.

Every function follows §3 of Liu & Stevens (arXiv 2006.03343):
classes (§3.3 lists), normals (§3.1), the wall model (§3.3,
eq. bc-bottom-immersed and the tensor rotation), the stress divergence
(§2.4, eqs. dudx/dudz/dwdz) and the direct forcing (§3.2, eq. u-*-IBM);
and the Smagorinsky stress with Mason's damping that feeds it (§2.2);
the AB2 update and the pressure projection around the stage (§2.4); and
Chester et al.'s original method that the paper simplifies (§1, §3.3).
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_long, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("IBM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
UV, W = 0, 1
FLUID, BAND, SOLID = 0, 1, 2


class _Grid(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int),
                ("dx", c_double), ("dy", c_double), ("dz", c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("band_width", c_double), ("phi_c", c_double), ("kappa", c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run oracle/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp = c_void_p
        L.ora_uv_class.argtypes = [c_double, c_double]
        L.ora_w_class.argtypes = [c_double, c_double]
        L.ora_classify.argtypes = [vp, vp, vp, vp, vp]
        L.ora_normal.argtypes = [vp, vp, c_long, c_long, c_long, vp]
        L.ora_interp.argtypes = [vp, vp, c_int, vp]
        L.ora_interp.restype = c_double
        L.ora_interp_scatter.argtypes = [vp, vp, c_int, vp, c_double]
        L.ora_local_stress.argtypes = [vp, vp, vp, c_int, c_long, c_long, c_long, vp, vp, vp,
                                       c_double, vp, vp, vp]
        L.ora_wall_stress.argtypes = [vp, vp, vp, vp, vp, vp, vp, c_double, vp, vp, vp]
        L.ora_divergence.argtypes = [vp, vp, vp]
        L.ora_divergence_transpose.argtypes = [vp, vp, vp]
        L.ora_forcing.argtypes = [vp, vp, vp, vp, vp, c_double]
        L.ora_drag.argtypes = [vp, vp, vp, vp, vp]
        L.ora_counts.argtypes = [vp, vp, vp, vp, vp]
        L.ora_stage_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, c_double, vp, vp, vp, vp, vp,
                                    vp, vp, vp, vp]
        L.ora_smagorinsky.argtypes = [vp, c_double, c_double, vp, vp, vp, vp, vp, c_double, vp,
                                      vp]
        L.ora_chester_class.argtypes = [c_double, c_double]
        L.ora_chester_counts.argtypes = [vp, vp, vp, vp, vp]
        L.ora_chester_wall_stress.argtypes = [vp, vp, vp, vp, vp, vp, vp, c_double, vp, vp, vp]
        L.ora_chester_extrapolate.argtypes = [vp, vp, vp, vp, vp]
        L.ora_chester_sor.argtypes = [vp, vp, vp, vp, c_double, c_int, vp]
        L.ora_num_threads.restype = c_int
        L.ora_set_threads.argtypes = [c_int]
        _lib = L
    return _lib


def num_threads():
    return lib().ora_num_threads()


def set_threads(n):
    """OpenMP threads of the following calls (for timing)."""
    lib().ora_set_threads(int(n))


# ------------------------------------------------------------------ helpers
def _grid(g):
    return _Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz)


def _params(band_width, phi_c, kappa=0.4):
    return _Params(band_width, phi_c, kappa)


def _f64(a, g=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if g is not None and a.shape != (g.nz, g.ny, g.nx):
        a = np.ascontiguousarray(a.reshape(g.nz, g.ny, g.nx))
    return a


def _p(a):
    return None if a is None else a.ctypes.data


def _parr(arrs):
    return (c_void_p * len(arrs))(*[_p(a) for a in arrs])


# ------------------------------------------------------------------- wrappers
def uv_class(phi, band_width):
    return lib().ora_uv_class(float(phi), float(band_width))


def w_class(phi, band_width):
    return lib().ora_w_class(float(phi), float(band_width))


def classify(g, band_width, phi_uv, phi_w, phi_c=None):
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    mask = np.empty(g.shape, dtype=np.uint8)
    gr, pr = _grid(g), _params(band_width, phi_c or band_width)
    lib().ora_classify(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), _p(mask))
    return mask


def counts(g, band_width, phi_uv, phi_w):
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    out = np.zeros(6, dtype=np.int64)
    gr, pr = _grid(g), _params(band_width, band_width)
    lib().ora_counts(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), _p(out))
    return out


def normal(g, phi, i, j, k):
    ph = _f64(phi, g)
    n = np.zeros(3)
    gr = _grid(g)
    lib().ora_normal(ctypes.byref(gr), _p(ph), i, j, k, _p(n))
    return n


def interp(g, f, kind, p):
    ff = _f64(f, g)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    gr = _grid(g)
    return lib().ora_interp(ctypes.byref(gr), _p(ff), kind, _p(pp))


def interp_scatter(g, f, kind, p, value):
    """Adds value * weights into the float64 array ``f`` in place."""
    assert f.dtype == np.float64 and f.flags.c_contiguous
    pp = np.ascontiguousarray(p, dtype=np.float64)
    gr = _grid(g)
    lib().ora_interp_scatter(ctypes.byref(gr), _p(f), kind, _p(pp), float(value))


def local_stress(g, band_width, phi_c, kappa, phi, kind, i, j, k, u, v, w, ln_ratio):
    ph, uu, vv, ww = (_f64(a, g) for a in (phi, u, v, w))
    tau = np.zeros(9)
    tw = c_double()
    U = c_double()
    gr, pr = _grid(g), _params(band_width, phi_c, kappa)
    lib().ora_local_stress(ctypes.byref(gr), ctypes.byref(pr), _p(ph), kind, i, j, k, _p(uu),
                           _p(vv), _p(ww), float(ln_ratio), _p(tau), ctypes.byref(tw),
                           ctypes.byref(U))
    return tau.reshape(3, 3), tw.value, U.value


def wall_stress(g, band_width, phi_c, kappa, phi_uv, phi_w, u, v, w, z0, log_z0, tau):
    """Returns (tau_out list of 6 arrays, stats[4]); inputs are not modified."""
    pu, pw, uu, vv, ww = (_f64(a, g) for a in (phi_uv, phi_w, u, v, w))
    lz = None if log_z0 is None else _f64(log_z0, g)
    t = [np.array(_f64(a, g), copy=True) for a in tau]
    stats = np.zeros(4)
    gr, pr = _grid(g), _params(band_width, phi_c, kappa)
    lib().ora_wall_stress(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), _p(uu), _p(vv),
                          _p(ww), float(z0), _p(lz), _parr(t), _p(stats))
    return t, stats


def divergence(g, tau):
    t = [_f64(a, g) for a in tau]
    div = [np.empty(g.shape) for _ in range(3)]
    gr = _grid(g)
    lib().ora_divergence(ctypes.byref(gr), _parr(t), _parr(div))
    return div


def smagorinsky(g, phi_uv, phi_w, u, v, w, z0=None, log_z0=None, cs=0.16, kappa=0.4):
    """§2.2 Smagorinsky stress with Mason damping (wall distance phi): six fields."""
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    vel = [_f64(a, g) for a in (u, v, w)]
    lz = None if log_z0 is None else _f64(log_z0, g)
    tau = [np.empty(g.shape) for _ in range(6)]
    gr = _grid(g)
    lib().ora_smagorinsky(ctypes.byref(gr), float(cs), float(kappa), _p(pu), _p(pw),
                          _p(vel[0]), _p(vel[1]), _p(vel[2]), float(z0 or 0.0),
                          None if lz is None else _p(lz), _parr(tau))
    return tau


def divergence_transpose(g, gdiv):
    gd = [_f64(a, g) for a in gdiv]
    gt = [np.zeros(g.shape) for _ in range(6)]
    gr = _grid(g)
    lib().ora_divergence_transpose(ctypes.byref(gr), _parr(gd), _parr(gt))
    return gt


def forcing(g, phi_uv, phi_w, ustar, gradp, dt):
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    us = [np.array(_f64(a, g), copy=True) for a in ustar]
    gp = None if gradp is None else [_f64(a, g) for a in gradp]
    gr = _grid(g)
    lib().ora_forcing(ctypes.byref(gr), _p(pu), _p(pw), _parr(us),
                      None if gp is None else _parr(gp), float(dt))
    return us


def drag(g, phi_uv, phi_w, div):
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    d = [_f64(a, g) for a in div]
    out = np.zeros(3)
    gr = _grid(g)
    lib().ora_drag(ctypes.byref(gr), _p(pu), _p(pw), _parr(d), _p(out))
    return out


def stage(wl, ustar=None):
    """One full pass on a ``workloads.configs.Workload``: classes, wall stress,
    divergence, forcing and drag.  ``ustar`` defaults to (u, v, w)."""
    g = wl.grid
    mask = classify(g, wl.band_width, wl.phi_uv, wl.phi_w)
    cnt = counts(g, wl.band_width, wl.phi_uv, wl.phi_w)
    tau, stats = wall_stress(g, wl.band_width, wl.phi_c, wl.kappa, wl.phi_uv, wl.phi_w,
                             wl.u, wl.v, wl.w, wl.z0, wl.log_z0, wl.tau)
    div = divergence(g, tau)
    us = forcing(g, wl.phi_uv, wl.phi_w, ustar if ustar is not None else (wl.u, wl.v, wl.w),
                 wl.gradp, wl.dt)
    dr = drag(g, wl.phi_uv, wl.phi_w, div)
    return dict(mask=mask, counts=cnt, tau=tau, stats=stats, div=div, ustar=us, drag=dr)


# ------------------------------------------- §2.4 pseudo-spectral horizontal
def spectral_derivative(f, axis, length):
    """eq. dudx: the derivative along a periodic axis of physical ``length``
    as the sum over wavenumbers of i k A_hat exp(i k x) (library FFT as the
    transform step).  For an even node count the Nyquist mode has no
    derivative (its i k A_hat term would not be real) and is dropped."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    m = np.fft.fftfreq(n, d=1.0 / n)            # mode numbers 0, 1, .., -1
    k = 2.0 * np.pi * m / length
    if n % 2 == 0:
        k[n // 2] = 0.0
    shape = [1] * f.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def divergence_spectral(g, tau):
    """The stress divergence of ``divergence`` with the horizontal derivatives
    taken pseudo-spectrally (eq. dudx) instead of by central differences; the
    vertical staggered differences (eqs. dudz, dwdz) and the zero padding at
    the ends are the same."""
    txx, tyy, tzz, txy, txz, tyz = (_f64(a, g) for a in tau)
    ddx = lambda a: spectral_derivative(a, 2, g.nx * g.dx)
    ddy = lambda a: spectral_derivative(a, 1, g.ny * g.dy)

    def above(a):                 # a[k + 1], zero above the top plane
        out = np.zeros_like(a)
        out[:-1] = a[1:]
        return out

    def below(a):                 # a[k - 1], zero below the bottom plane
        out = np.zeros_like(a)
        out[1:] = a[:-1]
        return out

    div_x = ddx(txx) + ddy(txy) + (above(txz) - txz) / g.dz
    div_y = ddx(txy) + ddy(tyy) + (above(tyz) - tyz) / g.dz
    div_z = ddx(txz) + ddy(tyz) + (tzz - below(tzz)) / g.dz
    return [div_x, div_y, div_z]


def stage_spectral(wl, ustar=None):
    """``stage`` with the pseudo-spectral horizontal derivatives."""
    out = stage(wl, ustar)
    g = wl.grid
    out["div"] = divergence_spectral(g, out["tau"])
    out["drag"] = drag(g, wl.phi_uv, wl.phi_w, out["div"])
    return out


# ------------------------------------ §2.4 AB2 update and pressure projection
def ab2_predict(u, rhs_now, rhs_prev, dt):
    """eq. u-inter: u* = u + dt (3/2 RHS'^t - 1/2 RHS^(t - dt)), per component."""
    return [np.asarray(a, np.float64) + dt * (1.5 * np.asarray(b, np.float64)
                                              - 0.5 * np.asarray(c, np.float64))
            for a, b, c in zip(u, rhs_now, rhs_prev)]


def _wavenumbers(n, length):
    """2 pi m / L for the FFT ordering of modes, the Nyquist mode of an even
    count set to 0 (as in ``spectral_derivative``)."""
    m = np.fft.fftfreq(n, d=1.0 / n)
    k = 2.0 * np.pi * m / length
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def _walls(nz):
    """Indices of the two wall w nodes: k = 0 on the floor (z = 0) and
    k = nz - 1 on the lid (z = (nz - 1) dz = Lz by eq. dxdydz)."""
    return 0, nz - 1


def divergence_velocity(g, u, v, w):
    """Discrete divergence D of a velocity on the staggered grid, on the uv
    layers k = 0 .. nz-2, the cells between the w nodes k and k + 1:
    pseudo-spectral du/dx + dv/dy (eq. dudx) plus (w[k+1] - w[k]) / dz
    (eq. dwdz), with w as given on the wall nodes.  The uv layer nz-1 lies
    above the lid at z = (nz - 1/2) dz > Lz, outside the domain: its entry is
    0."""
    u, v, w = (_f64(a, g) for a in (u, v, w))
    d = np.zeros(g.shape)
    if g.nz < 2:
        return d
    d[:-1] = (spectral_derivative(u, 2, g.nx * g.dx)[:-1]
              + spectral_derivative(v, 1, g.ny * g.dy)[:-1]
              + (w[1:] - w[:-1]) / g.dz)
    return d


def gradient_pressure(g, p, wall_gradient=None):
    """Discrete gradient G of a pressure on the uv layers: pseudo-spectral
    d/dx, d/dy on uv nodes (the layer above the lid included, where the
    caller's p is 0); (p[k] - p[k-1]) / dz on the interior w nodes
    1 <= k <= nz-2; on the two wall w nodes the wall-normal gradient of
    eq. p-bc, passed in as (bottom, top) planes (zero when None)."""
    p = _f64(p, g)
    gz = np.zeros_like(p)
    gz[1:-1] = (p[1:-1] - p[:-2]) / g.dz
    if wall_gradient is not None:
        kb, kt = _walls(g.nz)
        gz[kb] = wall_gradient[0]
        gz[kt] = wall_gradient[1]
    return [spectral_derivative(p, 2, g.nx * g.dx), spectral_derivative(p, 1, g.ny * g.dy), gz]


def pressure_poisson(g, ustar, dt):
    """eqs. p-Poisson, p-Poisson-Fourier on the uv layers k = 0 .. nz-2:
    [d2/dz2 - (kx^2 + ky^2)] p_hat = 2/(3 dt) (i kx u*_hat + i ky v*_hat +
    d/dz w_hat), where the wall w nodes enter with the value 0 that the
    projection leaves on them (eqs. bc-bottom-u3 and bc-top), and d2/dz2 is
    the vertical part of D G: the first and last rows lose their outer
    neighbour (the wall-normal gradient of eq. p-bc acts on the wall w node
    alone and does not enter the cells' equations).  Each horizontal mode is
    one tridiagonal system in z, solved here by a dense solve; a mode
    without horizontal wavenumber (kx = ky = 0 once Nyquist modes count as
    0: the mean and the Nyquist modes) is singular and takes p_hat = 0 at
    k = 0 in place of its first row.  The pressure of the layer above the
    lid is 0."""
    p = np.zeros(g.shape)
    m = g.nz - 1                                       # cells
    if m < 1:
        return p
    wb = np.array(_f64(ustar[2], g), copy=True)
    kb, kt = _walls(g.nz)
    wb[kb] = 0.0
    wb[kt] = 0.0
    rhs = 2.0 / (3.0 * dt) * divergence_velocity(g, ustar[0], ustar[1], wb)[:m]
    rh = np.fft.fft2(rhs, axes=(1, 2))                 # [m][ny][nx] complex
    kx = _wavenumbers(g.nx, g.nx * g.dx)
    ky = _wavenumbers(g.ny, g.ny * g.dy)
    c = 1.0 / g.dz ** 2
    ph = np.zeros_like(rh)
    for j in range(g.ny):
        for i in range(g.nx):
            K2 = kx[i] ** 2 + ky[j] ** 2
            A = np.zeros((m, m))
            for k in range(m):
                if k > 0:
                    A[k, k - 1] = c
                    A[k, k] -= c
                if k < m - 1:
                    A[k, k + 1] = c
                    A[k, k] -= c
                A[k, k] -= K2
            b = rh[:, j, i].copy()
            if K2 == 0.0:
                A[0, :] = 0.0
                A[0, 0] = 1.0
                b[0] = 0.0
            ph[:, j, i] = np.linalg.solve(A, b)
    p[:m] = np.real(np.fft.ifft2(ph, axes=(1, 2)))
    return p


def pressure_project(g, ustar, dt):
    """eq. u-t+1: u(t + dt) = u* - (3 dt / 2) G p, with p from
    ``pressure_poisson``.  On the wall w nodes G is the wall-normal gradient
    of eq. p-bc, the vertical momentum balance across the wall: with w = 0 on
    the wall before and after the step (eqs. bc-bottom-u3, bc-top) the
    update of eq. u-t+1 there requires dp/dz = 2 w* / (3 dt), where w* holds
    the step's vertical forcing and stress divergence at the wall.  Returns
    (u, v, w, p)."""
    p = pressure_poisson(g, ustar, dt)
    ws = _f64(ustar[2], g)
    kb, kt = _walls(g.nz)
    f = 2.0 / (3.0 * dt)
    gp = gradient_pressure(g, p, (f * ws[kb], f * ws[kt]))
    out = [_f64(a, g) - 1.5 * dt * b for a, b in zip(ustar, gp)]
    return out[0], out[1], out[2], p


# ------------------------------------------ §1: Chester et al.'s original
CH_FLUID, CH_BAND, CH_SOLID_BAND, CH_INTERIOR = 0, 1, 2, 3


def chester_class(phi, band_width):
    return lib().ora_chester_class(float(phi), float(band_width))


def chester_counts(g, band_width, phi_uv, phi_w):
    """[uv fluid, uv fluid band, uv solid band, uv interior, w ... the same]."""
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    out = np.zeros(8, dtype=np.int64)
    gr, pr = _grid(g), _params(band_width, band_width)
    lib().ora_chester_counts(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), _p(out))
    return out


def chester_wall_stress(g, band_width, phi_c, kappa, phi_uv, phi_w, u, v, w, z0, log_z0, tau):
    """Step 1 (near-wall model in the fluid band, zero for phi < 0): returns
    (tau list of 6 arrays, stats[4]); inputs are not modified."""
    pu, pw, uu, vv, ww = (_f64(a, g) for a in (phi_uv, phi_w, u, v, w))
    lz = None if log_z0 is None else _f64(log_z0, g)
    t = [np.array(_f64(a, g), copy=True) for a in tau]
    stats = np.zeros(4)
    gr, pr = _grid(g), _params(band_width, phi_c, kappa)
    lib().ora_chester_wall_stress(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), _p(uu),
                                  _p(vv), _p(ww), float(z0), _p(lz), _parr(t), _p(stats))
    return t, stats


def chester_extrapolate(g, band_width, phi_c, phi_uv, phi_w, tau):
    """Step 2 (linear extrapolation into the solid band): a new list of 6 arrays."""
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    t = [np.array(_f64(a, g), copy=True) for a in tau]
    gr, pr = _grid(g), _params(band_width, phi_c)
    lib().ora_chester_extrapolate(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), _parr(t))
    return t


def chester_sor(g, band_width, phi_uv, phi_w, omega, iterations, tau):
    """Step 3 (red-black SOR of the Laplace equation over the interior): a new
    list of 6 arrays."""
    pu, pw = _f64(phi_uv, g), _f64(phi_w, g)
    t = [np.array(_f64(a, g), copy=True) for a in tau]
    gr, pr = _grid(g), _params(band_width, band_width)
    lib().ora_chester_sor(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), float(omega),
                          int(iterations), _parr(t))
    return t


def chester_stage(wl, omega, iterations, ustar=None):
    """One pass of the original method on a ``workloads.configs.Workload``:
    the three steps, then the divergence, forcing and drag of ``stage``."""
    g = wl.grid
    tau, stats = chester_wall_stress(g, wl.band_width, wl.phi_c, wl.kappa, wl.phi_uv, wl.phi_w,
                                     wl.u, wl.v, wl.w, wl.z0, wl.log_z0, wl.tau)
    tau = chester_extrapolate(g, wl.band_width, wl.phi_c, wl.phi_uv, wl.phi_w, tau)
    tau = chester_sor(g, wl.band_width, wl.phi_uv, wl.phi_w, omega, iterations, tau)
    div = divergence(g, tau)
    us = forcing(g, wl.phi_uv, wl.phi_w, ustar if ustar is not None else (wl.u, wl.v, wl.w),
                 wl.gradp, wl.dt)
    dr = drag(g, wl.phi_uv, wl.phi_w, div)
    return dict(counts=chester_counts(g, wl.band_width, wl.phi_uv, wl.phi_w), tau=tau,
                stats=stats, div=div, ustar=us, drag=dr)


def stage_vjp(wl, g_tau, g_div, g_ustar, g_drag):
    """Reverse mode of one pass with ustar = u (see ``ora_stage_vjp``)."""
    g = wl.grid
    pu, pw, uu, vv, ww = (_f64(a, g) for a in (wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w))
    lz = None if wl.log_z0 is None else _f64(wl.log_z0, g)
    gt = None if g_tau is None else [None if a is None else _f64(a, g) for a in g_tau]
    gd = [_f64(a, g) for a in g_div]
    gs = [_f64(a, g) for a in g_ustar]
    gdr = np.ascontiguousarray(g_drag, dtype=np.float64)
    gu, gv, gw = (np.empty(g.shape) for _ in range(3))
    glz = None if lz is None else np.empty(g.shape)
    gr, pr = _grid(g), _params(wl.band_width, wl.phi_c, wl.kappa)
    lib().ora_stage_vjp(ctypes.byref(gr), ctypes.byref(pr), _p(pu), _p(pw), _p(uu), _p(vv),
                        _p(ww), float(wl.z0), _p(lz), None if gt is None else _parr(gt),
                        _parr(gd), _parr(gs), _p(gdr), _p(gu), _p(gv), _p(gw), _p(glz))
    return gu, gv, gw, glz
