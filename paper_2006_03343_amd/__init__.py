"""MI355X wall-modeled immersed boundary stage (Liu & Stevens, arXiv 2006.03343, §3).

A thin binding over the C ABI of ``libibm.so`` (``include/ibm.h``): argument
marshalling only.  Torch tensors provide device memory and the current
stream; every step of the stage runs in the library's HIP kernels.

    ctx = Context(nx, ny, nz, dtype=torch.float32, precision="mixed")
    ctx.prepare(phi_uv, phi_w, band_width=1.5)          # once per geometry
    ctx.wall_stress(u, v, w, tau, z0=1e-4)               # each step
    ctx.apply(tau, ustar, div, gradp=gp, dt=0.01, drag=drag)
"""
import numpy as np
import torch

from . import _lib
from ._lib import (IBM_F32, IBM_F64, IBM_GRID_UV, IBM_GRID_W, IBM_PREC_MIXED, IBM_PREC_PLAIN,
                   IbmError, IbmGrid, IbmParams, check, ptr_array)

__all__ = ["Context", "Batch", "IBMStage", "IbmError", "stage_forward"]

_DTYPES = {torch.float32: IBM_F32, torch.float64: IBM_F64}
_PREC = {"plain": IBM_PREC_PLAIN, "mixed": IBM_PREC_MIXED}


class Context:
    """One grid on one GPU: owns the library context (masks, band records)."""

    def __init__(self, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0, dtype=torch.float32,
                 precision="plain", device=None):
        self._lib = _lib.load()
        if dtype not in _DTYPES:
            raise TypeError(f"dtype must be float32 or float64, got {dtype}")
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.type != "cuda":
            raise ValueError("the IBM stage runs on a GPU device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.shape = (int(nz), int(ny), int(nx))
        self.n = int(nx) * int(ny) * int(nz)
        self.dtype = dtype
        self.precision = precision
        self.spacing = (float(dx), float(dy), float(dz))
        self._h = ctypes_void()
        g = IbmGrid(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz))
        with torch.cuda.device(self.device):
            check(self._lib.ibm_create(_byref(self._h), _byref(g), _DTYPES[dtype], _PREC[precision]))
        self.params = None

    @classmethod
    def _borrow(cls, handle, nx, ny, nz, spacing, dtype, precision, device):
        """A non-owning view of a context owned by a Batch."""
        self = cls.__new__(cls)
        self._lib = _lib.load()
        self.device, self.dtype, self.precision = device, dtype, precision
        self.shape = (int(nz), int(ny), int(nx))
        self.n = int(nx) * int(ny) * int(nz)
        self.spacing = spacing
        self._h = handle
        self._owned = False
        self.params = None
        return self

    # ------------------------------------------------------------- plumbing
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and getattr(self, "_owned", True):
            self._lib.ibm_destroy(self._h)
        self._h = ctypes_void()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _field(self, t, name, dtype=None):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, the context is on {self.device}")
        if t.dtype != (dtype or self.dtype):
            raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype or self.dtype}")
        if not t.is_contiguous() or t.numel() != self.n:
            raise ValueError(f"{name} must be contiguous with {self.n} elements {self.shape}")
        return t.data_ptr()

    def _fields(self, ts, name, count, optional=False):
        if ts is None:
            if optional:
                return None
            raise ValueError(f"{name} is required")
        ts = list(ts)
        if len(ts) != count:
            raise ValueError(f"{name} needs {count} fields")
        return [self._field(t, f"{name}[{i}]") for i, t in enumerate(ts)]

    # --------------------------------------------------------------- set-up
    def prepare(self, phi_uv, phi_w, band_width, phi_c=None, kappa=0.4):
        """Classes, normals and band records from the signed distance (once per geometry)."""
        p = IbmParams(float(band_width), float(phi_c) if phi_c else -1.0, float(kappa))
        with torch.cuda.device(self.device):
            check(self._lib.ibm_levelset_prepare(self._h, self._field(phi_uv, "phi_uv"),
                                                 self._field(phi_w, "phi_w"), _byref(p),
                                                 self._stream()))
        self.params = (float(band_width), float(phi_c) if phi_c else float(band_width), float(kappa))

    def counts(self):
        out = np.zeros(6, dtype=np.int64)
        check(self._lib.ibm_counts(self._h, out.ctypes.data_as(_lib.POINTER(_lib.c_int64))))
        return out

    def band_size(self, grid):
        n = _lib.c_int64(0)
        check(self._lib.ibm_band_size(self._h, grid, _byref(n)))
        return int(n.value)

    def band(self, grid):
        """(ascending linear indices, stored normals as float64 (n, 3)) of a grid's band nodes."""
        n = self.band_size(grid)
        idx = np.zeros(n, dtype=np.int32)
        nrm = np.zeros((n, 3), dtype=np.float64)
        check(self._lib.ibm_band_export(self._h, grid, idx.ctypes.data, nrm.ctypes.data))
        return idx, nrm

    def mask(self):
        m = np.zeros(self.shape, dtype=np.uint8)
        check(self._lib.ibm_mask_export(self._h, m.ctypes.data))
        return m

    def autotune(self, cache_path=None, force=False, batch=False):
        """Time tile shapes of the dense pass on this grid and keep the fastest
        (ibm_autotune); a JSON cache file, if given, is read and updated."""
        flags = (_lib.IBM_TUNE_FORCE if force else 0) | (_lib.IBM_TUNE_BATCH if batch else 0)
        with torch.cuda.device(self.device):
            check(self._lib.ibm_autotune(self._h, cache_path.encode() if cache_path else None,
                                         flags, self._stream()))
        return self.get_tile()

    def set_tile(self, vx, ty, kz, wpb=4):
        """Tile shape of the dense pass (speed only; see ibm_set_tile)."""
        check(self._lib.ibm_set_tile(self._h, int(vx), int(ty), int(kz), int(wpb)))

    def get_tile(self):
        out = np.zeros(4, dtype=np.int32)
        check(self._lib.ibm_get_tile(self._h, out.ctypes.data))
        return tuple(int(x) for x in out)

    # ------------------------------------------------------------ each step
    def wall_stress(self, u, v, w, tau, z0=None, log_z0=None, stats=None):
        """Wall-modeled stress written in place into ``tau`` (6 fields).
        ``stats``: optional float64 tensor of 4 on the device."""
        if (z0 is None) == (log_z0 is None):
            raise ValueError("give exactly one of z0 and log_z0")
        taus = self._fields(tau, "tau", 6)
        sp = None
        if stats is not None:
            if stats.dtype != torch.float64 or stats.numel() < 4 or stats.device != self.device:
                raise ValueError("stats must be a float64 device tensor with 4 elements")
            sp = stats.data_ptr()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_wall_stress(self._h, self._field(u, "u"), self._field(v, "v"),
                                            self._field(w, "w"), float(z0 or 0.0),
                                            self._field(log_z0, "log_z0"), ptr_array(taus), sp,
                                            self._stream()))

    def chester_prepare(self, phi_uv, phi_w):
        """Set-up of Chester et al.'s original method (after ``prepare``, same phi)."""
        with torch.cuda.device(self.device):
            check(self._lib.ibm_chester_prepare(self._h, self._field(phi_uv, "phi_uv"),
                                                self._field(phi_w, "phi_w"), self._stream()))

    def chester_counts(self):
        """[uv fluid, fluid band, solid band, interior, w ... the same]."""
        out = np.zeros(8, dtype=np.int64)
        check(self._lib.ibm_chester_counts(self._h, out.ctypes.data_as(_lib.POINTER(_lib.c_int64))))
        return out

    def chester_wall_stress(self, u, v, w, tau, omega, iterations, z0=None, log_z0=None,
                            stats=None):
        """The original method's stress in place in ``tau``: wall model in the
        fluid band, extrapolation into the solid band, ``iterations`` SOR sweeps
        over the interior."""
        if (z0 is None) == (log_z0 is None):
            raise ValueError("give exactly one of z0 and log_z0")
        taus = self._fields(tau, "tau", 6)
        sp = None
        if stats is not None:
            if stats.dtype != torch.float64 or stats.numel() < 4 or stats.device != self.device:
                raise ValueError("stats must be a float64 device tensor with 4 elements")
            sp = stats.data_ptr()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_chester_wall_stress(
                self._h, self._field(u, "u"), self._field(v, "v"), self._field(w, "w"),
                float(z0 or 0.0), self._field(log_z0, "log_z0"), ptr_array(taus), float(omega),
                int(iterations), sp, self._stream()))

    def apply(self, tau, ustar, div, gradp=None, dt=0.01, drag=None):
        """div = +div(tau); ustar forced in place where phi <= 0; drag (float64[3]) optional."""
        taus = self._fields(tau, "tau", 6)
        us = self._fields(ustar, "ustar", 3)
        dv = self._fields(div, "div", 3)
        gp = None
        if gradp is not None:
            gp = ptr_array([self._field(t, f"gradp[{i}]") for i, t in enumerate(gradp)])
        dp = None
        if drag is not None:
            if drag.dtype != torch.float64 or drag.numel() < 3 or drag.device != self.device:
                raise ValueError("drag must be a float64 device tensor with 3 elements")
            dp = drag.data_ptr()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_apply(self._h, ptr_array(taus), ptr_array(us), gp, float(dt),
                                      ptr_array(dv), dp, self._stream()))

    def stage(self, u, v, w, tau, ustar, div, z0=None, log_z0=None, gradp=None, dt=0.01,
              stats=None, drag=None):
        """``wall_stress`` then ``apply`` in one call (ibm_stage): one launch
        fewer, the same results."""
        if (z0 is None) == (log_z0 is None):
            raise ValueError("give exactly one of z0 and log_z0")
        taus = self._fields(tau, "tau", 6)
        us = self._fields(ustar, "ustar", 3)
        dv = self._fields(div, "div", 3)
        gp = None
        if gradp is not None:
            gp = ptr_array([self._field(t, f"gradp[{i}]") for i, t in enumerate(gradp)])
        sp = dp = None
        if stats is not None:
            if stats.dtype != torch.float64 or stats.numel() < 4 or stats.device != self.device:
                raise ValueError("stats must be a float64 device tensor with 4 elements")
            sp = stats.data_ptr()
        if drag is not None:
            if drag.dtype != torch.float64 or drag.numel() < 3 or drag.device != self.device:
                raise ValueError("drag must be a float64 device tensor with 3 elements")
            dp = drag.data_ptr()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_stage(self._h, self._field(u, "u"), self._field(v, "v"),
                                      self._field(w, "w"), float(z0 or 0.0),
                                      self._field(log_z0, "log_z0"), ptr_array(taus),
                                      ptr_array(us), gp, float(dt), ptr_array(dv), sp, dp,
                                      self._stream()))

    def apply_noalloc(self, tau, ustar, div, gradp=None, dt=0.01, drag=None):
        """``apply`` with its drag slots in the library's static device array
        (ibm_apply_noalloc): allocates nothing; overlapping calls on one GPU race."""
        taus = self._fields(tau, "tau", 6)
        us = self._fields(ustar, "ustar", 3)
        dv = self._fields(div, "div", 3)
        gp = None
        if gradp is not None:
            gp = ptr_array([self._field(t, f"gradp[{i}]") for i, t in enumerate(gradp)])
        dp = None
        if drag is not None:
            if drag.dtype != torch.float64 or drag.numel() < 3 or drag.device != self.device:
                raise ValueError("drag must be a float64 device tensor with 3 elements")
            dp = drag.data_ptr()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_apply_noalloc(self._h, ptr_array(taus), ptr_array(us), gp,
                                              float(dt), ptr_array(dv), dp, self._stream()))

    def apply_spectral(self, tau, ustar, div, gradp=None, dt=0.01, drag=None):
        """``apply`` with pseudo-spectral horizontal derivatives (power-of-two nx, ny)."""
        taus = self._fields(tau, "tau", 6)
        us = self._fields(ustar, "ustar", 3)
        dv = self._fields(div, "div", 3)
        gp = None
        if gradp is not None:
            gp = ptr_array([self._field(t, f"gradp[{i}]") for i, t in enumerate(gradp)])
        dp = None
        if drag is not None:
            if drag.dtype != torch.float64 or drag.numel() < 3 or drag.device != self.device:
                raise ValueError("drag must be a float64 device tensor with 3 elements")
            dp = drag.data_ptr()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_apply_spectral(self._h, ptr_array(taus), ptr_array(us), gp,
                                               float(dt), ptr_array(dv), dp, self._stream()))

    def ab2_predict(self, u, rhs_now, rhs_prev, dt, ustar):
        """ustar = u + dt (3/2 rhs_now - 1/2 rhs_prev), three components."""
        args = [ptr_array(self._fields(x, name, 3)) for x, name in
                ((u, "u"), (rhs_now, "rhs_now"), (rhs_prev, "rhs_prev"))]
        with torch.cuda.device(self.device):
            check(self._lib.ibm_ab2_predict(self._h, *args, float(dt),
                                            ptr_array(self._fields(ustar, "ustar", 3)),
                                            self._stream()))

    def pressure_project(self, ustar, dt, u_out, p_out):
        """Pressure Poisson solve and projection: u_out = ustar - (3 dt/2) G p."""
        with torch.cuda.device(self.device):
            check(self._lib.ibm_pressure_project(self._h, ptr_array(self._fields(ustar, "ustar", 3)),
                                                 float(dt),
                                                 ptr_array(self._fields(u_out, "u_out", 3)),
                                                 self._field(p_out, "p_out"), self._stream()))

    def sgs_stress(self, phi_uv, phi_w, u, v, w, tau, z0=None, log_z0=None, cs=0.16, kappa=0.4):
        """Smagorinsky stress with Mason's wall damping written into ``tau``
        (6 fields); the wall distance is phi of each node's grid."""
        if (z0 is None) == (log_z0 is None):
            raise ValueError("give exactly one of z0 and log_z0")
        taus = self._fields(tau, "tau", 6)
        with torch.cuda.device(self.device):
            check(self._lib.ibm_sgs_stress(self._h, self._field(phi_uv, "phi_uv"),
                                           self._field(phi_w, "phi_w"), self._field(u, "u"),
                                           self._field(v, "v"), self._field(w, "w"),
                                           float(z0 or 0.0), self._field(log_z0, "log_z0"),
                                           float(cs), float(kappa), ptr_array(taus),
                                           self._stream()))

    def apply_sgs(self, phi_uv, phi_w, u, v, w, tau, ustar, div, z0=None, log_z0=None, cs=0.16,
                  kappa=0.4, gradp=None, dt=0.01, drag=None):
        """``sgs_stress`` and ``apply`` in one pass: the Smagorinsky stress is
        formed on the fly; ``tau`` supplies the band values written by
        ``wall_stress``."""
        if (z0 is None) == (log_z0 is None):
            raise ValueError("give exactly one of z0 and log_z0")
        taus = self._fields(tau, "tau", 6)
        us = self._fields(ustar, "ustar", 3)
        dv = self._fields(div, "div", 3)
        gp = None
        if gradp is not None:
            gp = ptr_array([self._field(t, f"gradp[{i}]") for i, t in enumerate(gradp)])
        dp = None
        if drag is not None:
            if drag.dtype != torch.float64 or drag.numel() < 3 or drag.device != self.device:
                raise ValueError("drag must be a float64 device tensor with 3 elements")
            dp = drag.data_ptr()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_apply_sgs(self._h, self._field(phi_uv, "phi_uv"),
                                          self._field(phi_w, "phi_w"), self._field(u, "u"),
                                          self._field(v, "v"), self._field(w, "w"),
                                          float(z0 or 0.0), self._field(log_z0, "log_z0"),
                                          float(cs), float(kappa), ptr_array(taus), ptr_array(us),
                                          gp, float(dt), ptr_array(dv), dp, self._stream()))

    def vjp(self, u, v, w, g_div, g_ustar, g_drag, z0=None, log_z0=None, g_tau=None):
        """Reverse mode of one pass (ustar == u): returns (gu, gv, gw, glog_z0 or None)."""
        if (z0 is None) == (log_z0 is None):
            raise ValueError("give exactly one of z0 and log_z0")
        gd = self._fields(g_div, "g_div", 3)
        gs = self._fields(g_ustar, "g_ustar", 3)
        gt = None
        if g_tau is not None:
            gt = ptr_array([self._field(t, f"g_tau[{i}]") if t is not None else None
                            for i, t in enumerate(g_tau)])
        gdr = (_lib.c_double * 3)(*[float(x) for x in g_drag])
        gu, gv, gw = (torch.empty(self.shape, dtype=self.dtype, device=self.device) for _ in range(3))
        glz = torch.empty_like(gu) if log_z0 is not None else None
        with torch.cuda.device(self.device):
            check(self._lib.ibm_stage_vjp(self._h, self._field(u, "u"), self._field(v, "v"),
                                          self._field(w, "w"), float(z0 or 0.0),
                                          self._field(log_z0, "log_z0"), gt, ptr_array(gd),
                                          ptr_array(gs), gdr, gu.data_ptr(), gv.data_ptr(),
                                          gw.data_ptr(), glz.data_ptr() if glz is not None else None,
                                          self._stream()))
        return gu, gv, gw, glz


class Batch:
    """An ensemble of grids advanced together by three kernels whose blocks
    take work items of every case, one hipGraph launch per step (ibm_batch_*).  Bound tensors are kept alive by
    the batch until they are rebound or the batch is closed."""

    def __init__(self, grids, dtype=torch.float32, precision="plain", device=None):
        self._lib = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype, self.precision = dtype, precision
        self.grids = [tuple(g) + (1.0, 1.0, 1.0)[len(g) - 3:] for g in grids]
        arr = (IbmGrid * len(grids))(*[IbmGrid(int(g[0]), int(g[1]), int(g[2]), float(g[3]),
                                               float(g[4]), float(g[5])) for g in self.grids])
        self._h = ctypes_void()
        with torch.cuda.device(self.device):
            check(self._lib.ibm_batch_create(_byref(self._h), len(grids), arr, _DTYPES[dtype],
                                             _PREC[precision]))
        self._keep = [None] * len(grids)

    def __len__(self):
        return len(self.grids)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ibm_batch_destroy(self._h)
        self._h = ctypes_void()
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def case(self, i):
        """Non-owning Context of case i (counts, masks, band lists, tile shape)."""
        h = ctypes_void()
        check(self._lib.ibm_batch_case(self._h, int(i), _byref(h)))
        g = self.grids[i]
        return Context._borrow(h, g[0], g[1], g[2], g[3:6], self.dtype, self.precision, self.device)

    def prepare(self, phi_uv, phi_w, band_width, z0, phi_c=None, kappa=0.4):
        n = len(self.grids)
        cases = [self.case(i) for i in range(n)]
        pu = ptr_array([cases[i]._field(phi_uv[i], f"phi_uv[{i}]") for i in range(n)])
        pw = ptr_array([cases[i]._field(phi_w[i], f"phi_w[{i}]") for i in range(n)])
        z = (_lib.c_double * n)(*[float(x) for x in z0])
        p = IbmParams(float(band_width), float(phi_c) if phi_c else -1.0, float(kappa))
        with torch.cuda.device(self.device):
            check(self._lib.ibm_batch_prepare(self._h, pu, pw, _byref(p), z, self._stream()))
        self._keep = [None] * n

    def bind(self, i, u, v, w, tau, ustar, div, gradp=None, dt=0.01, log_z0=None, drag=None,
             stats=None):
        c = self.case(i)
        io = _lib.IbmCaseIO()
        io.u, io.v, io.w = c._field(u, "u"), c._field(v, "v"), c._field(w, "w")
        io.log_z0 = c._field(log_z0, "log_z0")
        for k, t in enumerate(tau):
            io.tau[k] = c._field(t, f"tau[{k}]")
        for k in range(3):
            io.ustar[k] = c._field(ustar[k], f"ustar[{k}]")
            io.div[k] = c._field(div[k], f"div[{k}]")
            io.gradp[k] = c._field(gradp[k], f"gradp[{k}]") if gradp is not None else None
        io.dt = float(dt)
        for name, t, m in (("drag", drag, 3), ("stats", stats, 4)):
            if t is not None and (t.dtype != torch.float64 or t.numel() < m or t.device != self.device):
                raise ValueError(f"{name} must be a float64 device tensor with {m} elements")
        io.drag_dev = drag.data_ptr() if drag is not None else None
        io.stats_dev = stats.data_ptr() if stats is not None else None
        check(self._lib.ibm_batch_bind(self._h, int(i), _byref(io)))
        self._keep[i] = (u, v, w, tau, ustar, div, gradp, log_z0, drag, stats)

    def tune(self, cache_path=None):
        with torch.cuda.device(self.device):
            check(self._lib.ibm_batch_tune(self._h, cache_path.encode() if cache_path else None,
                                           self._stream()))

    def run(self):
        """One step of every case without a graph."""
        with torch.cuda.device(self.device):
            check(self._lib.ibm_batch_run(self._h, self._stream()))

    def capture(self):
        """Record one step into a hipGraph.  Capture runs on a side stream (the
        null stream cannot be captured) ordered after the current stream."""
        with torch.cuda.device(self.device):
            side = torch.cuda.Stream(self.device)
            side.wait_stream(torch.cuda.current_stream(self.device))
            check(self._lib.ibm_batch_capture(self._h, side.cuda_stream))
            torch.cuda.current_stream(self.device).wait_stream(side)

    def launch(self):
        """One step of every case: one hipGraphLaunch of the captured graph."""
        with torch.cuda.device(self.device):
            check(self._lib.ibm_batch_launch(self._h, self._stream()))


def stage_forward(context, u, v, w, tau_sgs, gradp=None, dt=0.01, z0=None, log_z0=None):
    """One out-of-place pass: returns (tau (6,...), div (3,...), ustar_ib (3,...), drag (3,))."""
    tau = torch.stack(list(tau_sgs)).contiguous() if not isinstance(tau_sgs, torch.Tensor) \
        else tau_sgs.clone()
    context.wall_stress(u, v, w, list(tau), z0=z0, log_z0=log_z0)
    ustar = torch.stack([u, v, w]).contiguous()
    div = torch.empty_like(ustar)
    drag = torch.zeros(3, dtype=torch.float64, device=context.device)
    context.apply(list(tau), list(ustar), list(div), gradp=gradp, dt=dt, drag=drag)
    return tau, div, ustar, drag


class IBMStage(torch.autograd.Function):
    """Differentiable stage pass with respect to u, v, w and a per-node log z0.

    ``IBMStage.apply(context, u, v, w, log_z0, tau_sgs, gradp, dt)`` returns
    (tau, div, ustar_ib, drag).  The velocity is both sampled by the wall model
    and forced (ustar = u), out of place.  The backward is the library's
    hand-written adjoint (ibm_stage_vjp).
    """

    @staticmethod
    def forward(ctx, context, u, v, w, log_z0, tau_sgs, gradp, dt):
        tau, div, ustar, drag = stage_forward(context, u, v, w, tau_sgs, gradp, dt,
                                              log_z0=log_z0)
        ctx.context = context
        ctx.save_for_backward(u, v, w, log_z0)
        return tau, div, ustar, drag

    @staticmethod
    def backward(ctx, g_tau, g_div, g_ustar, g_drag):
        u, v, w, log_z0 = ctx.saved_tensors
        c = ctx.context
        z = lambda: torch.zeros(c.shape, dtype=c.dtype, device=c.device)
        gd = [g_div[i].contiguous() if g_div is not None else z() for i in range(3)]
        gs = [g_ustar[i].contiguous() if g_ustar is not None else z() for i in range(3)]
        gt = None if g_tau is None else [g_tau[i].contiguous() for i in range(6)]
        gdr = [0.0, 0.0, 0.0] if g_drag is None else g_drag.detach().double().cpu().tolist()
        gu, gv, gw, glz = c.vjp(u, v, w, gd, gs, gdr, log_z0=log_z0, g_tau=gt)
        return None, gu, gv, gw, glz, None, None, None


# small ctypes helpers kept local to avoid importing ctypes names everywhere
def ctypes_void():
    return _lib.c_void_p()


def _byref(x):
    return _lib.ctypes.byref(x)
