"""ibm_apply_noalloc (drag slots in the library's static device array, no
allocation) against ibm_apply on the same prepared context, through the C
ABI: div, ustar and drag equal bit for bit, on two calls in a row -- a float32
mixed ridge and then a smaller float64 cube, whose call finds the first
call's slots still in the shared array -- and the drag slots refused with
IBM_E_RANGE beyond the array's 43690 tiles (the call without drag still
runs)."""
import ctypes

import numpy as np
import pytest

from _gpu import torch_dev
from workloads import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _ptrs(ts):
    from paper_2006_03343_amd._lib import ptr_array
    return ptr_array([t.data_ptr() if t is not None else None for t in ts])


def _pair(wl, dtype, precision):
    """Both entry points on one context: (outputs of ibm_apply, of ibm_apply_noalloc)."""
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    torch, dev = torch_dev()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, tdt)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=tdt, precision=precision,
                      device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    u, v, w = T(wl.u), T(wl.v), T(wl.w)
    tau = [T(t) for t in wl.tau]
    ctx.wall_stress(u, v, w, tau, z0=wl.z0)
    gp = [T(t) for t in wl.gradp]
    s = torch.cuda.current_stream().cuda_stream
    outs = []
    for fn in (ctx._lib.ibm_apply, ctx._lib.ibm_apply_noalloc):
        us = [u.clone(), v.clone(), w.clone()]
        dv = [torch.full_like(u, float("nan")) for _ in range(3)]
        dr = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
        rc = fn(ctx._h, _ptrs(tau), _ptrs(us), _ptrs(gp), wl.dt, _ptrs(dv),
                ctypes.c_void_p(dr.data_ptr()), s)
        assert rc == _lib.IBM_OK, ctx._lib.ibm_last_error()
        torch.cuda.synchronize()
        outs.append(([d.cpu() for d in dv], [x.cpu() for x in us], dr.cpu()))
    return outs, ctx


def test_noalloc_equals_apply_twice():
    for wl, dtype, prec in ((configs.ridge(256, 128, 64), "f32", "mixed"),
                            (configs.cube(32, 16, 16), "f64", "plain")):
        g = wl.grid
        _say(f"apply_noalloc {wl.name} {g.nx}x{g.ny}x{g.nz} {dtype} {prec}")
        (ref, got), ctx = _pair(wl, dtype, prec)
        for a, b in zip(ref[0] + ref[1], got[0] + got[1]):
            assert bool((a == b).all())
        assert bool((ref[2] == got[2]).all()), (ref[2], got[2])
        assert bool(np.isfinite(got[2].numpy()).all())
        _say(f"drag {got[2].numpy()} tile {ctx.get_tile()}")


def test_noalloc_refuses_beyond_scratch():
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    torch, dev = torch_dev()
    wl = configs.cube(64, 256, 256)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    ctx = ibm.Context(64, 256, 256, dtype=torch.float32, device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), 1.5)
    ctx.set_tile(1, 1, 1, 1)                     # 65536 tiles: 196608 drag slots
    tau = [T(t) for t in wl.tau]
    us = [T(wl.u), T(wl.v), T(wl.w)]
    dv = [torch.zeros_like(us[0]) for _ in range(3)]
    dr = torch.zeros(3, dtype=torch.float64, device=dev)
    with pytest.raises(ibm.IbmError) as e:
        ctx.apply_noalloc(tau, us, dv, dt=0.01, drag=dr)
    assert e.value.code == _lib.IBM_E_RANGE
    ctx.apply_noalloc(tau, us, dv, dt=0.01)      # no drag: no slots needed
    ctx.set_tile(4, 1, 64, 1)                    # 256 tiles
    ctx.apply_noalloc(tau, us, dv, dt=0.01, drag=dr)
    torch.cuda.synchronize()
