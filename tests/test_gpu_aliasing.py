"""Entry points whose one launch reads some fields while writing others refuse
aliased arguments with IBM_E_ARG before anything is enqueued (the library's C
ABI called directly with raw device pointers): ibm_wall_stress (tau vs u, v,
w, log z0), ibm_apply and ibm_apply_spectral (div vs tau, gradp, ustar; ustar
vs tau), ibm_stage_vjp (gu, gv, gw, glog_z0 vs every input).  After each
refusal the outputs still hold their sentinel (nothing ran), and the
unaliased call succeeds."""
import ctypes

import numpy as np
import pytest

from _gpu import torch_dev
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    _, dev = torch_dev()
    wl = configs.cube(32, 16, 16)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ibm.Context(32, 16, 16, dtype=torch.float64, device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), 1.5)
    f = {k: T(getattr(wl, k)) for k in ("u", "v", "w")}
    f["tau"] = [T(t) for t in wl.tau]
    f["gp"] = [T(t) for t in wl.gradp]
    f["ustar"] = [f[k].clone() for k in ("u", "v", "w")]
    f["div"] = [torch.full_like(f["u"], 7.0) for _ in range(3)]
    f["lz"] = torch.full_like(f["u"], np.log(1e-3))
    return ctx, f, _lib, torch


def _ptrs(ts):
    from paper_2006_03343_amd._lib import ptr_array
    return ptr_array([t.data_ptr() if t is not None else None for t in ts])


def _stream(torch):
    return torch.cuda.current_stream().cuda_stream


def test_wall_stress_alias(setup):
    ctx, f, _lib, torch = setup
    L = ctx._lib
    u, v, w = f["u"], f["v"], f["w"]
    for bad in ([u] + f["tau"][1:], f["tau"][:5] + [w], [f["tau"][0]] * 6):
        rc = L.ibm_wall_stress(ctx._h, u.data_ptr(), v.data_ptr(), w.data_ptr(), 1e-3, None,
                               _ptrs(bad), None, _stream(torch))
        assert rc == _lib.IBM_E_ARG, rc
        assert b"alias" in L.ibm_last_error() or b"distinct" in L.ibm_last_error()
    lz = f["lz"]
    rc = L.ibm_wall_stress(ctx._h, u.data_ptr(), v.data_ptr(), w.data_ptr(), 0.0, lz.data_ptr(),
                           _ptrs([lz] + f["tau"][1:]), None, _stream(torch))
    assert rc == _lib.IBM_E_ARG
    tau = [t.clone() for t in f["tau"]]
    assert L.ibm_wall_stress(ctx._h, u.data_ptr(), v.data_ptr(), w.data_ptr(), 1e-3, None,
                             _ptrs(tau), None, _stream(torch)) == _lib.IBM_OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("spectral", [False, True])
def test_apply_alias(setup, spectral):
    ctx, f, _lib, torch = setup
    L = ctx._lib
    call = L.ibm_apply_spectral if spectral else L.ibm_apply
    tau, gp, us, dv = f["tau"], f["gp"], f["ustar"], f["div"]
    cases = [
        (tau, us, gp, [tau[0], dv[1], dv[2]]),          # div on tau
        (tau, us, gp, [dv[0], gp[1], dv[2]]),           # div on gradp
        (tau, us, gp, [dv[0], dv[1], us[2]]),           # div on ustar
        (tau, us, gp, [dv[0], dv[0], dv[2]]),           # div entries equal
        (tau, [us[0], tau[3], us[2]], gp, dv),          # ustar on tau
        (tau, [us[0], us[0], us[2]], gp, dv),           # ustar entries equal
    ]
    for t, u_, g_, d_ in cases:
        rc = call(ctx._h, _ptrs(t), _ptrs(u_), _ptrs(g_), 0.01, _ptrs(d_), None, _stream(torch))
        assert rc == _lib.IBM_E_ARG, rc
    torch.cuda.synchronize()
    assert all(bool((d == 7.0).all()) for d in dv)          # nothing ran
    us2 = [u.clone() for u in us]                      # kept alive: distinct addresses
    dv2 = [d.clone() for d in dv]
    rc = call(ctx._h, _ptrs(tau), _ptrs(us2), _ptrs(gp), 0.01, _ptrs(dv2), None, _stream(torch))
    assert rc == _lib.IBM_OK
    torch.cuda.synchronize()


def test_vjp_alias(setup):
    ctx, f, _lib, torch = setup
    L = ctx._lib
    u, v, w, lz = f["u"], f["v"], f["w"], f["lz"]
    gd = [torch.ones_like(u) for _ in range(3)]
    gs = [torch.ones_like(u) for _ in range(3)]
    gdr = (ctypes.c_double * 3)(1.0, 0.0, 0.0)
    gu, gv, gw, gl = (torch.full_like(u, 7.0) for _ in range(4))

    def call(outs, log_z0=lz):
        return L.ibm_stage_vjp(ctx._h, u.data_ptr(), v.data_ptr(), w.data_ptr(), 0.0,
                               log_z0.data_ptr(), None, _ptrs(gd), _ptrs(gs), gdr,
                               *[o.data_ptr() for o in outs], _stream(torch))
    for outs in ((u, gv, gw, gl), (gu, w, gw, gl), (gu, gv, gd[1], gl), (gu, gv, gw, lz),
                 (gu, gv, gs[0], gl), (gu, gu, gw, gl), (gu, gv, gw, gw)):
        assert call(outs) == _lib.IBM_E_ARG
    torch.cuda.synchronize()
    assert all(bool((o == 7.0).all()) for o in (gu, gv, gw, gl))
    assert call((gu, gv, gw, gl)) == _lib.IBM_OK
    torch.cuda.synchronize()
