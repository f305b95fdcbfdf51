"""GPU parity of the fused Smagorinsky stress and dense pass (ibm_apply_sgs).

Expected values from the oracle alone: its Smagorinsky stress (the same
function the ibm_sgs_stress tests pin) becomes the stage's input stress, then
the oracle's stage (classes, wall stress at band nodes, zero in the body,
divergence, forcing, drag).  Bars as for the stage: div normwise per component
<= 1e-12 (float64) and 2e-5 (float32), ustar likewise, drag within tol * dV *
sum |div|.  The tau buffers hold noise before ibm_wall_stress, so a read of
tau anywhere but a band node would show.  Cases: the cube, a ragged ridge
(several x segments, the last one short), the same with an odd nx, a small
hill in three
precisions, a per-node log z0 field, grids of one column, one row, one or
two planes and two rows, the 512 x 256 x 256 hill; the fused pass against
ibm_sgs_stress + ibm_wall_stress + ibm_apply on the GPU (div and ustar bit for bit),
also on 4096 x 4096 x 30 float64 and 8192 x 4096 x 30 float32 grids whose planes
shrink the chunks to 27; a 4096 x 4096 x 127 grid (near the 2^31 - 1 node limit
of a context) made of periodic copies of a hill cell, each copy equal to the
first and the first against the oracle; error paths, among them an x-y plane
beyond the pass's 32-bit reach.
"""
from dataclasses import replace

import numpy as np
import pytest

from _gpu import TOL, first_copy, normwise, tiled, torch_dev
from workloads import Grid, configs

pytestmark = pytest.mark.gpu
CS, KAPPA = 0.16, 0.4


def _say(msg):
    print(msg, flush=True)


def _run(wl, dtype, precision="plain", two_step=False, seed=3):
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, tdt)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=tdt, precision=precision,
                      device=dev)
    pu, pw = T(wl.phi_uv), T(wl.phi_w)
    ctx.prepare(pu, pw, wl.band_width, wl.phi_c, wl.kappa)
    u, v, w = T(wl.u), T(wl.v), T(wl.w)
    noise = np.random.default_rng(seed).standard_normal((6,) + g.shape) * 50.0
    tau = [T(a) for a in noise]
    lz = T(wl.log_z0) if wl.log_z0 is not None else None
    z0 = None if lz is not None else wl.z0
    ustar = [u.clone(), v.clone(), w.clone()]
    div = [torch.empty_like(u) for _ in range(3)]
    drag = torch.zeros(3, dtype=torch.float64, device=dev)
    gp = [T(t) for t in wl.gradp] if wl.gradp is not None else None
    if two_step:
        ctx.sgs_stress(pu, pw, u, v, w, tau, z0=z0, log_z0=lz, cs=CS, kappa=KAPPA)
        ctx.wall_stress(u, v, w, tau, z0=z0, log_z0=lz)
        ctx.apply(tau, ustar, div, gradp=gp, dt=wl.dt, drag=drag)
    else:
        ctx.wall_stress(u, v, w, tau, z0=z0, log_z0=lz)
        ctx.apply_sgs(pu, pw, u, v, w, tau, ustar, div, z0=z0, log_z0=lz, cs=CS, kappa=KAPPA,
                      gradp=gp, dt=wl.dt, drag=drag)
    torch.cuda.synchronize()
    return dict(div=[d.cpu().numpy() for d in div], ustar=[x.cpu().numpy() for x in ustar],
                drag=drag.cpu().numpy())


def _ref(ora, wl):
    tsgs = ora.smagorinsky(wl.grid, wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w,
                           z0=None if wl.log_z0 is not None else wl.z0, log_z0=wl.log_z0,
                           cs=CS, kappa=KAPPA)
    return ora.stage(replace(wl, tau=tsgs))


def _check(ora, wl, dtype, precision="plain"):
    got = _run(wl, dtype, precision)
    ref = _ref(ora, wl)
    errs = {}
    for c, nm in enumerate("xyz"):
        errs["div_" + nm] = normwise(got["div"][c], ref["div"][c])
        errs["ustar_" + nm] = normwise(got["ustar"][c], ref["ustar"][c])
    scale = wl.grid.dv * np.array([np.abs(d).sum() for d in ref["div"]])
    errs["drag"] = float(np.max(np.abs(got["drag"] - ref["drag"]) / np.maximum(scale, 1e-300)))
    assert max(errs.values()) <= TOL[dtype], errs
    return got, errs


def test_cube_f64(ora):
    _say("sgs+apply cube 64x32x32 f64")
    _, errs = _check(ora, configs.cube(), "f64")
    _say(f"errors {errs}")


def test_ragged_ridge(ora):
    wl = configs.ridge(100, 36, 40, H=8.0, L=20.0, x0=30.0).cast(np.float32)
    _say("sgs+apply ridge 100x36x40 f32 mixed")
    _, errs = _check(ora, wl, "f32", "mixed")
    _say(f"errors {errs}")


def test_odd_nx_float(ora):
    """Float with an odd nx: the last x segment is 39 of 60 nodes, and the lane
    pairs of the x differences wrap at an odd period."""
    wl = configs.ridge(99, 36, 40, H=8.0, L=20.0, x0=30.0).cast(np.float32)
    _say("sgs+apply ridge 99x36x40 f32 mixed (odd nx)")
    _, errs = _check(ora, wl, "f32", "mixed")
    _say(f"errors {errs}")


@pytest.mark.parametrize("dtype,prec", [("f64", "plain"), ("f32", "plain"), ("f32", "mixed")])
def test_small_hill(ora, dtype, prec):
    wl = configs.hill(128, 64, 32, H=12.0, L=30.0, x0=40.0, y0=32.0)
    if dtype == "f32":
        wl = wl.cast(np.float32)
    _say(f"sgs+apply hill 128x64x32 {dtype} {prec}")
    _, errs = _check(ora, wl, dtype, prec)
    _say(f"errors {errs}")


def test_per_node_log_z0(ora):
    wl = configs.fractal(64, 48, 40, rms=4.0).cast(np.float32)
    _say("sgs+apply fractal 64x48x40 log z0 f32 mixed")
    _, errs = _check(ora, wl, "f32", "mixed")
    _say(f"errors {errs}")


def test_degenerate_grids(ora):
    for shape, sp in (((1, 1, 12), (1.0, 1.0, 1.0)), ((7, 1, 9), (1.0, 1.0, 1.0)),
                      ((1, 6, 9), (0.5, 1.0, 1.0)), ((33, 5, 1), (1.0, 1.0, 1.0)),
                      ((20, 2, 2), (0.7, 1.3, 0.9)), ((130, 9, 7), (1.0, 1.0, 1.0))):
        g = Grid(*shape, *sp)
        wl = configs.flat(g, 1.25 * sp[2], theta=0.4, z0=1e-3, noise=0.3, tau_std=0.01,
                          gp_std=0.1, seed=shape[0])
        _say(f"sgs+apply flat {shape} spacing {sp} f64")
        _check(ora, wl, "f64")


def test_against_two_step_gpu():
    wl = configs.hill(128, 64, 40, H=16.0, L=40.0, x0=40.0, y0=32.0).cast(np.float32)
    _say("sgs+apply vs sgs_stress + wall_stress + apply, hill 128x64x40 f32 mixed")
    a = _run(wl, "f32", "mixed")
    b = _run(wl, "f32", "mixed", two_step=True)
    for c in range(3):
        # the two kernels share the stress formula and the divergence's order of operations
        assert np.array_equal(a["div"][c], b["div"][c])
        assert np.array_equal(a["ustar"][c], b["ustar"][c])
    assert np.allclose(a["drag"], b["drag"], rtol=1e-6, atol=0.0)


def test_hill_full_size(ora):
    """The 512 x 256 x 256 hill in float32 mixed, every node compared."""
    wl = configs.hill().cast(np.float32)
    _say("sgs+apply hill 512x256x256 f32 mixed")
    _, errs = _check(ora, wl, "f32", "mixed")
    _say(f"errors {errs}")


def test_errors():
    import torch
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    _, dev = torch_dev()
    _say("sgs+apply error paths")
    ctx = ibm.Context(8, 8, 8, dtype=torch.float64, device=dev)
    z = torch.zeros(8, 8, 8, dtype=torch.float64, device=dev)
    f = [z.clone() for _ in range(12)]
    with pytest.raises(ibm.IbmError) as e:             # not prepared
        ctx.apply_sgs(z, z, f[0], f[1], f[2], f[3:9], [f[9], f[10], f[11]], [z.clone()] * 3, z0=1e-3)
    assert e.value.code == _lib.IBM_E_STATE
    phi = torch.full((8, 8, 8), 3.0, dtype=torch.float64, device=dev)
    ctx.prepare(phi, phi, 1.5, 1.5, 0.4)
    div = [z.clone() for _ in range(3)]
    with pytest.raises(ibm.IbmError) as e:             # ustar aliases u
        ctx.apply_sgs(phi, phi, f[0], f[1], f[2], f[3:9], [f[0], f[10], f[11]], div, z0=1e-3)
    assert e.value.code == _lib.IBM_E_ARG
    with pytest.raises(ibm.IbmError) as e:             # div aliases tau
        ctx.apply_sgs(phi, phi, f[0], f[1], f[2], f[3:9], [f[9], f[10], f[11]],
                      [f[3], div[1], div[2]], z0=1e-3)
    assert e.value.code == _lib.IBM_E_ARG
    with pytest.raises(ibm.IbmError) as e:
        ctx.apply_sgs(phi, phi, f[0], f[1], f[2], f[3:9], [f[9], f[10], f[11]], div, z0=0.0)
    assert e.value.code == _lib.IBM_E_RANGE


def test_plane_beyond_reach_refused():
    """A block addresses its planes with 32-bit byte offsets, so an x-y plane
    of more than (2^32 - 1) / 5 bytes is refused: 16384 x 16384 in float32
    (1 GiB per plane) gives IBM_E_ARG, and nothing is launched."""
    import torch
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    _, dev = torch_dev()
    n = 16384
    _say(f"sgs+apply {n}x{n}x1 f32: plane beyond the fused pass's reach")
    ctx = ibm.Context(n, n, 1, dtype=torch.float32, device=dev)
    phi = torch.full((1, n, n), 3.0, dtype=torch.float32, device=dev)
    ctx.prepare(phi, phi, 1.5, 1.5, 0.4)
    f = [torch.zeros_like(phi) for _ in range(15)]
    with pytest.raises(ibm.IbmError) as e:
        ctx.apply_sgs(phi, phi, f[0], f[1], f[2], f[3:9], f[9:12], f[12:15], z0=1e-3)
    assert e.value.code == _lib.IBM_E_ARG and "4 GiB" in str(e.value)
    del ctx, phi, f
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,nx,ny", [("f64", 4096, 4096), ("f32", 8192, 4096)])
def test_large_plane_chunks(dtype, nx, ny):
    """x-y planes so large that a block's slab of 32 planes would pass the
    4 GiB reach of the fused pass's 32-bit offsets: 4096 x 4096 x 30 in float64
    and 8192 x 4096 x 30 in float32 mixed (503 M and 1007 M nodes, 4 GB per
    field) march in chunks of 27 planes and a ragged 3 (in float the loads run
    two planes ahead).  Against ibm_sgs_stress + ibm_wall_stress + ibm_apply,
    div and ustar bit for bit, drag to rounding."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    if torch.cuda.get_device_properties(dev).total_memory < 150 * 2 ** 30:
        pytest.skip("needs about 110 GiB of device memory")
    nz = 30
    _say(f"sgs+apply {nx}x{ny}x{nz} {dtype} wavy wall, chunks of 27 planes")
    f64 = torch.float64
    tdt = f64 if dtype == "f64" else torch.float32
    k = torch.arange(nz, dtype=f64, device=dev).view(nz, 1, 1)
    zs = 1.25 + 0.5 * torch.sin(torch.arange(nx, dtype=f64, device=dev) * (6.283185307179586 / nx))
    phi_uv = ((k + 0.5) - zs.view(1, 1, nx)).to(tdt).expand(nz, ny, nx).contiguous()
    phi_w = (k - zs.view(1, 1, nx)).to(tdt).expand(nz, ny, nx).contiguous()
    ctx = ibm.Context(nx, ny, nz, dtype=tdt, precision="plain" if dtype == "f64" else "mixed",
                      device=dev)
    ctx.prepare(phi_uv, phi_w, 1.5, None, KAPPA)
    assert ctx.band_size(0) > 0 and ctx.band_size(1) > 0
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    vel = [torch.randn((nz, ny, nx), generator=gen, dtype=tdt, device=dev) + (3.0 if c == 0 else 0.0)
           for c in range(3)]
    tau = [torch.empty_like(vel[0]) for _ in range(6)]
    ust = [[v.clone() for v in vel] for _ in range(2)]
    div = [[torch.empty_like(vel[0]) for _ in range(3)] for _ in range(2)]
    drag = [torch.zeros(3, dtype=f64, device=dev) for _ in range(2)]
    ctx.sgs_stress(phi_uv, phi_w, *vel, tau, z0=1e-3, cs=CS, kappa=KAPPA)
    ctx.wall_stress(*vel, tau, z0=1e-3)
    ctx.apply(tau, ust[0], div[0], dt=0.01, drag=drag[0])
    # tau's band values are the wall stress either way; the fused pass reads no other
    ctx.apply_sgs(phi_uv, phi_w, *vel, tau, ust[1], div[1], z0=1e-3, cs=CS, kappa=KAPPA,
                  dt=0.01, drag=drag[1])
    torch.cuda.synchronize()
    for c in range(3):
        assert torch.equal(div[0][c], div[1][c]), f"div component {c}"
        assert torch.equal(ust[0][c], ust[1][c]), f"ustar component {c}"
        assert bool(torch.isfinite(div[1][c]).all())
    assert torch.allclose(drag[0], drag[1], rtol=1e-12 if dtype == "f64" else 1e-6, atol=0.0)
    _say("div and ustar identical to the three-call path")
    del vel, tau, ust, div, phi_uv, phi_w, ctx
    torch.cuda.empty_cache()


def test_maximum_size_periodic_copies(ora):
    """4096 x 4096 x 127 in float32 mixed (2.13e9 nodes) as 64 x 64 copies of a
    64 x 64 x 127 hill cell: every copy's div and ustar must equal the first's
    bit for bit, the first must meet the bar against the oracle's Smagorinsky
    stress fed to its stage on the cell, and the drag is 4096 times the cell's."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    if torch.cuda.get_device_properties(dev).total_memory < 200 * 2 ** 30:
        pytest.skip("needs about 190 GiB of device memory")
    torch.cuda.empty_cache()
    cell = configs.hill(64, 64, 127, H=8.0, L=24.0, x0=32.0, y0=32.0).cast(np.float32)
    g = cell.grid
    rx = ry = 64
    nx, ny, nz = g.nx * rx, g.ny * ry, g.nz
    reps = rx * ry
    assert nx * ny * nz <= 2 ** 31 - 1
    _say(f"sgs+apply {nx}x{ny}x{nz} f32 mixed: {rx}x{ry} copies of a {g.nx}x{g.ny}x{g.nz} hill cell")
    big = lambda a: tiled(a, torch.float32, ry, rx)
    ctx = ibm.Context(nx, ny, nz, g.dx, g.dy, g.dz, dtype=torch.float32, precision="mixed",
                      device=dev)
    pu, pw = big(cell.phi_uv), big(cell.phi_w)
    ctx.prepare(pu, pw, cell.band_width, cell.phi_c, cell.kappa)
    u, v, w = big(cell.u), big(cell.v), big(cell.w)
    noise = np.random.default_rng(3).standard_normal((6,) + g.shape) * 50.0
    tau = [big(a) for a in noise]
    ustar = [u.clone(), v.clone(), w.clone()]
    div = [torch.empty_like(u) for _ in range(3)]
    gp = [big(t) for t in cell.gradp]
    drag = torch.zeros(3, dtype=torch.float64, device=dev)
    ctx.wall_stress(u, v, w, tau, z0=cell.z0)
    ctx.apply_sgs(pu, pw, u, v, w, tau, ustar, div, z0=cell.z0, cs=CS, kappa=KAPPA, gradp=gp,
                  dt=cell.dt, drag=drag)
    torch.cuda.synchronize()
    got = {name: [first_copy(f, g.shape, ry, rx) for f in fs]
           for name, fs in (("div", div), ("ustar", ustar))}
    del pu, pw, u, v, w, tau, ustar, div, gp, ctx
    torch.cuda.empty_cache()
    ref = _ref(ora, cell)
    errs = {}
    for c, nm in enumerate("xyz"):
        errs["div_" + nm] = normwise(got["div"][c], ref["div"][c])
        errs["ustar_" + nm] = normwise(got["ustar"][c], ref["ustar"][c])
    scale = reps * g.dv * np.array([np.abs(d).sum() for d in ref["div"]])
    errs["drag"] = float(np.max(np.abs(drag.cpu().numpy() - reps * ref["drag"]) / scale))
    _say(f"errors {errs}")
    assert max(errs.values()) <= TOL["f32"], errs
