"""GPU parity of the Smagorinsky stress with Mason's wall damping
(ibm_sgs_stress) against the oracle, component by component.

Bars (normwise per component: max |gpu - oracle| / max |oracle|): 1e-12 for
float64 storage, 2e-5 for float32; the oracle reads exactly the stored values.
Cases: the cube, a ragged ridge (no tile dimension divides the grid), a
small hill, a per-node log z0 field, one-column / one-row / one-plane and
anisotropic grids, the 512 x 256 x 256 hill, and 4096 x 4096 x 127 grids (near
the 2^31 - 1 node limit of a context) made of periodic copies of a hill cell,
each copy equal to the first; tile shapes change nothing
(bit for bit); views that are not 16-byte aligned take the one-node-per-lane
path and agree too.
"""
import numpy as np
import pytest

from _gpu import TOL, first_copy, normwise, tiled, torch_dev
from workloads import Grid, configs

pytestmark = pytest.mark.gpu
CS, KAPPA = 0.16, 0.4


def _say(msg):
    print(msg, flush=True)


def _run(wl, dtype, tile=None, offset=0):
    """ibm_sgs_stress on the workload; ``offset`` > 0 passes every field as a
    view starting ``offset`` elements into a larger buffer."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g = wl.grid

    def T(a):
        buf = torch.empty(g.n + offset, dtype=tdt, device=dev)
        view = buf[offset:].view(g.shape)
        view.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, tdt))
        return view

    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=tdt, device=dev)
    if tile is not None:
        ctx.set_tile(*tile)
    tau = [T(np.zeros(g.shape)) for _ in range(6)]
    lz = T(wl.log_z0) if wl.log_z0 is not None else None
    ctx.sgs_stress(T(wl.phi_uv), T(wl.phi_w), T(wl.u), T(wl.v), T(wl.w), tau,
                   z0=None if lz is not None else wl.z0, log_z0=lz, cs=CS, kappa=KAPPA)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in tau]


def _check(ora, wl, dtype, tile=None, offset=0):
    got = _run(wl, dtype, tile, offset)
    ref = ora.smagorinsky(wl.grid, wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w,
                          z0=None if wl.log_z0 is not None else wl.z0, log_z0=wl.log_z0,
                          cs=CS, kappa=KAPPA)
    errs = [normwise(a, b) for a, b in zip(got, ref)]
    assert max(errs) <= TOL[dtype], errs
    return got, errs


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cube(ora, dtype):
    wl = configs.cube()
    if dtype == "f32":
        wl = wl.cast(np.float32)
    _say(f"sgs cube 64x32x32 {dtype}")
    _, errs = _check(ora, wl, dtype)
    _say(f"errors {errs}")


@pytest.mark.parametrize("dtype,tile", [("f64", (2, 1, 16, 4)), ("f64", (1, 1, 5, 2)),
                                        ("f32", (4, 1, 9, 4)), ("f32", (1, 1, 3, 1)),
                                        ("f32", (2, 1, 40, 3))])
def test_ragged_ridge(ora, dtype, tile):
    wl = configs.ridge(100, 36, 40, H=8.0, L=20.0, x0=30.0)
    if dtype == "f32":
        wl = wl.cast(np.float32)
    _say(f"sgs ridge 100x36x40 {dtype} tile {tile}")
    _, errs = _check(ora, wl, dtype, tile)
    _say(f"errors {errs}")


def test_tile_shapes_bitwise_identical():
    wl = configs.hill(128, 64, 64, H=16.0, L=40.0, x0=40.0, y0=32.0).cast(np.float32)
    _say("sgs hill 128x64x64 f32, tile shapes")
    base = _run(wl, "f32", (1, 1, 64, 1))
    for t in ((4, 1, 7, 4), (2, 1, 16, 2), (4, 1, 128, 1)):
        got = _run(wl, "f32", t)
        for c in range(6):
            assert np.array_equal(got[c], base[c]), (t, c)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_per_node_log_z0(ora, dtype):
    wl = configs.fractal(64, 48, 40, rms=4.0)
    if dtype == "f32":
        wl = wl.cast(np.float32)
    _say(f"sgs fractal 64x48x40 log z0 {dtype}")
    _, errs = _check(ora, wl, dtype)
    _say(f"errors {errs}")


def test_misaligned_views(ora):
    wl = configs.hill(128, 64, 40, H=16.0, L=40.0, x0=40.0, y0=32.0).cast(np.float32)
    _say("sgs hill 128x64x40 f32, views one element into their buffers")
    got, errs = _check(ora, wl, "f32", (4, 1, 16, 1), offset=1)
    base = _run(wl, "f32", (1, 1, 16, 1))
    for c in range(6):
        assert np.array_equal(got[c], base[c]), c


def test_degenerate_grids(ora):
    for shape, sp in (((1, 1, 12), (1.0, 1.0, 1.0)), ((7, 1, 9), (1.0, 1.0, 1.0)),
                      ((1, 6, 9), (0.5, 1.0, 1.0)), ((33, 5, 1), (1.0, 1.0, 1.0)),
                      ((20, 12, 10), (0.7, 1.3, 0.9))):
        g = Grid(*shape, *sp)
        wl = configs.flat(g, 1.25 * sp[2], theta=0.4, z0=1e-3, noise=0.3, tau_std=0.01,
                          gp_std=0.1, seed=shape[0])
        _say(f"sgs flat {shape} spacing {sp} f64")
        _check(ora, wl, "f64")


def test_errors():
    import torch
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    _, dev = torch_dev()
    _say("sgs error paths")
    ctx = ibm.Context(8, 8, 8, dtype=torch.float64, device=dev)
    z = torch.zeros(8, 8, 8, dtype=torch.float64, device=dev)
    tau = [z.clone() for _ in range(6)]
    for kw, code in ((dict(z0=0.0), _lib.IBM_E_RANGE), (dict(z0=1e-3, cs=-1.0), _lib.IBM_E_RANGE),
                     (dict(z0=1e-3, kappa=0.0), _lib.IBM_E_RANGE)):
        with pytest.raises(ibm.IbmError) as e:
            ctx.sgs_stress(z, z, z, z, z, tau, **kw)
        assert e.value.code == code
    u = z.clone()
    with pytest.raises(ibm.IbmError) as e:
        ctx.sgs_stress(z, z, u, z.clone(), z.clone(), [u] + tau[1:], z0=1e-3)
    assert e.value.code == _lib.IBM_E_ARG


def test_hill_full_size(ora):
    """The 512 x 256 x 256 hill in float32, every node compared."""
    wl = configs.hill().cast(np.float32)
    _say("sgs hill 512x256x256 f32")
    _, errs = _check(ora, wl, "f32")
    _say(f"errors {errs}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_maximum_size_periodic_copies(ora, dtype):
    """4096 x 4096 x 127 (2.13e9 nodes) as 64 x 64 copies of a 64 x 64 x 127 hill
    cell: the grid is periodic in x and y, so every copy's stress must equal the
    first's bit for bit, and the first must meet the bar against the oracle's
    Smagorinsky stress on the cell."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    need = 200 if dtype == "f64" else 110
    if torch.cuda.get_device_properties(dev).total_memory < need * 2 ** 30:
        pytest.skip(f"needs about {need - 10} GiB of device memory")
    torch.cuda.empty_cache()
    cell = configs.hill(64, 64, 127, H=8.0, L=24.0, x0=32.0, y0=32.0)
    if dtype == "f32":
        cell = cell.cast(np.float32)
    g = cell.grid
    rx = ry = 64
    nx, ny, nz = g.nx * rx, g.ny * ry, g.nz
    assert nx * ny * nz <= 2 ** 31 - 1
    _say(f"sgs {nx}x{ny}x{nz} {dtype}: {rx}x{ry} copies of a {g.nx}x{g.ny}x{g.nz} hill cell")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    big = lambda a: tiled(a, tdt, ry, rx)
    ctx = ibm.Context(nx, ny, nz, g.dx, g.dy, g.dz, dtype=tdt, device=dev)
    tau = [torch.empty((nz, ny, nx), dtype=tdt, device=dev) for _ in range(6)]
    ctx.sgs_stress(big(cell.phi_uv), big(cell.phi_w), big(cell.u), big(cell.v), big(cell.w), tau,
                   z0=cell.z0, cs=CS, kappa=KAPPA)
    torch.cuda.synchronize()
    got = [first_copy(t, g.shape, ry, rx) for t in tau]
    del tau, ctx
    torch.cuda.empty_cache()
    ref = ora.smagorinsky(g, cell.phi_uv, cell.phi_w, cell.u, cell.v, cell.w, z0=cell.z0,
                          cs=CS, kappa=KAPPA)
    errs = [normwise(a, b) for a, b in zip(got, ref)]
    _say(f"errors {errs}")
    assert max(errs) <= TOL[dtype], errs
