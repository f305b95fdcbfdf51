"""GPU parity of the AB2 update and the pressure projection
(ibm_ab2_predict, ibm_pressure_project) against the oracle.

* small grids (float64 and float32), among them the longest transforms along
  x and along y of each type (2048 points in float, 1024 in double): u, v, w
  after the projection and the pressure, normwise per field <= 1e-12
  (float64) and 2e-5 (float32);
* the projected field is discretely divergence-free in every cell (the
  oracle's D applied to the GPU's output) and w is exactly 0 on the floor's
  and the lid's w nodes, also where w* is not 0 there; with w* = 0 on both
  walls of an 8 x 8 x 9 grid the lid's w stays 0;
* output in place of the input;
* the 512 x 256 x 256 hill in float32: the divergence of the projected
  field, and the pressure's spectrum at sampled horizontal modes against
  the oracle's dense solve of those modes' systems (normwise over the
  sampled modes: float32 rounding of the transforms scales with the whole
  field, not with one high mode's small amplitude);
* 2048 x 2048 x 511 in float32 (near the 2^31 - 1 node limit of a context, at
  the longest float transforms), made of periodic copies of a small cell:
  every node of every copy against the oracle's projection of the cell;
* AB2 against its formula, also on 4096 x 4096 x 127 (near the node limit) as
  periodic copies of a cell; error paths (lengths beyond the longest transform
  refused).
"""
import numpy as np
import pytest

from _gpu import TOL, first_copy, normwise, tiled, torch_dev
from workloads import Grid

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _fields(g, seed, wall=False):
    rng = np.random.default_rng(seed)
    u, v, w = rng.standard_normal((3,) + g.shape)
    if wall:
        w[0] = 0.0
        w[-1] = 0.0
    return [u, v, w]


def _project(g, vel, dt, dtype, in_place=False):
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=tdt, device=dev)
    us = [torch.from_numpy(np.ascontiguousarray(a)).to(dev, tdt) for a in vel]
    out = us if in_place else [torch.empty_like(a) for a in us]
    p = torch.empty_like(us[0])
    ctx.pressure_project(us, dt, out, p)
    torch.cuda.synchronize()
    return [a.cpu().numpy().astype(np.float64) for a in out], p.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape,sp,dtype", [((8, 8, 6), (1.0, 1.0, 1.0), "f64"),
                                            ((16, 8, 9), (0.7, 1.3, 0.9), "f64"),
                                            ((32, 16, 12), (1.0, 1.0, 1.0), "f32"),
                                            ((4, 2, 1), (1.0, 1.0, 1.0), "f64"),
                                            ((1, 8, 5), (1.0, 1.0, 1.0), "f64"),
                                            # x teams within one wave, the mirror
                                            # slots by lane permutation: the
                                            # shortest and the longest such rows
                                            ((8, 16, 4), (1.0, 1.0, 1.0), "f32"),
                                            ((256, 8, 5), (0.9, 1.1, 1.0), "f32"),
                                            ((512, 4, 3), (1.0, 1.0, 1.0), "f64"),
                                            # an odd number of x rows (ny = 1): the
                                            # last row pair has one row, and teams
                                            # past the end read clamped rows
                                            ((64, 1, 5), (1.0, 1.0, 1.0), "f32"),
                                            ((512, 1, 7), (1.0, 1.0, 1.3), "f64"),
                                            # the longest transforms each type takes
                                            ((2048, 4, 3), (1.0, 1.0, 1.0), "f32"),
                                            ((4, 2048, 3), (1.0, 1.0, 1.0), "f32"),
                                            ((1024, 4, 3), (1.0, 1.0, 1.0), "f64"),
                                            ((4, 1024, 3), (1.0, 1.0, 1.0), "f64")])
def test_projection_matches_oracle(ora, shape, sp, dtype):
    g = Grid(*shape, *sp)
    vel = _fields(g, sum(shape), wall=False)
    if dtype == "f32":
        vel = [a.astype(np.float32).astype(np.float64) for a in vel]
    dt = 0.017
    _say(f"projection {shape} {dtype}")
    out, p = _project(g, vel, dt, dtype)
    ru, rv, rw, rp = ora.pressure_project(g, vel, dt)
    errs = [normwise(a, b) for a, b in zip(out + [p], [ru, rv, rw, rp])]
    _say(f"errors u v w p {errs}")
    assert max(errs) <= TOL[dtype], errs


@pytest.mark.parametrize("dtype,bar", [("f64", 1e-10), ("f32", 2e-5)])
def test_divergence_free_and_in_place(ora, dtype, bar):
    g = Grid(64, 32, 24, 1.0, 1.0, 0.8)
    vel = _fields(g, 7)
    if dtype == "f32":
        vel = [a.astype(np.float32).astype(np.float64) for a in vel]
    _say(f"projection 64x32x24 {dtype}: divergence after, in place")
    out, p = _project(g, vel, 0.01, dtype, in_place=True)
    d0 = np.abs(ora.divergence_velocity(g, *vel)).max()
    d1 = np.abs(ora.divergence_velocity(g, *out)).max()
    _say(f"max |D u| before {d0:.3e}, after {d1:.3e}")
    assert d1 <= bar * d0
    # the floor's and the lid's w nodes are walls (eqs. bc-bottom-u3, bc-top)
    assert np.abs(out[2][0]).max() == 0.0 and np.abs(out[2][-1]).max() == 0.0
    assert np.abs(vel[2][0]).max() > 0.0 and np.abs(vel[2][-1]).max() > 0.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lid_stays_zero(ora, dtype):
    g = Grid(8, 8, 9)
    vel = _fields(g, 13, wall=True)
    if dtype == "f32":
        vel = [a.astype(np.float32).astype(np.float64) for a in vel]
    _say(f"projection 8x8x9 {dtype}: w = 0 on both walls")
    out, p = _project(g, vel, 0.01, dtype)
    assert np.abs(out[2][-1]).max() == 0.0 and np.abs(out[2][0]).max() == 0.0
    ru, rv, rw, rp = ora.pressure_project(g, vel, 0.01)
    assert np.abs(rw[-1]).max() == 0.0
    errs = [normwise(a, b) for a, b in zip(out + [p], [ru, rv, rw, rp])]
    _say(f"errors u v w p {errs}")
    assert max(errs) <= TOL[dtype], errs


def test_hill_size_sampled_modes(ora):
    g = Grid(512, 256, 256)
    vel = [a.astype(np.float32).astype(np.float64) for a in _fields(g, 11)]
    dt = 0.01
    _say("projection 512x256x256 f32: divergence and sampled modes of p")
    out, p = _project(g, vel, dt, "f32")
    d0 = np.abs(ora.divergence_velocity(g, *vel)).max()
    d1 = np.abs(ora.divergence_velocity(g, *out)).max()
    _say(f"max |D u| before {d0:.3e}, after {d1:.3e}")
    assert d1 <= 2e-5 * d0
    # pressure spectrum at sampled modes vs dense solves of their systems over
    # the nz - 1 cells, the wall w taken as 0 in the right-hand side
    m = g.nz - 1
    wb = vel[2].copy()
    wb[0] = 0.0
    wb[-1] = 0.0
    rhs = 2.0 / (3.0 * dt) * ora.divergence_velocity(g, vel[0], vel[1], wb)[:m]
    rh = np.fft.fft2(rhs, axes=(1, 2))
    ph = np.fft.fft2(p[:m], axes=(1, 2))
    assert np.abs(p[m]).max() == 0.0                          # above the lid
    kx = 2 * np.pi * np.fft.fftfreq(g.nx, d=1.0 / g.nx) / g.lx
    ky = 2 * np.pi * np.fft.fftfreq(g.ny, d=1.0 / g.ny) / g.ly
    kx[g.nx // 2] = 0.0
    ky[g.ny // 2] = 0.0
    rng = np.random.default_rng(12)
    modes = [(0, 0), (g.nx // 2, 0), (1, 0), (0, 1), (3, 7), (g.nx - 5, g.ny // 2 + 3)]
    modes += [(int(rng.integers(g.nx)), int(rng.integers(g.ny))) for _ in range(10)]
    c = 1.0 / g.dz ** 2
    num = den = 0.0
    for i, j in modes:
        K2 = kx[i] ** 2 + ky[j] ** 2
        A = np.diag(np.full(m - 1, c), 1) + np.diag(np.full(m - 1, c), -1)
        A -= np.diag(A.sum(axis=1) + K2)
        b = rh[:, j, i].copy()
        if K2 == 0.0:
            A[0, :] = 0.0
            A[0, 0] = 1.0
            b[0] = 0.0
        ref = np.linalg.solve(A, b)
        num = max(num, np.abs(ph[:, j, i] - ref).max())
        den = max(den, np.abs(ref).max())
    # normwise over the sampled modes, as for every other output
    _say(f"sampled modes: normwise error {num / den:.2e}")
    assert num <= 2e-5 * den


def test_ab2(ora):
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    g = Grid(20, 12, 7)
    rng = np.random.default_rng(5)
    u, rn, rp = ([rng.standard_normal(g.shape) for _ in range(3)] for _ in range(3))
    ctx = ibm.Context(g.nx, g.ny, g.nz, dtype=torch.float64, device=dev)
    T = lambda a: torch.from_numpy(a).to(dev)
    out = [torch.empty(g.shape, dtype=torch.float64, device=dev) for _ in range(3)]
    ctx.ab2_predict([T(a) for a in u], [T(a) for a in rn], [T(a) for a in rp], 0.03, out)
    ref = ora.ab2_predict(u, rn, rp, 0.03)
    for a, b in zip(out, ref):
        assert normwise(a.cpu().numpy(), b) <= 1e-15


def test_errors():
    import torch
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    _, dev = torch_dev()
    ctx = ibm.Context(12, 8, 4, dtype=torch.float64, device=dev)
    f = [torch.zeros(4, 8, 12, dtype=torch.float64, device=dev) for _ in range(4)]
    with pytest.raises(ibm.IbmError) as e:
        ctx.pressure_project(f[:3], 0.01, f[:3], f[3])
    assert e.value.code == _lib.IBM_E_UNSUPPORTED              # nx = 12
    ctx = ibm.Context(16, 8, 4, dtype=torch.float64, device=dev)
    f = [torch.zeros(4, 8, 16, dtype=torch.float64, device=dev) for _ in range(4)]
    with pytest.raises(ibm.IbmError) as e:
        ctx.pressure_project(f[:3], 0.0, f[:3], f[3])
    assert e.value.code == _lib.IBM_E_RANGE
    with pytest.raises(ibm.IbmError) as e:
        ctx.pressure_project(f[:3], 0.01, f[:3], f[0])
    assert e.value.code == _lib.IBM_E_ARG
    for shape, tdt in (((3, 2, 4096), torch.float32), ((3, 4096, 2), torch.float32),
                       ((3, 2, 2048), torch.float64), ((3, 2048, 2), torch.float64)):
        # beyond the longest transform of the storage type
        ctx = ibm.Context(shape[2], shape[1], shape[0], dtype=tdt, device=dev)
        f = [torch.zeros(shape, dtype=tdt, device=dev) for _ in range(4)]
        with pytest.raises(ibm.IbmError) as e:
            ctx.pressure_project(f[:3], 0.01, [torch.empty_like(f[0]) for _ in range(3)], f[3])
        assert e.value.code == _lib.IBM_E_UNSUPPORTED


def test_maximum_size_periodic_copies(ora):
    """2048 x 2048 x 511 in float32 (2.14e9 nodes) as 128 x 128 copies of a
    16 x 16 x 511 cell of random velocities.  The data hold only the modes
    whose wavenumbers the cell has (its Nyquist modes land on the grid's), so
    the projected velocity and the pressure are the cell's, copied: every node
    of every copy against the oracle's projection of the cell, normwise per
    field within the float32 bar."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    if torch.cuda.get_device_properties(dev).total_memory < 200 * 2 ** 30:
        pytest.skip("needs about 150 GiB of device memory")
    torch.cuda.empty_cache()
    cell = Grid(16, 16, 511)
    vel = [a.astype(np.float32).astype(np.float64) for a in _fields(cell, 21, wall=False)]
    rx = ry = 128
    nx, ny, nz = cell.nx * rx, cell.ny * ry, cell.nz
    assert nx * ny * nz <= 2 ** 31 - 1
    dt = 0.013
    _say(f"projection {nx}x{ny}x{nz} f32: {rx}x{ry} copies of a {cell.nx}x{cell.ny}x{nz} cell")
    ctx = ibm.Context(nx, ny, nz, cell.dx, cell.dy, cell.dz, dtype=torch.float32, device=dev)
    us = [tiled(a, torch.float32, ry, rx) for a in vel]
    out = [torch.empty_like(us[0]) for _ in range(3)]
    p = torch.empty_like(us[0])
    ctx.pressure_project(us, dt, out, p)
    torch.cuda.synchronize()
    del us, ctx
    ref = ora.pressure_project(cell, vel, dt)
    errs = []
    for f, r in zip(out + [p], ref):
        rt = torch.from_numpy(np.ascontiguousarray(r, dtype=np.float64)).to(dev)
        cv = f.view(nz, ry, cell.ny, rx, cell.nx)
        num = 0.0
        for k0 in range(0, nz, 32):
            d = (cv[k0:k0 + 32].double() - rt[k0:k0 + 32, None, :, None, :]).abs().max()
            num = max(num, float(d))
        errs.append(num / float(np.abs(r).max()))
    del out, p
    torch.cuda.empty_cache()
    _say(f"errors u v w p {errs}")
    assert max(errs) <= TOL["f32"], errs


def test_ab2_maximum_size(ora):
    """AB2 on 4096 x 4096 x 127 in float32 (2.13e9 nodes) as 64 x 64 copies of
    a 64 x 64 x 127 cell: every copy equal to the first, the first against the
    oracle's AB2 of the cell within the float32 bar."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    if torch.cuda.get_device_properties(dev).total_memory < 150 * 2 ** 30:
        pytest.skip("needs about 110 GiB of device memory")
    torch.cuda.empty_cache()
    cell = Grid(64, 64, 127)
    rng = np.random.default_rng(9)
    u, rn, rp = ([rng.standard_normal(cell.shape).astype(np.float32).astype(np.float64)
                  for _ in range(3)] for _ in range(3))
    rx = ry = 64
    nx, ny, nz = cell.nx * rx, cell.ny * ry, cell.nz
    assert nx * ny * nz <= 2 ** 31 - 1
    _say(f"ab2 {nx}x{ny}x{nz} f32: {rx}x{ry} copies of a {cell.nx}x{cell.ny}x{nz} cell")
    big = lambda a: tiled(a, torch.float32, ry, rx)
    ctx = ibm.Context(nx, ny, nz, dtype=torch.float32, device=dev)
    out = [torch.empty((nz, ny, nx), dtype=torch.float32, device=dev) for _ in range(3)]
    ctx.ab2_predict([big(a) for a in u], [big(a) for a in rn], [big(a) for a in rp], 0.03, out)
    torch.cuda.synchronize()
    got = [first_copy(o, cell.shape, ry, rx) for o in out]
    del out, ctx
    torch.cuda.empty_cache()
    ref = ora.ab2_predict(u, rn, rp, 0.03)
    errs = [normwise(a, b) for a, b in zip(got, ref)]
    _say(f"errors {errs}")
    assert max(errs) <= TOL["f32"], errs
