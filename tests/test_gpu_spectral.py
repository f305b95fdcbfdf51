"""GPU parity of the pseudo-spectral divergence mode (ibm_apply_spectral)
against the oracle's stage with pseudo-spectral horizontal derivatives.

Same bars as the central-difference stage (normwise per output: 1e-12 for
float64, 2e-5 for float32; masks and forcing exact).  The SGS stress inputs
are white noise, so every case carries Nyquist-mode content: a leak of one
packed field's Nyquist term into the other would show.  Cases: the cube,
small hills in three precisions, per-node log z0, grids with one row, one
column, one plane and two nodes (float64, and in float32 with the y pass's
512-thread blocks on uneven team layouts), the 512 x 256 x 256 hill, fields one
element into their buffers (float32: the y pass then takes one column per
access instead of 8-byte column pairs), the longest transforms along x and
along y in both precisions, 2048 x 2048 x 511 (near the 2^31 - 1 node limit
of a context) as periodic copies of a hill cell, every copy against the
oracle on the cell; a grid size that is not a power of two, or one beyond the
longest transform, is refused.
"""
import numpy as np
import pytest

from _gpu import TOL, compare, first_copy, normwise, run_gpu, tiled, torch_dev
from workloads import Grid, configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _ref(ora, wl):
    return ora.stage_spectral(wl)


def test_cube_f64(ora):
    wl = configs.cube()
    _say("spectral cube 64x32x32 f64")
    out, _ = run_gpu(wl, "f64", spectral=True)
    errs = compare(out, _ref(ora, wl), wl, TOL["f64"])
    _say(f"errors {errs}")


@pytest.mark.parametrize("dtype,prec", [("f64", "plain"), ("f32", "plain"), ("f32", "mixed")])
def test_small_hill(ora, dtype, prec):
    wl = configs.hill(128, 64, 32, H=12.0, L=30.0, x0=40.0, y0=32.0)
    if dtype == "f32":
        wl = wl.cast(np.float32)
    _say(f"spectral hill 128x64x32 {dtype} {prec}")
    out, _ = run_gpu(wl, dtype, prec, spectral=True)
    errs = compare(out, _ref(ora, wl), wl, TOL[dtype])
    _say(f"errors {errs}")


def test_per_node_log_z0(ora):
    wl = configs.fractal(64, 32, 40, rms=4.0).cast(np.float32)
    _say("spectral fractal 64x32x40 f32 mixed, log z0 field")
    out, _ = run_gpu(wl, "f32", "mixed", spectral=True)
    errs = compare(out, _ref(ora, wl), wl, TOL["f32"])
    _say(f"errors {errs}")


def test_degenerate_grids(ora):
    for shape in ((2, 1, 5), (1, 4, 6), (8, 2, 3), (16, 8, 1), (1, 1, 4)):
        g = Grid(*shape)
        wl = configs.flat(g, 1.25, theta=0.4, z0=1e-3, noise=0.2, tau_std=0.01, gp_std=0.1,
                          seed=shape[0] + 10 * shape[1])
        _say(f"spectral flat {shape} f64")
        out, _ = run_gpu(wl, "f64", spectral=True)
        compare(out, _ref(ora, wl), wl, TOL["f64"])


@pytest.mark.parametrize("shape", [(2, 256, 5), (4, 64, 7), (128, 2, 6), (8, 1024, 3),
                                   (1024, 8, 3), (2, 1, 5), (1, 4, 6), (16, 8, 1)])
def test_float_team_layouts(ora, shape):
    """Float32 mixed on grids whose 512-thread y blocks hold a few columns of
    many teams, many columns of few teams, or columns beyond the grid (nx of
    1 or 2 against 16 teams), and x transforms of 1 to 1024 points."""
    g = Grid(*shape)
    wl = configs.flat(g, 1.25, theta=0.4, z0=1e-3, noise=0.2, tau_std=0.01, gp_std=0.1,
                      seed=shape[0] + 10 * shape[1]).cast(np.float32)
    _say(f"spectral flat {shape} f32 mixed")
    out, _ = run_gpu(wl, "f32", "mixed", spectral=True)
    errs = compare(out, _ref(ora, wl), wl, TOL["f32"])
    _say(f"errors {errs}")


def test_misaligned_views(ora):
    wl = configs.hill(128, 64, 32, H=12.0, L=30.0, x0=40.0, y0=32.0).cast(np.float32)
    _say("spectral hill 128x64x32 f32 mixed, fields one element into their buffers")
    out, _ = run_gpu(wl, "f32", "mixed", spectral=True, offset=1)
    ref = _ref(ora, wl)
    errs = compare(out, ref, wl, TOL["f32"])
    _say(f"errors {errs}")
    base, _ = run_gpu(wl, "f32", "mixed", spectral=True)
    for c in range(3):
        assert np.abs(out["div"][c] - base["div"][c]).max() <= 1e-6 * np.abs(base["div"][c]).max()


def test_not_a_power_of_two():
    import torch
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    _, dev = torch_dev()
    wl = configs.ridge(100, 36, 40, H=8.0, L=20.0, x0=30.0)
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ibm.Context(g.nx, g.ny, g.nz, dtype=torch.float64, device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), 1.5)
    f = [T(t) for t in wl.tau]
    u = [T(wl.u).clone() for _ in range(3)]
    d = [torch.empty_like(u[0]) for _ in range(3)]
    with pytest.raises(ibm.IbmError) as e:
        ctx.apply_spectral(f, u, d)
    assert e.value.code == _lib.IBM_E_UNSUPPORTED


def test_hill_full_size(ora):
    wl = configs.hill().cast(np.float32)
    _say("spectral hill 512x256x256 f32 mixed")
    out, _ = run_gpu(wl, "f32", "mixed", spectral=True)
    errs = compare(out, _ref(ora, wl), wl, TOL["f32"])
    _say(f"errors {errs}")


@pytest.mark.parametrize("shape,dtype", [((2048, 4, 6), "f32"), ((4, 2048, 6), "f32"),
                                         ((1024, 4, 6), "f64"), ((4, 1024, 6), "f64")])
def test_maximum_lengths(ora, shape, dtype):
    """The longest transforms each storage type takes (2048 points in float,
    1024 in double), along x and along y."""
    g = Grid(*shape)
    wl = configs.flat(g, 1.25, theta=0.4, z0=1e-3, noise=0.2, tau_std=0.01, gp_std=0.1,
                      seed=shape[0] + 3 * shape[1])
    if dtype == "f32":
        wl = wl.cast(np.float32)
    _say(f"spectral flat {shape} {dtype} (maximum transform length)")
    out, _ = run_gpu(wl, dtype, "mixed" if dtype == "f32" else "plain", spectral=True)
    errs = compare(out, _ref(ora, wl), wl, TOL[dtype])
    _say(f"errors {errs}")


@pytest.mark.parametrize("shape,dtype", [((4096, 2, 3), "f32"), ((2, 4096, 3), "f32"),
                                         ((2048, 2, 3), "f64"), ((2, 2048, 3), "f64")])
def test_beyond_maximum_length(shape, dtype):
    import torch
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    _, dev = torch_dev()
    g = Grid(*shape)
    wl = configs.flat(g, 1.25, theta=0.4, z0=1e-3, noise=0.2, tau_std=0.01, gp_std=0.1, seed=1)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, tdt)
    ctx = ibm.Context(g.nx, g.ny, g.nz, dtype=tdt, device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), 1.25)
    f = [T(t) for t in wl.tau]
    u = [T(wl.u).clone() for _ in range(3)]
    d = [torch.empty_like(u[0]) for _ in range(3)]
    _say(f"spectral {shape} {dtype}: refused")
    with pytest.raises(ibm.IbmError) as e:
        ctx.apply_spectral(f, u, d)
    assert e.value.code == _lib.IBM_E_UNSUPPORTED


def test_maximum_size_periodic_copies(ora):
    """2048 x 2048 x 511 in float32 mixed (2.14e9 nodes, at the longest float
    transforms) as 128 x 128 copies of a 16 x 16 x 511 hill cell.  The fields
    hold only the cell's wavenumbers (its Nyquist modes land on the grid's), so
    each copy's outputs are the cell's: the wall stress, a local operation,
    equal in every copy bit for bit; div and ustar at every node of every copy
    against the oracle's spectral stage on the cell; class bytes in every copy
    and counts 16384 times the cell's; the drag 16384 times the cell's."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    if torch.cuda.get_device_properties(dev).total_memory < 200 * 2 ** 30:
        pytest.skip("needs about 180 GiB of device memory")
    torch.cuda.empty_cache()
    cell = configs.hill(16, 16, 511, H=4.0, L=6.0, x0=8.0, y0=8.0).cast(np.float32)
    g = cell.grid
    rx = ry = 128
    nx, ny, nz = g.nx * rx, g.ny * ry, g.nz
    reps = rx * ry
    assert nx * ny * nz <= 2 ** 31 - 1
    _say(f"spectral {nx}x{ny}x{nz} f32 mixed: {rx}x{ry} copies of a {g.nx}x{g.ny}x{nz} hill cell")
    big = lambda a: tiled(a, torch.float32, ry, rx)
    ctx = ibm.Context(nx, ny, nz, g.dx, g.dy, g.dz, dtype=torch.float32, precision="mixed",
                      device=dev)
    pu, pw = big(cell.phi_uv), big(cell.phi_w)
    ctx.prepare(pu, pw, cell.band_width, cell.phi_c, cell.kappa)
    del pu, pw
    u, v, w = big(cell.u), big(cell.v), big(cell.w)
    tau = [big(t) for t in cell.tau]
    ustar = [u.clone(), v.clone(), w.clone()]
    div = [torch.empty_like(u) for _ in range(3)]
    gp = [big(t) for t in cell.gradp]
    drag = torch.zeros(3, dtype=torch.float64, device=dev)
    ctx.wall_stress(u, v, w, tau, z0=cell.z0)
    ctx.apply_spectral(tau, ustar, div, gradp=gp, dt=cell.dt, drag=drag)
    torch.cuda.synchronize()
    ref = _ref(ora, cell)
    got_tau = [first_copy(t, g.shape, ry, rx) for t in tau]
    del u, v, w, tau, gp
    errs = {}
    band_uv = (ref["mask"] & 3) == 1
    band_w = ((ref["mask"] >> 2) & 3) == 1
    for c in range(6):
        sel = band_uv if c < 4 else band_w
        errs[f"tau{c}"] = normwise(got_tau[c][sel], ref["tau"][c][sel])
        assert (got_tau[c][~sel] == ref["tau"][c][~sel]).all(), f"tau {c} off the band"
    for name, fs in (("div", div), ("ustar", ustar)):
        for c, f in enumerate(fs):
            rt = torch.from_numpy(np.ascontiguousarray(ref[name][c], dtype=np.float64)).to(dev)
            cv = f.view(nz, ry, g.ny, rx, g.nx)
            num = 0.0
            for k0 in range(0, nz, 32):
                d = (cv[k0:k0 + 32].double() - rt[k0:k0 + 32, None, :, None, :]).abs().max()
                num = max(num, float(d))
            errs[f"{name}{c}"] = num / float(np.abs(ref[name][c]).max())
    del div, ustar
    mask = ctx.mask().reshape(nz, ry, g.ny, rx, g.nx)
    for k in range(nz):
        assert (mask[k] == ref["mask"][k][None, :, None, :]).all(), f"class bytes, plane {k}"
    del mask
    assert list(ctx.counts()) == [reps * int(c) for c in ref["counts"]]
    scale = reps * g.dv * np.array([np.abs(d).sum() for d in ref["div"]])
    errs["drag"] = float(np.max(np.abs(drag.cpu().numpy() - reps * ref["drag"]) / scale))
    del ctx
    torch.cuda.empty_cache()
    _say(f"errors {errs}")
    assert max(errs.values()) <= TOL["f32"], errs
