"""GPU parity of the pseudo-spectral divergence mode (ibm_apply_spectral)
against the oracle's stage with pseudo-spectral horizontal derivatives.

Same bars as the central-difference stage (normwise per output: 1e-12 for
float64, 2e-5 for float32; masks and forcing exact).  The SGS stress inputs
are white noise, so every case carries Nyquist-mode content: a leak of one
packed field's Nyquist term into the other would show.  Cases: the cube,
small hills in three precisions, per-node log z0, grids with one row, one
column, one plane and two nodes, the 512 x 256 x 256 hill, fields one
element into their buffers (float32: the y pass then takes one column per
access instead of 8-byte column pairs), the longest transforms along x and
along y in both precisions; a grid size that is not a power of two, or one
beyond the longest transform, is refused.
"""
import numpy as np
import pytest

from _gpu import TOL, compare, run_gpu, torch_dev
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
