"""GPU classes and band statistics on flat walls at the §4.1 offsets.

* Class bytes, forcing flags and counts at z_w = 1, 1.25, 1.5, 1.75 with band
  widths 1.5 and 1.0, in float32 and float64, against the hand-derived layer
  table ``tests/golden/flat_wall_layers.txt``: the offsets 1.5 and 1.75 put
  phi exactly on -phi_b or 2 phi_b, where a bound taken open instead of
  closed changes the table (both sides compare the stored value widened to
  double against double thresholds).
* The whole stage on those walls against the oracle (log profile).
* The band statistics in closed form with the two node sets' bands on walls
  at different heights (sums per set, max |U_r| over all records, count).
"""
import os

import numpy as np
import pytest

from _gpu import TOL, compare, run_gpu, torch_dev
from workloads import Grid, configs, terrain

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "flat_wall_layers.txt")
KAPPA = 0.4


def _say(msg):
    print(msg, flush=True)


def _rows():
    out = []
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if line:
            v = line.split()
            out.append((float(v[0]), float(v[1]), *map(int, v[2:])))
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"b{r[0]}-zw{r[1]}")
def test_flat_wall_layer_table(ora, row, dtype):
    b, zw, uvb, uvs, uvf, wb, ws, wf = row
    g = Grid(64, 6, 9)
    wl = configs.flat(g, zw, theta=0.4, noise=0.05, tau_std=0.01, gp_std=0.1, band_width=b,
                      phi_c=1.5)
    if dtype == "f32":
        wl = wl.cast(np.float32)
    _say(f"flat wall z_w {zw} band {b} {dtype}")
    out, ctx = run_gpu(wl, dtype, "mixed" if dtype == "f32" else "plain")
    mask = out["mask"]
    cols = g.nx * g.ny
    uvc, wc = mask & 3, (mask >> 2) & 3
    assert (uvc == 1).sum() == uvb * cols and (uvc == 2).sum() == uvs * cols
    assert ((mask >> 4) & 1).sum() == uvf * cols
    assert (wc == 1).sum() == wb * cols and (wc == 2).sum() == ws * cols
    assert ((mask >> 5) & 1).sum() == wf * cols
    assert list(out["counts"]) == [(g.nz - uvb - uvs) * cols, uvb * cols, uvs * cols,
                                   (g.nz - wb - ws) * cols, wb * cols, ws * cols]
    errs = compare(out, ora.stage(wl), wl, TOL[dtype])
    _say(f"errors {errs}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("za,zb,a,c", [(1.0, 3.25, -2.0, 1.5), (3.25, 1.0, -2.0, 1.5)])
def test_band_statistics_two_walls(za, zb, a, c, dtype):
    """The GPU's band statistics against the closed form of the oracle's pin."""
    import paper_2006_03343_amd as ibm
    torch, dev = torch_dev()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g = Grid(64, 5, 12)
    b, phi_c, z0, theta = 1.5, 1.5, 1e-3, 0.6
    pu = terrain.flat(g, za)[0]
    pw = terrain.flat(g, zb)[1]
    zuv = (np.arange(g.nz) + 0.5)[:, None, None] * np.ones(g.shape)
    prof = a + c * zuv
    u, v = prof * np.cos(theta), prof * np.sin(theta)
    w = np.random.default_rng(3).standard_normal(g.shape)
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev, tdt)
    ctx = ibm.Context(g.nx, g.ny, g.nz, dtype=tdt, device=dev)
    ctx.prepare(T(pu), T(pw), b, phi_c, KAPPA)
    st = torch.zeros(4, dtype=torch.float64, device=dev)
    ctx.wall_stress(T(u), T(v), T(w), [torch.zeros(g.shape, dtype=tdt, device=dev)
                                       for _ in range(6)], z0=z0, stats=st)
    torch.cuda.synchronize()
    got = st.cpu().numpy()
    Ua, Ub = abs(a + c * (za + phi_c)), abs(a + c * (zb + phi_c))
    tw = lambda U: -(KAPPA * U / np.log(phi_c / z0)) ** 2
    nuv = int(((pu >= 0) & (pu <= b)).sum())
    nw = int((np.abs(pw) <= b / 2).sum())
    tol = TOL[dtype]
    _say(f"stats {got} closed form {[nuv * tw(Ua), nw * tw(Ub), max(Ua, Ub), nuv + nw]}")
    assert abs(got[0] - nuv * tw(Ua)) <= tol * abs(nuv * tw(Ua))
    assert abs(got[1] - nw * tw(Ub)) <= tol * abs(nw * tw(Ub))
    assert abs(got[2] - max(Ua, Ub)) <= tol * max(Ua, Ub)
    assert got[3] == nuv + nw
