"""GPU tests of the ensemble path (ibm_batch_*) and of the tile autotuner.

* every case of a batch equals a plain per-case call (ibm_wall_stress then
  ibm_apply) with the same tile shape, bit for bit: stress, divergence,
  forced velocity, drag and band statistics; one case is also held to the
  oracle; also a batch of one-column, one-row, one- and two-plane and ragged
  cases;
* seeded random ensembles (random grids, degenerate ones among them, and
  random tile shapes): every case bit for bit against plain calls, eager and
  through a captured graph, the largest against the oracle;
* the 64-case ensemble the benchmark times (105.6 M points, one graph
  launch): all 64 cases bit for bit against plain per-case calls, one case
  of each grid shape and the last case against the oracle, every node;
* replays of the captured hipGraph, with eager work and synchronisations in
  between, each equal the eager result;
* two cases of 4096 x 4096 x 64 (2^31 nodes together, each a set of periodic
  copies of a hill cell): each copy equal to the first, the first against the
  oracle on the cell, counts, drag and statistics 4096 times the cell's;
* the autotuner writes and re-reads its cache and keeps a valid shape.
"""
import json
import os

import numpy as np
import pytest

from _gpu import TOL, compare, first_copy, tiled, torch_dev
from workloads import Grid, configs

pytestmark = pytest.mark.gpu

SHAPES = [(64, 32, 24), (48, 40, 20), (32, 32, 16), (64, 64, 24), (48, 40, 20), (80, 24, 18)]
TILES = {"f32": [(4, 2, 16, 1), (2, 1, 5, 1), (1, 2, 7, 1), (4, 1, 32, 1), (2, 2, 3, 1), (1, 1, 64, 1)],
         "f64": [(2, 2, 16, 1), (1, 1, 5, 1), (2, 1, 7, 1), (1, 2, 32, 1), (2, 2, 3, 1), (1, 1, 64, 1)]}


def _say(msg):
    print(msg, flush=True)


def _cases(dtype, log_z0=False):
    wls = []
    for i, s in enumerate(SHAPES):
        wl = configs.fractal(*s, rms=3.0, seed_offset=i) if log_z0 else configs.bumps_case(i, s)
        if dtype == "f32":
            wl = wl.cast(np.float32)
        wls.append(wl)
    return wls


class Fields:
    """Device copies of one case's inputs plus output buffers."""

    def __init__(self, wl, tdt, dev):
        import torch
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, tdt)
        self.u, self.v, self.w = T(wl.u), T(wl.v), T(wl.w)
        self.lz = T(wl.log_z0) if wl.log_z0 is not None else None
        self.tau0 = torch.stack([T(t) for t in wl.tau]).contiguous()
        self.gp = [T(t) for t in wl.gradp]
        self.tau = self.tau0.clone()
        self.ustar = torch.stack([self.u, self.v, self.w]).contiguous()
        self.div = torch.zeros_like(self.ustar)
        self.drag = torch.zeros(3, dtype=torch.float64, device=dev)
        self.stats = torch.zeros(4, dtype=torch.float64, device=dev)

    def reset(self):
        import torch
        self.tau.copy_(self.tau0)
        self.ustar.copy_(torch.stack([self.u, self.v, self.w]))
        self.div.zero_()
        self.drag.zero_()
        self.stats.zero_()

    def snapshot(self):
        return {k: getattr(self, k).cpu().numpy().copy()
                for k in ("tau", "div", "ustar", "drag", "stats")}


def _plain(wl, tile, tdt, prec, dev):
    import paper_2006_03343_amd as ibm
    g = wl.grid
    f = Fields(wl, tdt, dev)
    ctx = ibm.Context(g.nx, g.ny, g.nz, dtype=tdt, precision=prec, device=dev)
    ctx.set_tile(*tile)
    T = lambda a: __import__("torch").from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, tdt)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    ctx.wall_stress(f.u, f.v, f.w, list(f.tau), z0=None if f.lz is not None else wl.z0,
                    log_z0=f.lz, stats=f.stats)
    ctx.apply(list(f.tau), list(f.ustar), list(f.div), gradp=f.gp, dt=wl.dt, drag=f.drag)
    return f.snapshot()


def _batch(wls, tiles, tdt, prec, dev):
    import torch
    import paper_2006_03343_amd as ibm
    b = ibm.Batch([(w.grid.nx, w.grid.ny, w.grid.nz) for w in wls], dtype=tdt, precision=prec,
                  device=dev)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, tdt)
    b.prepare([T(w.phi_uv) for w in wls], [T(w.phi_w) for w in wls], 1.5, [w.z0 for w in wls],
              phi_c=1.5)
    if tiles is not None:
        for i, t in enumerate(tiles):
            b.case(i).set_tile(*t)
    fs = [Fields(w, tdt, dev) for w in wls]
    for i, (w, f) in enumerate(zip(wls, fs)):
        b.bind(i, f.u, f.v, f.w, list(f.tau), list(f.ustar), list(f.div), gradp=f.gp, dt=w.dt,
               log_z0=f.lz, drag=f.drag, stats=f.stats)
    return b, fs


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs"


@pytest.mark.parametrize("dtype,prec,lz", [("f32", "mixed", False), ("f64", "plain", False),
                                           ("f32", "plain", True)])
def test_batch_equals_plain_calls(ora, dtype, prec, lz):
    torch, dev = torch_dev()
    tdt = torch.float32 if dtype == "f32" else torch.float64
    wls = _cases(dtype, lz)
    tiles = TILES[dtype]
    _say(f"batch of {len(wls)} cases {dtype} {prec} log_z0={lz}: run vs plain calls")
    b, fs = _batch(wls, tiles, tdt, prec, dev)
    b.run()
    torch.cuda.synchronize()
    for i, (w, f) in enumerate(zip(wls, fs)):
        _same(f.snapshot(), _plain(w, tiles[i], tdt, prec, dev), f"case {i}")
    # one case against the oracle
    ref = ora.stage(wls[1])
    out = dict(tau=fs[1].tau.cpu().numpy(), div=fs[1].div.cpu().numpy(),
               ustar=fs[1].ustar.cpu().numpy(), drag=fs[1].drag.cpu().numpy(),
               stats=fs[1].stats.cpu().numpy(), mask=b.case(1).mask(), counts=b.case(1).counts())
    compare(out, ref, wls[1], TOL[dtype])


def test_graph_replays_match_eager():
    torch, dev = torch_dev()
    wls = _cases("f32")
    _say("batch f32 mixed: captured graph, 3 replays with eager work between")
    b, fs = _batch(wls, TILES["f32"], torch.float32, "mixed", dev)
    b.run()
    torch.cuda.synchronize()
    eager = [f.snapshot() for f in fs]
    b.capture()
    for rep in range(3):
        for f in fs:
            f.reset()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device=dev).sum()    # unrelated eager work
        b.launch()
        torch.cuda.synchronize()
        for i, f in enumerate(fs):
            _same(f.snapshot(), eager[i], f"replay {rep} case {i}")
        del junk


def test_tile_change_after_capture():
    """A tile change on a case after capture makes launch refuse the stale graph;
    run rebuilds the work tables, and a new capture replays the new shapes."""
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    torch, dev = torch_dev()
    wls = _cases("f32")[:3]
    tiles = list(TILES["f32"][:3])
    _say("batch f32 mixed: tile change after capture")
    b, fs = _batch(wls, tiles, torch.float32, "mixed", dev)
    b.capture()
    tiles[0] = (1, 1, 3, 2)       # more tiles than before: the case's slots are reallocated
    b.case(0).set_tile(*tiles[0])
    with pytest.raises(ibm.IbmError) as e:
        b.launch()
    assert e.value.code == _lib.IBM_E_STATE
    b.run()
    torch.cuda.synchronize()
    for i, (w, f) in enumerate(zip(wls, fs)):
        _same(f.snapshot(), _plain(w, tiles[i], torch.float32, "mixed", dev), f"run, case {i}")
        f.reset()
    b.capture()
    b.launch()
    torch.cuda.synchronize()
    for i, (w, f) in enumerate(zip(wls, fs)):
        _same(f.snapshot(), _plain(w, tiles[i], torch.float32, "mixed", dev), f"replay, case {i}")


def test_batch_errors():
    import paper_2006_03343_amd as ibm
    from paper_2006_03343_amd import _lib
    torch, dev = torch_dev()
    _say("batch error paths")
    wls = _cases("f32")[:2]
    b = ibm.Batch([(w.grid.nx, w.grid.ny, w.grid.nz) for w in wls], dtype=torch.float32,
                  device=dev)
    with pytest.raises(ibm.IbmError) as e:
        b.run()
    assert e.value.code == _lib.IBM_E_STATE
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    b.prepare([T(w.phi_uv) for w in wls], [T(w.phi_w) for w in wls], 1.5, [w.z0 for w in wls])
    with pytest.raises(ibm.IbmError) as e:
        b.run()                                   # case 0 and 1 unbound
    assert e.value.code == _lib.IBM_E_STATE
    with pytest.raises(ibm.IbmError) as e:
        b.launch()                                # nothing captured
    assert e.value.code == _lib.IBM_E_STATE
    with pytest.raises(ibm.IbmError) as e:
        b.prepare([T(w.phi_uv) for w in wls], [T(w.phi_w) for w in wls], 1.5, [2.0, 1e-3])
    assert e.value.code == _lib.IBM_E_RANGE


def test_autotune_cache(tmp_path):
    import paper_2006_03343_amd as ibm
    torch, dev = torch_dev()
    wl = configs.hill(256, 128, 64, H=16.0, L=40.0, x0=64.0, y0=64.0).cast(np.float32)
    g = wl.grid
    _say("autotune 256x128x64 f32 mixed")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ibm.Context(g.nx, g.ny, g.nz, dtype=torch.float32, precision="mixed", device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), 1.5, 1.5)
    path = str(tmp_path / "tune.json")
    vel = [T(wl.u), T(wl.v), T(wl.w)]
    pu, pw = T(wl.phi_uv), T(wl.phi_w)

    def sgs():
        tau = [torch.empty_like(vel[0]) for _ in range(6)]
        ctx.sgs_stress(pu, pw, *vel, tau, z0=1e-3)
        return [t.cpu().numpy() for t in tau]

    before = sgs()                                 # on the default tile
    t1 = ctx.autotune(path)
    entries = json.load(open(path))
    assert len(entries) == 2                       # the dense pass's shape and the Smagorinsky kernel's
    dense = [v for k, v in entries.items() if k.endswith("|plain")]
    own = [v for k, v in entries.items() if k.endswith("|sgs")]
    assert len(dense) == 1 and dense[0][:4] == list(t1) and len(own) == 1 and own[0][1] == 1
    after = sgs()                                  # on its own tuned tile
    assert all(np.array_equal(x, y) for x, y in zip(before, after))
    ctx.set_tile(1, 1, 4, 1)
    t2 = ctx.autotune(path)                        # read back from the cache
    assert t2 == t1
    t3 = ctx.autotune(path, force=True, batch=True)
    assert t3[1] <= 2 and len(json.load(open(path))) == 3
    # the divergence does not depend on the tile shape
    wls = _cases("f32")[:3]
    b, fs = _batch(wls, None, torch.float32, "mixed", dev)
    b.tune(path)
    b.run()
    torch.cuda.synchronize()
    for i, (w, f) in enumerate(zip(wls, fs)):
        tile = b.case(i).get_tile()
        assert tile[1] <= 2
        _same(f.snapshot(), _plain(w, tile, torch.float32, "mixed", dev), f"tuned case {i}")


DEGENERATE = [(1, 1, 12), (7, 1, 9), (1, 6, 9), (33, 5, 1), (20, 2, 2), (130, 9, 8)]
DEGENERATE_TILES = {"f32": [(1, 1, 4, 1), (1, 2, 3, 1), (1, 1, 16, 1), (1, 1, 1, 1), (4, 1, 2, 1),
                            (2, 2, 5, 1)],
                    "f64": [(1, 1, 4, 1), (1, 1, 5, 1), (1, 2, 2, 1), (1, 2, 1, 1), (2, 2, 3, 1),
                            (2, 1, 5, 1)]}


@pytest.mark.parametrize("dtype,prec", [("f32", "mixed"), ("f64", "plain")])
def test_degenerate_cases(ora, dtype, prec):
    """Cases of one column, one row, one or two planes and a ragged grid in one
    batch, each with its own tile: every case equals its plain calls bit for
    bit, and one of them the oracle.  (Cases with vx > 1 keep their stacked
    stress and divergence components 16-byte aligned, as binding requires.)"""
    torch, dev = torch_dev()
    tdt = torch.float32 if dtype == "f32" else torch.float64
    wls = []
    for i, shape in enumerate(DEGENERATE):
        wl = configs.flat(Grid(*shape), 1.25, theta=0.4, z0=1e-3, noise=0.3, tau_std=0.01,
                          gp_std=0.1, seed=7 + i)
        assert wl.band_width == 1.5 and wl.phi_c == 1.5      # as the batch prepares them
        wls.append(wl.cast(np.float32) if dtype == "f32" else wl)
    tiles = DEGENERATE_TILES[dtype]
    _say(f"batch of degenerate cases {DEGENERATE} {dtype} {prec}")
    b, fs = _batch(wls, tiles, tdt, prec, dev)
    b.run()
    torch.cuda.synchronize()
    for i, (w, f) in enumerate(zip(wls, fs)):
        _same(f.snapshot(), _plain(w, tiles[i], tdt, prec, dev), f"case {i} {DEGENERATE[i]}")
    ref = ora.stage(wls[5])
    out = dict(tau=fs[5].tau.cpu().numpy(), div=fs[5].div.cpu().numpy(),
               ustar=fs[5].ustar.cpu().numpy(), drag=fs[5].drag.cpu().numpy(),
               stats=fs[5].stats.cpu().numpy(), mask=b.case(5).mask(), counts=b.case(5).counts())
    compare(out, ref, wls[5], TOL[dtype])


def _random_ensemble(seed, dtype):
    """Seeded random ensemble: 6-10 cases of random shapes (a few degenerate:
    one row, one column, one or two planes), bump terrains or flat walls, and
    random tile shapes (vx > 1 only where the row splits into whole vectors
    and the stacked fields stay 16-byte aligned)."""
    rng = np.random.Generator(np.random.PCG64(200603343 + 77 + seed))
    ncase = int(rng.integers(6, 11))
    wls, tiles = [], []
    for i in range(ncase):
        if rng.random() < 0.3:
            shape = (int(rng.integers(1, 90)), int(rng.integers(1, 6)), int(rng.integers(1, 12)))
            wl = configs.flat(Grid(*shape), float(rng.choice([1.0, 1.25, 1.5, 1.75])), theta=0.4,
                              z0=1e-3, noise=0.3, tau_std=0.01, gp_std=0.1, seed=seed * 100 + i)
        else:
            shape = (int(rng.integers(8, 140)), int(rng.integers(4, 48)), int(rng.integers(6, 40)))
            wl = configs.bumps_case(1000 + 100 * seed + i, shape)
        wls.append(wl.cast(np.float32) if dtype == "f32" else wl)
        n = shape[0] * shape[1] * shape[2]
        vmax, item = (4, 4) if dtype == "f32" else (2, 8)
        # vx > 1 needs each stacked stress and divergence component 16-byte aligned
        vx = int(rng.choice([v for v in (1, 2, 4)
                             if v <= vmax and shape[0] % v == 0 and (v == 1 or n * item % 16 == 0)]))
        tiles.append((vx, int(rng.choice([1, 2])), int(rng.integers(1, 33)), 1))
    return wls, tiles


@pytest.mark.parametrize("seed,dtype,prec", [(0, "f32", "mixed"), (1, "f32", "mixed"),
                                             (2, "f64", "plain")])
def test_random_ensembles_equal_plain_calls(ora, seed, dtype, prec):
    """Batches of random grids and tile shapes (uneven work items, slices of
    very different lengths, cases with and without forcing): every case equals
    its plain per-case calls bit for bit, after the eager run and after a
    captured graph's launch; the largest case also against the oracle."""
    torch, dev = torch_dev()
    tdt = torch.float32 if dtype == "f32" else torch.float64
    wls, tiles = _random_ensemble(seed, dtype)
    shapes = [(w.grid.nx, w.grid.ny, w.grid.nz) for w in wls]
    _say(f"random ensemble seed {seed} {dtype} {prec}: {list(zip(shapes, tiles))}")
    b, fs = _batch(wls, tiles, tdt, prec, dev)
    plain = [_plain(w, tiles[i], tdt, prec, dev) for i, w in enumerate(wls)]
    b.run()
    torch.cuda.synchronize()
    for i, f in enumerate(fs):
        _same(f.snapshot(), plain[i], f"eager case {i} {shapes[i]} tile {tiles[i]}")
    for f in fs:
        f.reset()
    b.capture()
    b.launch()
    torch.cuda.synchronize()
    for i, f in enumerate(fs):
        _same(f.snapshot(), plain[i], f"graph case {i} {shapes[i]} tile {tiles[i]}")
    big = int(np.argmax([np.prod(s) for s in shapes]))
    ref = ora.stage(wls[big])
    out = dict(tau=fs[big].tau.cpu().numpy(), div=fs[big].div.cpu().numpy(),
               ustar=fs[big].ustar.cpu().numpy(), drag=fs[big].drag.cpu().numpy(),
               stats=fs[big].stats.cpu().numpy(), mask=b.case(big).mask(),
               counts=b.case(big).counts())
    compare(out, ref, wls[big], TOL[dtype])


def test_ensemble_full_size(ora, tmp_path):
    """The 64-case ensemble as the benchmark times it (105.6 M points, float32
    mixed, tiles from the shipped autotuner cache, one graph launch): every
    case equal bit for bit to plain per-case calls on the same tile (stress,
    divergence, forced velocity, drag, statistics), which covers the late
    items of each XCD work slice; one case of each grid shape and the last
    case of the work list against the oracle's stage, every node."""
    import shutil
    import paper_2006_03343_amd as ibm
    torch, dev = torch_dev()
    shapes = configs.ensemble_shapes(64)
    wls = [configs.bumps_case(i, s).cast(np.float32) for i, s in enumerate(shapes)]
    _say(f"ensemble of {len(wls)} cases, {sum(a * b * c for a, b, c in shapes)} points, f32 mixed")
    cache = str(tmp_path / "tune.json")
    shutil.copy(os.path.join(os.path.dirname(ibm.__file__), "tune_gfx950.json"), cache)
    b, fs = _batch(wls, None, torch.float32, "mixed", dev)
    b.tune(cache)
    b.capture()
    b.launch()
    torch.cuda.synchronize()
    for i, (w, f) in enumerate(zip(wls, fs)):
        tile = b.case(i).get_tile()
        _same(f.snapshot(), _plain(w, tile, torch.float32, "mixed", dev), f"case {i} tile {tile}")
    _say("all 64 cases equal the plain calls bit for bit")
    picked = sorted({s: i for i, s in reversed(list(enumerate(shapes)))}.values())
    for i in picked + [len(wls) - 1]:
        _say(f"case {i} {shapes[i]} tile {b.case(i).get_tile()} vs the oracle")
        out = dict(tau=fs[i].tau.cpu().numpy(), div=fs[i].div.cpu().numpy(),
                   ustar=fs[i].ustar.cpu().numpy(), drag=fs[i].drag.cpu().numpy(),
                   stats=fs[i].stats.cpu().numpy(), mask=b.case(i).mask(),
                   counts=b.case(i).counts())
        errs = compare(out, ora.stage(wls[i]), wls[i], TOL["f32"])
        _say(f"errors {errs}")


def test_batch_beyond_2_31_nodes_in_total(ora):
    """Two float32 mixed cases of 4096 x 4096 x 64 (1.07e9 nodes each, 2^31 in
    all): the batched kernels index each case from its own bases.  Each case is
    64 x 64 periodic copies of a 64 x 64 x 64 hill cell, so every copy's outputs
    equal the first's bit for bit and the first meets the bar against the
    oracle's stage on the cell; counts, drag and band statistics are 4096 times
    the cell's."""
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    if torch.cuda.get_device_properties(dev).total_memory < 230 * 2 ** 30:
        pytest.skip("needs about 190 GiB of device memory")
    torch.cuda.empty_cache()
    cells = [configs.hill(64, 64, 64, H=8.0, L=24.0, x0=32.0, y0=32.0).cast(np.float32),
             configs.hill(64, 64, 64, H=12.0, L=20.0, x0=28.0, y0=36.0, seed_offset=1).cast(np.float32)]
    g = cells[0].grid
    rx = ry = 64
    reps = rx * ry
    nx, ny, nz = g.nx * rx, g.ny * ry, g.nz
    assert 2 * nx * ny * nz >= 2 ** 31
    _say(f"batch of 2 cases {nx}x{ny}x{nz} f32 mixed, {rx}x{ry} copies of hill cells")
    big = lambda a: tiled(a, torch.float32, ry, rx)
    b = ibm.Batch([(nx, ny, nz)] * 2, dtype=torch.float32, precision="mixed", device=dev)
    b.prepare([big(c.phi_uv) for c in cells], [big(c.phi_w) for c in cells], cells[0].band_width,
              [c.z0 for c in cells], phi_c=cells[0].phi_c)
    io = []
    for i, c in enumerate(cells):
        u, v, w = big(c.u), big(c.v), big(c.w)
        d = dict(u=u, v=v, w=w, tau=[big(t) for t in c.tau], gp=[big(t) for t in c.gradp],
                 ustar=[u.clone(), v.clone(), w.clone()], div=[torch.empty_like(u) for _ in range(3)],
                 drag=torch.zeros(3, dtype=torch.float64, device=dev),
                 stats=torch.zeros(4, dtype=torch.float64, device=dev))
        b.bind(i, u, v, w, d["tau"], d["ustar"], d["div"], gradp=d["gp"], dt=c.dt, drag=d["drag"],
               stats=d["stats"])
        io.append(d)
    b.run()
    torch.cuda.synchronize()
    for i, (c, d) in enumerate(zip(cells, io)):
        out = {k: np.stack([first_copy(f, g.shape, ry, rx) for f in d[k]])
               for k in ("tau", "div", "ustar")}
        ref = ora.stage(c)
        mask = b.case(i).mask().reshape(nz, ry, g.ny, rx, g.nx)
        for k in range(nz):
            assert (mask[k] == ref["mask"][k][None, :, None, :]).all(), f"case {i} plane {k}"
        del mask
        assert list(b.case(i).counts()) == [reps * int(x) for x in ref["counts"]]
        out.update(mask=ref["mask"], counts=ref["counts"], drag=None, stats=None)
        errs = compare(out, ref, c, TOL["f32"])
        scale = reps * g.dv * np.array([np.abs(x).sum() for x in ref["div"]])
        errs["drag"] = float(np.max(np.abs(d["drag"].cpu().numpy() - reps * ref["drag"]) / scale))
        st, s_ref = d["stats"].cpu().numpy(), ref["stats"]
        errs["stats_sum"] = float(np.abs(st[:2] - reps * s_ref[:2]).max() / (reps * np.abs(s_ref[:2]).max()))
        errs["stats_max"] = abs(st[2] - s_ref[2]) / s_ref[2]
        assert st[3] == reps * s_ref[3]
        _say(f"case {i} errors {errs}")
        assert max(errs.values()) <= TOL["f32"], errs
    del b, io
    torch.cuda.empty_cache()
