"""Benchmark of the wall-modeled IBM stage on one MI355X.

One step = one stage pass over the whole grid through ibm_stage: the wall
stress (band wall model + solid zeroing + band statistics) and the dense
pass (stress divergence + in-body forcing + drag), on the axisymmetric cos^2 hill
512 x 256 x 256 (H = 32, L = 80 cells, z0 = 2e-4 H), float32 storage in the
mixed-precision mode.  Inputs are generated (seeded, synthetic), copied to
HBM and the geometry prepared before the timed region.

Printed: one JSON line.  ``value`` is grid points per second of the stage
(nx*ny*nz*steps / time of ``steps`` back-to-back passes between two HIP
events).  ``stage`` gives the whole pass's fraction of the HBM roofline on
its algorithmic bytes (dense pass, solid zeroing, band records, one read of
every velocity node the samples touch) and the time of the same pass as two
calls (ibm_wall_stress, ibm_apply).  ``roofline`` is the dense kernel (ibm_apply): algorithmic bytes per
launch divided by its mean launch duration, from HIP events on the kernel's
stream around ``steps`` back-to-back launches of it in the same run.  ``fp64_plain`` repeats the measurement with float64 storage.
``cpu_baseline`` times the FP64 CPU oracle (a test checker, never tuned) on
full passes of the same hill.  ``batched`` compares the 64-case ensemble of
Gaussian-bump terrains advanced by one hipGraph launch of the batched kernels
(float32, mixed) with the same cases advanced by plain per-case float64 calls.
``adjoint`` times the stage, the forward pass and the hand-written reverse
mode on the 256 x 128 x 128 fractal terrain with a per-node log z0 field
(float32 mixed), and on a 512 x 256 x 256 fractal whose working set is well
above the 256 MB Infinity Cache; the reverse mode's roofline is against its
algorithmic bytes (``adjoint_bytes``).
``chester`` times Chester et al.'s original method (wall model in its fluid
band, extrapolation into a solid band, 10 red-black SOR sweeps over the body)
beside the simplified stage on the same hill.
``sgs`` times the Smagorinsky stress with Mason's wall damping that feeds
the stage (ibm_sgs_stress, float32 on the same hill: its roofline against
44 algorithmic bytes per node) and the three calls in a row (SGS stress, wall
stress, dense pass).
``spectral`` times ibm_apply_spectral, the dense pass with the paper's
pseudo-spectral horizontal derivatives, on the same hill (three launches:
x transforms, y transforms, vertical differences with forcing and drag).
``terrains`` reports the same figures for the wall-mounted cube (64 x 32 x 32,
float64; cache-resident, so no roofline claim) and the 2-D ridge
(256 x 128 x 128, 100 passes in float64, float32 and float32 mixed; its
float32 working set fits the 256 MB Infinity Cache, so its fraction is
flagged).  Dense-pass tile shapes come from the autotuner's cache shipped with
the package (``--retune`` times them again and rewrites it).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
WARM_MS = 150.0                # minimum warm-up of each leg after the headline, ms
TUNE_CACHE = os.environ.get("IBM_TUNE_CACHE",
                            os.path.join(ROOT, "paper_2006_03343_amd", "tune_gfx950.json"))
PROFILE = os.path.join(ROOT, "profiles", "k_apply_hill512x256x256_f32_mixed.txt")


def measured_traffic(tile):
    """HBM bytes per k_apply launch from the committed counter profile, if the
    dense pass's device code and launch code (kernels.h, and stage.hip up to
    the end of its anonymous namespace) and the tile shape are the ones that
    were profiled."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2006_03343_amd", "csrc")
    stage = open(os.path.join(csrc, "stage.hip"), "rb").read()
    stage = stage[:stage.index(b"}  // namespace\n")]
    h = hashlib.sha256(open(os.path.join(csrc, "kernels.h"), "rb").read() + stage).hexdigest()
    try:
        lines = open(PROFILE).read().splitlines()
    except OSError:
        return None
    kv = dict(ln.split(": ", 1) for ln in lines if ": " in ln and not ln.startswith(" "))
    if kv.get("source_sha256 (csrc/kernels.h + launch half of csrc/stage.hip)") != h:
        return None
    if kv.get("tile") != ",".join(str(x) for x in tile):
        return None
    return int(kv["traffic_bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def apply_bytes(wl, mask, s):
    """Algorithmic HBM bytes of one ibm_apply launch."""
    g = wl.grid
    n = g.n
    wrow = (g.nx + 15) // 16
    f_uv = int(((mask >> 4) & 1).sum())
    f_w = int(((mask >> 5) & 1).sum())
    dense = n * 9 * s                       # read 6 stress components, write 3 divergence
    flags = g.ny * g.nz * wrow * 4          # 2-bit forcing flags
    forcing = f_uv * 4 * s + f_w * 2 * s    # read grad p, write u* at forced nodes
    return dense + flags + forcing


def gathered_nodes(ctx, wl):
    """Distinct velocity nodes the band records' trilinear samples touch:
    (uv-grid nodes, read for u and v; w-grid nodes, read for w).  The sample
    point of a record at node x is x + (phi_c - phi) n (the exported unit
    normal); index coordinates periodic in x and y, vertical clamped."""
    import numpy as np
    g = wl.grid
    touched = [set(), set()]
    uvn, wn = [], []
    for grid, phi, zoff in ((0, wl.phi_uv, 0.5), (1, wl.phi_w, 0.0)):
        idx, nrm = ctx.band(grid)
        if idx.size == 0:
            continue
        k, j, i = np.unravel_index(idx.astype(np.int64), g.shape)
        ph = np.asarray(phi, np.float64).ravel()[idx]
        shift = wl.phi_c - ph
        px = i * g.dx + shift * nrm[:, 0]
        py = j * g.dy + shift * nrm[:, 1]
        pz = (k + zoff) * g.dz + shift * nrm[:, 2]
        for kind, out in ((0, uvn), (1, wn)):
            zi = np.clip(pz / g.dz - (0.5 if kind == 0 else 0.0), 0, g.nz - 1)
            i0 = np.floor(px / g.dx).astype(np.int64)
            j0 = np.floor(py / g.dy).astype(np.int64)
            k0 = np.floor(zi).astype(np.int64)
            for di in (0, 1):
                for dj in (0, 1):
                    for dk in (0, 1):
                        kk = np.minimum(k0 + dk, g.nz - 1)
                        out.append((kk * g.ny + (j0 + dj) % g.ny) * g.nx + (i0 + di) % g.nx)
    n_uv = int(np.unique(np.concatenate(uvn)).size) if uvn else 0
    n_w = int(np.unique(np.concatenate(wn)).size) if wn else 0
    return n_uv, n_w


def stage_bytes(wl, mask, s, gathered):
    """Algorithmic HBM bytes of one whole stage pass: the dense pass
    (``apply_bytes``), the solid zeroing, the band records' minimum (index,
    normal, phi) and stress writes, and one read of every velocity node the
    samples touch (u and v on the uv grid, w on the w grid)."""
    band_uv = int(((mask & 3) == 1).sum())
    band_w = int((((mask >> 2) & 3) == 1).sum())
    solid_uv = int(((mask & 3) == 2).sum())
    solid_w = int((((mask >> 2) & 3) == 2).sum())
    return (apply_bytes(wl, mask, s) + solid_uv * 4 * s + solid_w * 2 * s
            + band_uv * (4 + 4 * s + 4 * s) + band_w * (4 + 4 * s + 2 * s)
            + s * (2 * gathered[0] + gathered[1]))


def run_gpu(wl, dtype, precision, steps, warmup, tile=None, min_warm_ms=0.0):
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    dev = torch.device("cuda", 0)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, tdt)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=tdt, precision=precision,
                      device=dev)
    t0 = time.time()
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    torch.cuda.synchronize()
    t_prep = time.time() - t0
    if tile:
        ctx.set_tile(*tile)
    else:
        ctx.autotune(TUNE_CACHE)
    u, v, w = T(wl.u), T(wl.v), T(wl.w)
    tau = torch.stack([T(t) for t in wl.tau]).contiguous()
    gp = [T(t) for t in wl.gradp]
    ustar = torch.stack([u, v, w]).contiguous()
    div = torch.empty_like(ustar)
    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    drag = torch.zeros(3, dtype=torch.float64, device=dev)
    taus, uss, divs = list(tau), list(ustar), list(div)

    def step():
        ctx.stage(u, v, w, taus, uss, divs, z0=wl.z0, gradp=gp, dt=wl.dt, stats=stats,
                  drag=drag)

    def two_calls():
        ctx.wall_stress(u, v, w, taus, z0=wl.z0, stats=stats)
        ctx.apply(taus, uss, divs, gradp=gp, dt=wl.dt, drag=drag)

    def both():
        step()
        two_calls()

    # the headline takes exactly ``warmup`` warm-up steps; the other legs also
    # warm up for at least min_warm_ms
    _warm(both, warmup, min_warm_ms)
    # the timed region: ``steps`` back-to-back steps between two events
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for _ in range(steps):
        step()
    end.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(end)
    # per-kernel launch durations: each call ``steps`` times back to back
    # between two events on the launch stream (a pass is idempotent: the
    # stress and forced velocity it writes do not change its inputs), so the
    # mean is the launch's duration plus the inter-launch gap of the queue
    def each(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ws_ms = each(lambda: ctx.wall_stress(u, v, w, taus, z0=wl.z0, stats=stats))
    ap_ms = each(lambda: ctx.apply(taus, uss, divs, gradp=gp, dt=wl.dt, drag=drag))
    two_ms = each(two_calls)
    mask = ctx.mask()
    res = dict(ms_per_step=total_ms / steps, wall_s=t_wall, wall_stress_ms=ws_ms, apply_ms=ap_ms,
               two_calls_ms=two_ms, prepare_s=t_prep, tile=ctx.get_tile(),
               counts=[int(x) for x in ctx.counts()], mask=mask,
               gathered=gathered_nodes(ctx, wl), drag=drag.cpu().tolist(),
               stats=stats.cpu().tolist())
    del ctx, u, v, w, tau, gp, ustar, div
    torch.cuda.empty_cache()
    return res


def _warm(fn, warmup, min_ms=WARM_MS):
    """``warmup`` untimed calls of ``fn``, then more until ``min_ms`` of wall
    time has passed, so a leg's short timed region does not start while the
    GPU's clocks are still rising after the host-side set-up before it."""
    import torch
    t0 = time.perf_counter()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    while (time.perf_counter() - t0) * 1e3 < min_ms:
        fn()
        torch.cuda.synchronize()


def stream_triad(n=33554432, reps=50):
    """The GPU's measured streaming rate: torch's c = a + 0.5 b on float32
    fields of n elements (3 x 134 MB at the default, above the 256 MB
    Infinity Cache), 12 bytes per element per call, timed over ``reps`` calls
    after a warm-up."""
    import torch
    dev = torch.device("cuda", 0)
    a = torch.rand(n, device=dev)
    b = torch.rand(n, device=dev)
    c = torch.empty_like(a)
    _warm(lambda: torch.add(a, b, alpha=0.5, out=c), 5)
    e0, e1 = _events(2)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.add(a, b, alpha=0.5, out=c)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b, c
    torch.cuda.empty_cache()
    return 12.0 * n / (ms * 1e-3) / 1e9


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def run_ensemble(steps, warmup, ncases=64):
    """64 Gaussian-bump terrains on uneven grids: batched float32 (mixed) graph
    launches vs plain per-case float64 calls."""
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    from workloads import configs
    dev = torch.device("cuda", 0)
    shapes = configs.ensemble_shapes(ncases)
    t0 = time.time()
    f32, f64 = [], []
    z0 = []
    for i, shp in enumerate(shapes):
        wl = configs.bumps_case(i, shp)
        z0.append(wl.z0)
        for store, tdt in ((f32, torch.float32), (f64, torch.float64)):
            if tdt == torch.float32:
                w = wl.cast(np.float32)
            else:
                w = wl
            T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, tdt)
            d = dict(phi_uv=T(w.phi_uv), phi_w=T(w.phi_w), u=T(w.u), v=T(w.v), w=T(w.w),
                     tau=torch.stack([T(t) for t in w.tau]).contiguous(),
                     gp=[T(t) for t in w.gradp], dt=w.dt)
            d["ustar"] = torch.stack([d["u"], d["v"], d["w"]]).contiguous()
            d["div"] = torch.empty_like(d["ustar"])
            d["drag"] = torch.zeros(3, dtype=torch.float64, device=dev)
            d["stats"] = torch.zeros(4, dtype=torch.float64, device=dev)
            store.append(d)
        del wl
    npts = sum(a * b * c for a, b, c in shapes)
    log(f"ensemble: {ncases} cases, {npts} points, generated in {time.time() - t0:.1f} s")
    # batched float32, mixed precision, one graph launch per step
    b = ibm.Batch(shapes, dtype=torch.float32, precision="mixed", device=dev)
    b.prepare([d["phi_uv"] for d in f32], [d["phi_w"] for d in f32], 1.5, z0, phi_c=1.5)
    b.tune(TUNE_CACHE)
    for i, d in enumerate(f32):
        b.bind(i, d["u"], d["v"], d["w"], list(d["tau"]), list(d["ustar"]), list(d["div"]),
               gradp=d["gp"], dt=d["dt"], drag=d["drag"], stats=d["stats"])
    b.capture()
    _warm(b.launch, warmup)
    e0, e1 = _events(2)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        b.launch()
    e1.record()
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1) / steps
    # plain float64: two calls per case per step
    ctxs = []
    for shp, d, z in zip(shapes, f64, z0):
        c = ibm.Context(*shp, dtype=torch.float64, device=dev)
        c.prepare(d["phi_uv"], d["phi_w"], 1.5, 1.5)
        c.autotune(TUNE_CACHE)
        ctxs.append((c, d, z))

    def plain_step():
        for c, d, z in ctxs:
            c.wall_stress(d["u"], d["v"], d["w"], list(d["tau"]), z0=z, stats=d["stats"])
            c.apply(list(d["tau"]), list(d["ustar"]), list(d["div"]), gradp=d["gp"], dt=d["dt"],
                    drag=d["drag"])

    _warm(plain_step, warmup)
    steps64 = max(5, steps // 4)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps64):
        plain_step()
    e1.record()
    torch.cuda.synchronize()
    ms64 = e0.elapsed_time(e1) / steps64
    res = {"cases": ncases, "points": npts, "shapes": sorted(set(shapes)),
           "f32_mixed_batched_graph": {"value": npts / (ms32 * 1e-3), "ms_per_step": ms32,
                                       "launches_per_step": 1},
           "f64_plain_per_case": {"value": npts / (ms64 * 1e-3), "ms_per_step": ms64,
                                  "launches_per_step": 4 * ncases},
           "ratio": ms64 / ms32}
    del b, ctxs, f32, f64
    torch.cuda.empty_cache()
    return res


def adjoint_bytes(n, s, flags, nrec, gathered):
    """Algorithmic HBM bytes of one ibm_stage_vjp call (no stress cotangent,
    a log z0 field): per node g_ustar read and gu, gv, gw, glog_z0 written
    (7 s) and the forcing flags; per band record its index, normal and phi
    (4 + 4 s), its log z0 read and glog_z0 written (2 s) and the three
    divergence cotangents at its node (3 s); one read of every velocity node
    the samples touch (u, v on the uv grid, w on the w grid)."""
    return n * 7 * s + flags + nrec * (4 + 4 * s + 2 * s + 3 * s) + s * (2 * gathered[0] + gathered[1])


def run_adjoint(steps, warmup, shape=(256, 128, 128)):
    """The stage (ibm_stage), the autograd forward and the reverse mode on the
    fractal terrain with a per-node log z0 field (float32, mixed)."""
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    from workloads import configs
    dev = torch.device("cuda", 0)
    wl = configs.fractal(*shape).cast(np.float32)
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ibm.Context(g.nx, g.ny, g.nz, dtype=torch.float32, precision="mixed", device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    ctx.autotune(TUNE_CACHE)
    u, v, w, lz = T(wl.u), T(wl.v), T(wl.w), T(wl.log_z0)
    tau0 = [T(t) for t in wl.tau]
    gp = [T(t) for t in wl.gradp]
    fwd = lambda: ibm.stage_forward(ctx, u, v, w, tau0, gp, wl.dt, log_z0=lz)
    tau, div, us, drag = fwd()
    bwd = lambda: ctx.vjp(u, v, w, list(div), list(us), [1.0, 0.0, 0.0], log_z0=lz)
    ts = [t.clone() for t in tau0]
    ust = [x.clone() for x in (u, v, w)]
    dv = [torch.empty_like(u) for _ in range(3)]
    dr = torch.zeros(3, dtype=torch.float64, device=dev)
    stage = lambda: ctx.stage(u, v, w, ts, ust, dv, log_z0=lz, gradp=gp, dt=wl.dt, drag=dr)
    def all_three():
        fwd()
        bwd()
        stage()

    _warm(all_three, warmup)
    e0, e1, e2, e3 = _events(4)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        fwd()
    e1.record()
    for _ in range(steps):
        bwd()
    e2.record()
    for _ in range(steps):
        stage()
    e3.record()
    torch.cuda.synchronize()
    f_ms, b_ms = e0.elapsed_time(e1) / steps, e1.elapsed_time(e2) / steps
    s_ms = e2.elapsed_time(e3) / steps
    counts = ctx.counts()
    nrec = int(counts[1] + counts[4])
    gathered = gathered_nodes(ctx, wl)
    flags = g.ny * g.nz * ((g.nx + 15) // 16) * 4
    nb = adjoint_bytes(g.n, 4, flags, nrec, gathered)
    gbs = nb / (b_ms * 1e-3) / 1e9
    del ctx
    torch.cuda.empty_cache()
    return {"workload": f"fractal {g.nx}x{g.ny}x{g.nz}, per-node log z0, f32 mixed",
            "band_records": nrec, "stage_ms": s_ms, "forward_ms": f_ms, "backward_ms": b_ms,
            "backward_over_stage": b_ms / s_ms,
            "backward_points_per_s": g.n / (b_ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_call": nb},
            "note": "stage = ibm_stage; forward = the autograd op's out-of-place pass incl. "
                    "tensor copies; backward = ibm_stage_vjp"}


def run_chester(wl, steps, warmup, omega=1.5, sweeps=10):
    """Chester et al.'s original method against the simplified stage on the
    same hill (float32 mixed): ibm_chester_wall_stress (wall model on its
    fluid band, extrapolation into the solid band, ``sweeps`` red-black SOR
    sweeps over the body interior) followed by ibm_apply, against ibm_stage;
    also with no sweep (steps 1 and 2 alone) and the cost per sweep."""
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    dev = torch.device("cuda", 0)
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=torch.float32,
                      precision="mixed", device=dev)
    pu, pw = T(wl.phi_uv), T(wl.phi_w)
    ctx.prepare(pu, pw, wl.band_width, wl.phi_c, wl.kappa)
    ctx.autotune(TUNE_CACHE)
    t0 = time.time()
    ctx.chester_prepare(pu, pw)
    torch.cuda.synchronize()
    t_prep = time.time() - t0
    u, v, w = T(wl.u), T(wl.v), T(wl.w)
    tau = [T(t) for t in wl.tau]
    gp = [T(t) for t in wl.gradp]
    ustar = [u.clone(), v.clone(), w.clone()]
    div = [torch.empty_like(u) for _ in range(3)]
    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    drag = torch.zeros(3, dtype=torch.float64, device=dev)

    def chester(n):
        ctx.chester_wall_stress(u, v, w, tau, omega, n, z0=wl.z0, stats=stats)
        ctx.apply(tau, ustar, div, gradp=gp, dt=wl.dt, drag=drag)

    def simplified():
        ctx.stage(u, v, w, tau, ustar, div, z0=wl.z0, gradp=gp, dt=wl.dt, stats=stats,
                  drag=drag)

    def timed(fn):
        _warm(fn, warmup)
        e0, e1 = _events(2)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_simple = timed(simplified)
    ms_ch = timed(lambda: chester(sweeps))
    ms_ch0 = timed(lambda: chester(0))
    counts = [int(x) for x in ctx.chester_counts()]
    del ctx, tau, ustar, div
    torch.cuda.empty_cache()
    return {"workload": f"hill {g.nx}x{g.ny}x{g.nz}, float32 mixed, omega {omega}",
            "sweeps": sweeps, "chester_ms": ms_ch, "chester_points_per_s": g.n / (ms_ch * 1e-3),
            "chester_no_sweep_ms": ms_ch0, "ms_per_sweep": (ms_ch - ms_ch0) / sweeps,
            "simplified_ms": ms_simple, "chester_over_simplified": ms_ch / ms_simple,
            "chester_prepare_s": t_prep,
            "classes_uv": dict(zip(("fluid", "fluid_band", "solid_band", "interior"), counts[:4])),
            "classes_w": dict(zip(("fluid", "fluid_band", "solid_band", "interior"), counts[4:])),
            "launches_per_step": {"chester": 4 + 2 * sweeps + 1, "simplified": 3},
            "note": "chester = ibm_chester_wall_stress + ibm_apply; simplified = ibm_stage; "
                    "both one GPU, same inputs"}


def run_sgs(wl, steps, warmup):
    """ibm_sgs_stress on the hill (float32), alone and followed by the stage;
    the fused ibm_apply_sgs after the wall stress against that sequence."""
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    dev = torch.device("cuda", 0)
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=torch.float32,
                      precision="mixed", device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    ctx.autotune(TUNE_CACHE)
    pu, pw, u, v, w = (T(x) for x in (wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w))
    tau = torch.empty((6,) + g.shape, dtype=torch.float32, device=dev)
    taus = list(tau)
    gp = [T(t) for t in wl.gradp]
    ustar = torch.stack([u, v, w]).contiguous()
    div = torch.empty_like(ustar)
    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    drag = torch.zeros(3, dtype=torch.float64, device=dev)
    sgs = lambda: ctx.sgs_stress(pu, pw, u, v, w, taus, z0=wl.z0, kappa=wl.kappa)

    def step():
        sgs()
        ctx.wall_stress(u, v, w, taus, z0=wl.z0, stats=stats)
        ctx.apply(taus, list(ustar), list(div), gradp=gp, dt=wl.dt, drag=drag)

    def timed(fn):
        _warm(fn, warmup)
        e0, e1 = _events(2)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    fused = lambda: ctx.apply_sgs(pu, pw, u, v, w, taus, list(ustar), list(div), z0=wl.z0,
                                  kappa=wl.kappa, gradp=gp, dt=wl.dt, drag=drag)

    def fused_step():
        ctx.wall_stress(u, v, w, taus, z0=wl.z0, stats=stats)
        fused()

    ms_sgs = timed(sgs)
    ms_all = timed(step)
    ms_fused_step = timed(fused_step)
    ms_fused = timed(fused)
    gbs = g.n * 11 * 4 / (ms_sgs * 1e-3) / 1e9
    # fused pass, algorithmic: u, v, w, phi_uv, phi_w and the class byte in,
    # div out, the band stress at band nodes, forcing at forced nodes
    mask = ctx.mask()
    band_uv = int(((mask & 3) == 1).sum())
    band_w = int((((mask >> 2) & 3) == 1).sum())
    f_uv = int(((mask >> 4) & 1).sum())
    f_w = int(((mask >> 5) & 1).sum())
    fused_bytes = g.n * (5 * 4 + 1 + 3 * 4) + band_uv * 16 + band_w * 8 + f_uv * 16 + f_w * 8
    fgbs = fused_bytes / (ms_fused * 1e-3) / 1e9
    del ctx, tau, ustar, div
    torch.cuda.empty_cache()
    return {"workload": f"hill {g.nx}x{g.ny}x{g.nz}, float32, cs 0.16, kappa {wl.kappa}",
            "sgs_ms": ms_sgs, "sgs_points_per_s": g.n / (ms_sgs * 1e-3),
            "sgs_roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                             "bytes_per_launch": g.n * 11 * 4},
            "sgs_wall_stress_apply_ms": ms_all,
            "sgs_wall_stress_apply_points_per_s": g.n / (ms_all * 1e-3),
            "wall_stress_apply_sgs_ms": ms_fused_step,
            "wall_stress_apply_sgs_points_per_s": g.n / (ms_fused_step * 1e-3),
            "fused_over_sequence": ms_all / ms_fused_step,
            "apply_sgs_ms": ms_fused,
            "apply_sgs_roofline": {"bound": "hbm", "achieved": fgbs, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": fgbs / HBM_PEAK_GBS,
                                   "bytes_per_launch": fused_bytes}}


def run_spectral(wl, steps, warmup):
    """ibm_apply_spectral on the hill (float32, mixed), after one wall stress."""
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    dev = torch.device("cuda", 0)
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=torch.float32,
                      precision="mixed", device=dev)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    ctx.autotune(TUNE_CACHE)
    u, v, w = T(wl.u), T(wl.v), T(wl.w)
    tau = [T(t) for t in wl.tau]
    gp = [T(t) for t in wl.gradp]
    ustar = [u.clone(), v.clone(), w.clone()]
    div = [torch.empty_like(u) for _ in range(3)]
    drag = torch.zeros(3, dtype=torch.float64, device=dev)
    ctx.wall_stress(u, v, w, tau, z0=wl.z0)
    fn = lambda: ctx.apply_spectral(tau, ustar, div, gradp=gp, dt=wl.dt, drag=drag)
    _warm(fn, warmup)
    e0, e1 = _events(2)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    mask = ctx.mask()
    wrow = (g.nx + 15) // 16
    # algorithmic: what the dense pass moves (6 stresses in, 3 divergences
    # out, flags, forcing); the passes: x 6 field accesses per node (3 in, 3
    # out), y 15 (3 stresses, 3 divergences read and written, 6 stress values
    # for the vertical differences), flags
    nbytes = apply_bytes(wl, mask, 4)
    pass_bytes = g.n * 4 * (6 + 15) + g.ny * g.nz * wrow * 4
    del ctx, tau, ustar, div
    torch.cuda.empty_cache()
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": f"hill {g.nx}x{g.ny}x{g.nz}, float32 mixed",
            "ms": ms, "points_per_s": g.n / (ms * 1e-3), "bytes_per_call": nbytes,
            "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "pass_bytes_per_call": pass_bytes,
            "pass_GBs": pass_bytes / (ms * 1e-3) / 1e9,
            "note": "2 launches and the drag finalize; frac on the algorithmic bytes of the "
                    "stage's dense pass, pass_GBs on what the two transform passes move"}


def run_projection(wl, steps, warmup):
    """ibm_ab2_predict and ibm_pressure_project on the hill's grid (float32):
    the time advance around the stage."""
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    dev = torch.device("cuda", 0)
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=torch.float32, device=dev)
    vel = [T(wl.u), T(wl.v), T(wl.w)]
    vel[2][0].zero_()
    rn = [T(t) for t in wl.tau[:3]]
    rp = [T(t) for t in wl.tau[3:]]
    ustar = [torch.empty_like(a) for a in vel]
    uo = [torch.empty_like(a) for a in vel]
    p = torch.empty_like(vel[0])

    def timed(fn):
        _warm(fn, warmup)
        e0, e1 = _events(2)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ab2_ms = timed(lambda: ctx.ab2_predict(vel, rn, rp, wl.dt, ustar))
    proj_ms = timed(lambda: ctx.pressure_project(ustar, wl.dt, uo, p))
    # algorithmic: AB2 reads u, rhs, rhs_prev and writes u* (3 components);
    # the projection reads u*, v*, w* and writes u, v, w, p
    ab2_bytes = g.n * 4 * 4 * 3
    proj_bytes = g.n * 4 * 7
    # what the passes move per node over half spectra (about 4 B per node per
    # complex field): forward x 24 (u*, v*, w* in, three spectra out),
    # forward y 20 (three in; H, w_hat out), the solve 28 (its workspace, p_hat
    # and the vertical difference out), inverse y 20 (p_hat and the difference
    # in; P, DY, DZ out), inverse x 44 (P twice, DY, DZ, u*, v*, w* in; p, u,
    # v, w out)
    pass_bytes = g.n * (24 + 20 + 28 + 20 + 44)
    del ctx, vel, rn, rp, ustar, uo, p
    torch.cuda.empty_cache()
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9
    return {"workload": f"{g.nx}x{g.ny}x{g.nz}, float32",
            "ab2_ms": ab2_ms, "ab2_GBs": gbs(ab2_bytes, ab2_ms),
            "ab2_frac": gbs(ab2_bytes, ab2_ms) / HBM_PEAK_GBS,
            "project_ms": proj_ms, "project_points_per_s": g.n / (proj_ms * 1e-3),
            "project_algorithmic_GBs": gbs(proj_bytes, proj_ms),
            "project_algorithmic_frac": gbs(proj_bytes, proj_ms) / HBM_PEAK_GBS,
            "project_pass_GBs": gbs(pass_bytes, proj_ms),
            "note": "projection: 5 launches (x forward, y forward, solve, y inverse, x "
                    "inverse) over half spectra; algorithmic bytes 28 per node, "
                    f"the passes move {pass_bytes // g.n} per node"}


def run_terrains(steps, warmup):
    """Stage throughput on the cube (float64) and the ridge (float64, float32,
    float32 mixed)."""
    import numpy as np

    from workloads import configs
    res = {}
    cube = configs.cube()
    ridge64 = configs.ridge()
    ridge32 = ridge64.cast(np.float32)
    for name, wl, dtype, prec, claim in (
            ("cube 64x32x32 f64 plain", cube, "f64", "plain", "none: cache-resident"),
            ("ridge 256x128x128 f64 plain", ridge64, "f64", "plain", "flagged: fits the MALL"),
            ("ridge 256x128x128 f32 plain", ridge32, "f32", "plain", "flagged: fits the MALL"),
            ("ridge 256x128x128 f32 mixed", ridge32, "f32", "mixed", "flagged: fits the MALL")):
        r = run_gpu(wl, dtype, prec, steps, warmup, min_warm_ms=WARM_MS)
        s = 8 if dtype == "f64" else 4
        gbs = apply_bytes(wl, r["mask"], s) / (r["apply_ms"] * 1e-3) / 1e9
        res[name] = {"value": wl.grid.n / (r["ms_per_step"] * 1e-3), "unit": "grid-points/s",
                     "ms_per_step": r["ms_per_step"], "apply_ms": r["apply_ms"],
                     "wall_stress_ms": r["wall_stress_ms"], "apply_GBs": gbs,
                     "apply_frac": gbs / HBM_PEAK_GBS, "roofline_claim": claim,
                     "tile": list(r["tile"])}
        log(f"{name}: {res[name]['value']:.3e} points/s, apply {gbs:.0f} GB/s")
    return res


def cpu_baseline(wl, budget_s=12.0, max_passes=40):
    """The FP64 oracle timed on full passes of the same workload (per-step work:
    wall stress, divergence, forcing, drag)."""
    import oracle
    g = wl.grid
    passes = 0
    t_total = 0.0
    while passes < max_passes and t_total < budget_s:
        t0 = time.perf_counter()
        tau, _ = oracle.wall_stress(g, wl.band_width, wl.phi_c, wl.kappa, wl.phi_uv, wl.phi_w,
                                    wl.u, wl.v, wl.w, wl.z0, wl.log_z0, wl.tau)
        div = oracle.divergence(g, tau)
        oracle.forcing(g, wl.phi_uv, wl.phi_w, (wl.u, wl.v, wl.w), wl.gradp, wl.dt)
        oracle.drag(g, wl.phi_uv, wl.phi_w, div)
        t_total += time.perf_counter() - t0
        passes += 1
    cores = oracle.num_threads()
    # the same pass with one thread, on a 256 x 128 x 128 hill
    from workloads import configs
    ws = configs.hill(256, 128, 128, H=16.0, L=40.0, x0=64.0, y0=64.0)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        tau1, _ = oracle.wall_stress(ws.grid, ws.band_width, ws.phi_c, ws.kappa, ws.phi_uv,
                                     ws.phi_w, ws.u, ws.v, ws.w, ws.z0, ws.log_z0, ws.tau)
        div1 = oracle.divergence(ws.grid, tau1)
        oracle.forcing(ws.grid, ws.phi_uv, ws.phi_w, (ws.u, ws.v, ws.w), ws.gradp, ws.dt)
        oracle.drag(ws.grid, ws.phi_uv, ws.phi_w, div1)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=g.n * passes / t_total, unit="grid-points/s", cores=cores,
                kind="oracle",
                sample=f"{passes} full FP64 pass(es) of the {g.nx}x{g.ny}x{g.nz} hill "
                       f"(wall stress, divergence, forcing, drag), {t_total:.1f} s",
                single_thread={"value": ws.grid.n / t1, "unit": "grid-points/s", "cores": 1,
                               "sample": f"one pass of a 256x128x128 hill, {t1:.1f} s"},
                host={"cpu": model, "nproc": os.cpu_count()})


def _oracle_rate(fn, points, what, budget_s=3.0):
    """The oracle timed beside a GPU leg: repeated calls within ``budget_s``."""
    import oracle
    calls, t = 0, 0.0
    while calls < 20 and t < budget_s:
        t0 = time.perf_counter()
        fn()
        t += time.perf_counter() - t0
        calls += 1
    return dict(value=points * calls / t, unit="grid-points/s", cores=oracle.num_threads(),
                kind="oracle", sample=f"{calls} call(s) on {what}, {t:.1f} s")


def cpu_oracle_rows(wl):
    """The oracle of the Smagorinsky stress, the spectral stage and the
    pressure projection, each on a bounded sample."""
    import numpy as np

    import oracle
    from workloads import Grid, configs
    g = wl.grid
    out = {}
    out["sgs"] = _oracle_rate(
        lambda: oracle.smagorinsky(g, wl.phi_uv, wl.phi_w, wl.u, wl.v, wl.w, z0=wl.z0,
                                   kappa=wl.kappa),
        g.n, f"the {g.nx}x{g.ny}x{g.nz} hill (FP64 C, OpenMP)")
    ws = configs.hill(256, 128, 128, H=16.0, L=40.0, x0=64.0, y0=64.0)
    out["spectral"] = _oracle_rate(lambda: oracle.stage_spectral(ws), ws.grid.n,
                                   "a 256x128x128 hill (wall stress, FFT divergence, forcing, "
                                   "drag; FP64)")
    gp = Grid(128, 64, 64)
    vel = list(np.random.default_rng(1).standard_normal((3,) + gp.shape))
    vel[2][0] = 0.0
    out["projection"] = _oracle_rate(lambda: oracle.pressure_project(gp, vel, wl.dt), gp.n,
                                     "a 128x64x64 grid (FP64 FFTs, a dense solve per mode: "
                                     "its cost grows as nz^3)")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the float64 comparison run")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-case ensemble")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-terrains", action="store_true", help="skip the cube and ridge runs")
    ap.add_argument("--no-sgs", action="store_true", help="skip the Smagorinsky stress runs")
    ap.add_argument("--no-chester", action="store_true",
                    help="skip Chester et al.'s original method")
    ap.add_argument("--no-spectral", action="store_true", help="skip the pseudo-spectral mode")
    ap.add_argument("--no-projection", action="store_true",
                    help="skip the AB2 update and the pressure projection")
    ap.add_argument("--retune", action="store_true",
                    help="time the tile shapes again and rewrite the autotuner's cache")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 384 MiB device-to-device copy three times, the "
                         "reference that scales FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--tile", type=str, default=None, help="vx,ty,kz,wpb for ibm_apply")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the stage has no multi-GPU path, so the figure "
              "is one GPU's throughput; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from workloads import configs

    if args.retune and os.path.exists(TUNE_CACHE):
        os.remove(TUNE_CACHE)
    t0 = time.time()
    wl64 = configs.hill()
    wl = wl64.cast(np.float32)
    log(f"workload generated in {time.time() - t0:.1f} s")
    tile = tuple(int(x) for x in args.tile.split(",")) if args.tile else None

    r32 = run_gpu(wl, "f32", "mixed", args.steps, args.warmup, tile)
    log(f"f32 mixed: {r32['ms_per_step']:.4f} ms/step through ibm_stage, "
        f"{r32['two_calls_ms']:.4f} as two calls (wall_stress {r32['wall_stress_ms']:.4f}, "
        f"apply {r32['apply_ms']:.4f}) tile {r32['tile']}")
    g = wl.grid
    value = g.n / (r32["ms_per_step"] * 1e-3)
    b_apply = apply_bytes(wl, r32["mask"], 4)
    achieved = b_apply / (r32["apply_ms"] * 1e-3) / 1e9
    triad = stream_triad()
    log(f"stream triad (torch, 3 x 134 MB float32): {triad:.0f} GB/s; k_apply at "
        f"{achieved / triad * 100:.1f} % of it")
    b_stage = stage_bytes(wl, r32["mask"], 4, r32["gathered"])
    stage_gbs = b_stage / (r32["ms_per_step"] * 1e-3) / 1e9
    out = {
        "metric": "IBM stage grid-points/s + % HBM roofline; batched FP32 vs plain FP64, same GPU",
        "value": value,
        "unit": "grid-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cos2 hill 512x256x256 (H=32, L=80 cells, z0=2e-4 H, band 1.5, "
                               "phi_c 1.5), mixed precision, one wall_stress + apply pass per step",
                   "nx": g.nx, "ny": g.ny, "nz": g.nz, "points": g.n, "precision": "mixed",
                   "tile": list(r32["tile"]), "band_records": r32["counts"][1] + r32["counts"][4]},
        "roofline": {"bound": "hbm", "kernel": "ibm_apply (k_apply)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(r32["tile"]),
                     "bytes_per_launch": b_apply, "launch_ms": r32["apply_ms"],
                     "stream_triad_GBs": triad, "frac_of_triad": achieved / triad},
        "kernels_ms": {"wall_stress": r32["wall_stress_ms"], "apply": r32["apply_ms"]},
        "stage": {"entry": "ibm_stage (wall stress, dense pass, one launch summing both "
                           "sets of slots)",
                  "bytes_per_pass": b_stage, "achieved_GBs": stage_gbs,
                  "frac": stage_gbs / HBM_PEAK_GBS,
                  "two_calls_ms_per_step": r32["two_calls_ms"],
                  "gathered_nodes": list(r32["gathered"])},
        "prepare_s": r32["prepare_s"],
    }
    if not args.no_f64:
        r64 = run_gpu(wl64, "f64", "plain", max(10, args.steps // 2), args.warmup,
                      min_warm_ms=WARM_MS)
        b64 = apply_bytes(wl64, r64["mask"], 8)
        out["fp64_plain"] = {"value": g.n / (r64["ms_per_step"] * 1e-3),
                             "ms_per_step": r64["ms_per_step"],
                             "apply_ms": r64["apply_ms"], "wall_stress_ms": r64["wall_stress_ms"],
                             "apply_GBs": b64 / (r64["apply_ms"] * 1e-3) / 1e9,
                             "f32_mixed_over_f64": r64["ms_per_step"] / r32["ms_per_step"]}
        log(f"f64 plain: {r64['ms_per_step']:.4f} ms/step")
    if not args.no_batch:
        out["batched"] = run_ensemble(args.steps, args.warmup)
        log(f"ensemble: {out['batched']['ratio']:.1f}x (f32 batched graph over f64 plain)")
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint(max(5, args.steps // 4), args.warmup)
        out["adjoint"]["above_mall"] = run_adjoint(max(5, args.steps // 4), args.warmup,
                                                   (512, 256, 256))
        log(f"adjoint: {out['adjoint']}")
    if not args.no_chester:
        out["chester"] = run_chester(wl, args.steps, args.warmup)
        log(f"chester: {out['chester']['chester_ms']:.4f} ms per step with "
            f"{out['chester']['sweeps']} sweeps ({out['chester']['ms_per_sweep'] * 1e3:.1f} us "
            f"per sweep) vs simplified {out['chester']['simplified_ms']:.4f} ms: "
            f"{out['chester']['chester_over_simplified']:.2f}x")
    if not args.no_sgs:
        out["sgs"] = run_sgs(wl, args.steps, args.warmup)
        log(f"sgs: {out['sgs']['sgs_ms']:.4f} ms ({out['sgs']['sgs_roofline']['frac'] * 100:.1f} % "
            f"of HBM peak); sgs + stage {out['sgs']['sgs_wall_stress_apply_ms']:.4f} ms; "
            f"wall stress + fused {out['sgs']['wall_stress_apply_sgs_ms']:.4f} ms (fused pass "
            f"{out['sgs']['apply_sgs_ms']:.4f} ms, "
            f"{out['sgs']['apply_sgs_roofline']['frac'] * 100:.1f} % of HBM peak)")
    if not args.no_spectral:
        out["spectral"] = run_spectral(wl, args.steps, args.warmup)
        log(f"spectral: {out['spectral']['ms']:.4f} ms per ibm_apply_spectral "
            f"({out['spectral']['frac'] * 100:.1f} % of HBM peak on algorithmic bytes, passes at "
            f"{out['spectral']['pass_GBs']:.0f} GB/s)")
    if not args.no_projection:
        out["projection"] = run_projection(wl, args.steps, args.warmup)
        log(f"projection: {out['projection']['project_ms']:.4f} ms per ibm_pressure_project, "
            f"ab2 {out['projection']['ab2_ms']:.4f} ms")
    if not args.no_terrains:
        out["terrains"] = run_terrains(args.steps, args.warmup)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl)
        log(f"cpu: {out['cpu_baseline']}")
        rows = cpu_oracle_rows(wl)
        for leg in ("sgs", "spectral", "projection"):
            if leg in out:
                out[leg]["cpu_oracle"] = rows[leg]
        log(f"cpu oracle beside the legs: {rows}")
    if args.calib_copy:
        src = torch.ones(3 << 25, dtype=torch.float32, device="cuda")    # 402,653,184 bytes
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 4
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
