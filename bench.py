"""Benchmark of the wall-modeled IBM stage on one MI355X.

One step = one stage pass over the whole grid: ibm_wall_stress (band wall
model + solid zeroing + band statistics) followed by ibm_apply (stress
divergence + in-body forcing + drag), on the axisymmetric cos^2 hill
512 x 256 x 256 (H = 32, L = 80 cells, z0 = 2e-4 H), float32 storage in the
mixed-precision mode.  Inputs are generated (seeded, synthetic), copied to
HBM and the geometry prepared before the timed region.

Printed: one JSON line.  ``value`` is grid points per second of the stage
(nx*ny*nz*steps / time).  ``roofline`` is the dense kernel (ibm_apply):
algorithmic bytes per launch divided by its mean duration, measured with HIP
events recorded on the kernel's stream around every launch of the timed
region.  ``fp64_plain`` repeats the measurement with float64 storage.
``cpu_baseline`` times the FP64 CPU oracle (a test checker, never tuned) on
full passes of the same hill.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s


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


def run_gpu(wl, dtype, precision, steps, warmup, tile=None):
    import numpy as np
    import torch

    import paper_2006_03343_amd as ibm
    dev = torch.device("cuda", 0)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, tdt)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=tdt, precision=precision,
                      device=dev)
    if tile:
        ctx.set_tile(*tile)
    t0 = time.time()
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    torch.cuda.synchronize()
    t_prep = time.time() - t0
    u, v, w = T(wl.u), T(wl.v), T(wl.w)
    tau = torch.stack([T(t) for t in wl.tau]).contiguous()
    gp = [T(t) for t in wl.gradp]
    ustar = torch.stack([u, v, w]).contiguous()
    div = torch.empty_like(ustar)
    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    drag = torch.zeros(3, dtype=torch.float64, device=dev)
    taus, uss, divs = list(tau), list(ustar), list(div)

    def step():
        ctx.wall_stress(u, v, w, taus, z0=wl.z0, stats=stats)
        ctx.apply(taus, uss, divs, gradp=gp, dt=wl.dt, drag=drag)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for e in ev:
        e[0].record()
        ctx.wall_stress(u, v, w, taus, z0=wl.z0, stats=stats)
        e[1].record()
        ctx.apply(taus, uss, divs, gradp=gp, dt=wl.dt, drag=drag)
        e[2].record()
    end.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(end)
    ws_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    ap_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    mask = ctx.mask()
    res = dict(ms_per_step=total_ms / steps, wall_s=t_wall, wall_stress_ms=ws_ms, apply_ms=ap_ms,
               prepare_s=t_prep, tile=ctx.get_tile(), counts=[int(x) for x in ctx.counts()],
               mask=mask, drag=drag.cpu().tolist(), stats=stats.cpu().tolist())
    del ctx, u, v, w, tau, gp, ustar, div
    torch.cuda.empty_cache()
    return res


def cpu_baseline(wl, budget_s=12.0, max_passes=4):
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
    return dict(value=g.n * passes / t_total, unit="grid-points/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"{passes} full FP64 pass(es) of the {g.nx}x{g.ny}x{g.nz} hill "
                       f"(wall stress, divergence, forcing, drag), {t_total:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the float64 comparison run")
    ap.add_argument("--tile", type=str, default=None, help="vx,ty,kz,wpb for ibm_apply")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the stage has no multi-GPU path in this build "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from workloads import configs

    t0 = time.time()
    wl64 = configs.hill()
    wl = wl64.cast(np.float32)
    log(f"workload generated in {time.time() - t0:.1f} s")
    tile = tuple(int(x) for x in args.tile.split(",")) if args.tile else None

    r32 = run_gpu(wl, "f32", "mixed", args.steps, args.warmup, tile)
    log(f"f32 mixed: {r32['ms_per_step']:.4f} ms/step (wall_stress {r32['wall_stress_ms']:.4f}, "
        f"apply {r32['apply_ms']:.4f}) tile {r32['tile']}")
    g = wl.grid
    value = g.n / (r32["ms_per_step"] * 1e-3)
    b_apply = apply_bytes(wl, r32["mask"], 4)
    achieved = b_apply / (r32["apply_ms"] * 1e-3) / 1e9
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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": b_apply, "launch_ms": r32["apply_ms"]},
        "kernels_ms": {"wall_stress": r32["wall_stress_ms"], "apply": r32["apply_ms"]},
        "prepare_s": r32["prepare_s"],
    }
    if not args.no_f64:
        r64 = run_gpu(wl64, "f64", "plain", max(10, args.steps // 2), args.warmup)
        b64 = apply_bytes(wl64, r64["mask"], 8)
        out["fp64_plain"] = {"value": g.n / (r64["ms_per_step"] * 1e-3),
                             "ms_per_step": r64["ms_per_step"],
                             "apply_ms": r64["apply_ms"], "wall_stress_ms": r64["wall_stress_ms"],
                             "apply_GBs": b64 / (r64["apply_ms"] * 1e-3) / 1e9,
                             "f32_mixed_over_f64": r64["ms_per_step"] / r32["ms_per_step"]}
        log(f"f64 plain: {r64['ms_per_step']:.4f} ms/step")
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl)
        log(f"cpu: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
