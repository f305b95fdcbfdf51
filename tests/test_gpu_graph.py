"""A whole time step captured in one HIP graph (torch.cuda.CUDAGraph): the AB2
update, the Smagorinsky stress, the wall stress, the dense pass (central and
pseudo-spectral), the fused SGS pass and the pressure projection.  After one
eager step (first calls size the reduction slots, build the twiddle tables and
the projection workspace) the entry points allocate nothing, synchronise
nothing and set no memory, so the step can be captured; each replay, with eager
work and a synchronisation between replays that clobber every output, equals
the eager step bit for bit (every kernel is deterministic)."""
import numpy as np
import pytest

from _gpu import torch_dev
from workloads import configs

pytestmark = pytest.mark.gpu


def test_time_step_graph():
    import torch
    import paper_2006_03343_amd as ibm
    _, dev = torch_dev()
    wl = configs.hill(128, 64, 32, H=12.0, L=30.0, x0=40.0, y0=32.0).cast(np.float32)
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=torch.float32,
                      precision="mixed", device=dev)
    pu, pw = T(wl.phi_uv), T(wl.phi_w)
    ctx.prepare(pu, pw, wl.band_width, wl.phi_c, wl.kappa)
    vel = [T(wl.u), T(wl.v), T(wl.w)]
    rng = np.random.default_rng(4)
    rn = [T(0.1 * rng.standard_normal(g.shape)) for _ in range(3)]
    rp = [T(0.1 * rng.standard_normal(g.shape)) for _ in range(3)]
    gp = [T(t) for t in wl.gradp]
    ustar = [torch.empty_like(vel[0]) for _ in range(3)]
    ustar2 = [torch.empty_like(vel[0]) for _ in range(3)]
    tau = [torch.empty_like(vel[0]) for _ in range(6)]
    div = [torch.empty_like(vel[0]) for _ in range(3)]
    div_s = [torch.empty_like(vel[0]) for _ in range(3)]
    div_f = [torch.empty_like(vel[0]) for _ in range(3)]
    uo = [torch.empty_like(vel[0]) for _ in range(3)]
    p = torch.empty_like(vel[0])
    drag, drag_s, drag_f = (torch.zeros(3, dtype=torch.float64, device=dev) for _ in range(3))
    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    dt = wl.dt

    def step():
        ctx.ab2_predict(vel, rn, rp, dt, ustar)
        for a, b in zip(ustar2, ustar):
            a.copy_(b)
        ctx.sgs_stress(pu, pw, *vel, tau, z0=wl.z0, kappa=wl.kappa)
        ctx.wall_stress(*vel, tau, z0=wl.z0, stats=stats)
        ctx.apply(tau, ustar, div, gradp=gp, dt=dt, drag=drag)
        ctx.apply_spectral(tau, ustar2, div_s, gradp=gp, dt=dt, drag=drag_s)
        ctx.apply_sgs(pu, pw, *vel, tau, ustar2, div_f, z0=wl.z0, kappa=wl.kappa, gradp=gp,
                      dt=dt, drag=drag_f)
        ctx.pressure_project(ustar, dt, uo, p)

    outputs = ustar + ustar2 + tau + div + div_s + div_f + uo + [p, drag, drag_s, drag_f, stats]
    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in outputs]
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        for t in outputs:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(outputs, ref)):
            assert torch.equal(a, b), f"replay {rep}: output {i} differs from the eager step"
        print(f"replay {rep}: every output equals the eager step", flush=True)
