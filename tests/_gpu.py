"""Helpers shared by the GPU tests: run the library on a workload, compare with the oracle."""
import numpy as np

TOL = {"f64": 1e-12, "f32": 2e-5}


def torch_dev():
    import torch
    return torch, torch.device("cuda", 0)


def normwise(got, exp):
    """max |got - exp| / max |exp| (0 if exp is identically 0 and got matches)."""
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    den = float(np.abs(exp).max()) if exp.size else 0.0
    num = float(np.abs(got - exp).max()) if exp.size else 0.0
    if den == 0.0:
        return num
    return num / den


def run_gpu(wl, dtype="f64", precision="plain", tile=None, stats=True, drag=True,
            in_place=False, spectral=False, offset=0):
    """One stage pass of the library (ibm_wall_stress then ibm_apply;
    ``in_place``: ustar is u, v, w themselves; ``offset`` > 0: the stacked
    stresses, velocities, ustar and divergence start that many elements into
    their buffers); returns numpy outputs and the context."""
    import paper_2006_03343_amd as ibm
    torch, dev = torch_dev()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g = wl.grid
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, tdt)
    ctx = ibm.Context(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, dtype=tdt, precision=precision,
                      device=dev)
    if tile is not None:
        ctx.set_tile(*tile)
    ctx.prepare(T(wl.phi_uv), T(wl.phi_w), wl.band_width, wl.phi_c, wl.kappa)
    def stacked(arrs):
        buf = torch.empty(len(arrs) * g.n + offset, dtype=tdt, device=dev)
        view = buf[offset:].view(len(arrs), g.nz, g.ny, g.nx)
        for i, a in enumerate(arrs):
            view[i].copy_(a)
        return view

    tau = stacked([T(t) for t in wl.tau])
    st = torch.zeros(4, dtype=torch.float64, device=dev) if stats else None
    lz = T(wl.log_z0) if wl.log_z0 is not None else None
    vel = stacked([T(wl.u), T(wl.v), T(wl.w)])
    u, v, w = vel
    ustar = vel if in_place else stacked(list(vel))
    div = stacked([torch.zeros_like(u)] * 3)
    dr = torch.zeros(3, dtype=torch.float64, device=dev) if drag else None
    gp = [T(t) for t in wl.gradp] if wl.gradp is not None else None
    z0 = None if lz is not None else wl.z0
    ctx.wall_stress(u, v, w, list(tau), z0=z0, log_z0=lz, stats=st)
    (ctx.apply_spectral if spectral else ctx.apply)(list(tau), list(ustar), list(div), gradp=gp,
                                                    dt=wl.dt, drag=dr)
    torch.cuda.synchronize()
    out = dict(tau=tau.cpu().numpy(), div=div.cpu().numpy(), ustar=ustar.cpu().numpy(),
               stats=st.cpu().numpy() if stats else None, drag=dr.cpu().numpy() if drag else None,
               mask=ctx.mask(), counts=ctx.counts())
    return out, ctx


def compare(out, ref, wl, tol, check_masks=True):
    """Assert the parity bar; returns a dict of per-output normwise errors."""
    errs = {}
    if check_masks:
        assert (out["mask"] == ref["mask"]).all(), "mask bytes differ"
        assert list(out["counts"]) == list(ref["counts"]), (out["counts"], ref["counts"])
    band_uv = (ref["mask"] & 3) == 1
    band_w = ((ref["mask"] >> 2) & 3) == 1
    names = ["xx", "yy", "zz", "xy", "xz", "yz"]
    for c in range(6):
        sel = band_uv if c < 4 else band_w
        errs["tau_" + names[c]] = normwise(out["tau"][c][sel], ref["tau"][c][sel])
        # everything outside the band is copied or zeroed: exact
        assert (out["tau"][c][~sel] == ref["tau"][c][~sel]).all(), f"tau_{names[c]} off the band"
    for c, nm in enumerate("xyz"):
        errs["div_" + nm] = normwise(out["div"][c], ref["div"][c])
        errs["ustar_" + nm] = normwise(out["ustar"][c], ref["ustar"][c])
    if out["drag"] is not None:
        scale = wl.grid.dv * np.array([np.abs(d).sum() for d in ref["div"]])
        errs["drag"] = float(np.max(np.abs(out["drag"] - ref["drag"]) / np.maximum(scale, 1e-300)))
    if out["stats"] is not None:
        s = ref["stats"]
        nb = band_uv.sum() + band_w.sum()
        errs["stats_sum"] = float(max(abs(out["stats"][0] - s[0]), abs(out["stats"][1] - s[1]))
                                  / max(np.abs(s[:2]).max(), 1e-300))
        errs["stats_max"] = abs(out["stats"][2] - s[2]) / max(s[2], 1e-300)
        assert out["stats"][3] == s[3] == nb
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"above {tol}: {bad}"
    return errs


def tiled(a, dtype, ry, rx):
    """A cell's field (nz, cy, cx) repeated ry times along y and rx times along x
    on the GPU: the field of a grid that is ry x rx periodic copies of the cell."""
    import torch
    _, dev = torch_dev()
    small = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev, dtype)
    return small.repeat(1, ry, rx)


def first_copy(f, cell_shape, ry, rx):
    """Assert that every copy of the cell in the periodic field f equals the
    first bit for bit; return the first as a numpy array."""
    nz, cy, cx = cell_shape
    cv = f.view(nz, ry, cy, rx, cx)
    assert bool((cv == cv[:, :1, :, :1, :]).all()), "periodic copies differ"
    return cv[:, 0, :, 0, :].cpu().numpy()
