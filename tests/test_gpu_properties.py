"""Property-based GPU parity (hypothesis, derandomized, a few examples): the
whole stage on random tilted planes, band widths 2 phi_b in [dz, 1.5 dz],
phi_c in [2 phi_b, 4 phi_b] and anisotropic spacings, float64 against the
oracle at the usual bar (masks identical, normwise <= 1e-12)."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

from _gpu import TOL, compare, run_gpu
from workloads import Grid, configs, terrain

pytestmark = pytest.mark.gpu


@settings(max_examples=8, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(polar=st.floats(0.0, 1.2), azim=st.floats(0.0, 2 * math.pi), off=st.floats(0.0, 1.0),
       beta=st.floats(1.0, 1.5), gamma=st.floats(1.0, 2.0), dx=st.floats(0.6, 1.6),
       dy=st.floats(0.6, 1.6), dz=st.floats(0.6, 1.6))
def test_random_tilted_planes(ora, polar, azim, off, beta, gamma, dx, dy, dz):
    g = Grid(40, 28, 18, dx, dy, dz)
    n_hat = (math.sin(polar) * math.cos(azim), math.sin(polar) * math.sin(azim), math.cos(polar))
    wl = configs.flat(g, 1.0, noise=0.3, tau_std=0.01, gp_std=0.1, seed=int(1000 * off))
    wl.phi_uv, wl.phi_w = terrain.plane(g, (20 * dx, 14 * dy, (5 + off) * dz), n_hat)
    wl.band_width = beta * dz
    wl.phi_c = gamma * wl.band_width
    wl.z0 = 1e-3 * dz
    print(f"plane n={np.round(n_hat, 3)} off={off:.3f} b={wl.band_width:.3f} "
          f"phi_c={wl.phi_c:.3f} spacing=({dx:.3f}, {dy:.3f}, {dz:.3f})", flush=True)
    out, _ = run_gpu(wl, "f64")
    compare(out, ora.stage(wl), wl, TOL["f64"])
