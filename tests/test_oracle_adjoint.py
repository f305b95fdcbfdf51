"""Pin of the oracle's reverse mode against central finite differences of its forward.

The forward pieces are pinned on their own (closed forms, covariance,
telescoping); here the hand-written reverse mode of the whole stage is held
to FP64 central differences along random directions in (u, v, w, log z0).
"""
import dataclasses

import numpy as np
import pytest

from workloads import configs


def _perturbed(wl, eps, d):
    return dataclasses.replace(wl, u=wl.u + eps * d[0], v=wl.v + eps * d[1], w=wl.w + eps * d[2],
                               log_z0=wl.log_z0 + eps * d[3])


def _loss(ora, wl, G_tau, G_drag, w_ustar=1.0):
    r = ora.stage(wl)
    J = float(np.dot(r["drag"], G_drag))
    J += 0.5 * sum(float((a * a).sum()) for a in r["div"])
    J += 0.5 * w_ustar * sum(float((a * a).sum()) for a in r["ustar"])
    if G_tau is not None:
        J += sum(float((a * b).sum()) for a, b in zip(r["tau"], G_tau))
    return J, r


@pytest.mark.parametrize("with_gtau", [False, True])
def test_reverse_mode_matches_central_differences(ora, with_gtau):
    wl = configs.fractal(16, 12, 12, rms=2.0)
    g = wl.grid
    rng = np.random.default_rng(17 + with_gtau)
    G_tau = [rng.standard_normal(g.shape) for _ in range(6)] if with_gtau else None
    G_drag = np.array([1.0, 0.0, 0.0]) if not with_gtau else rng.standard_normal(3)
    J0, r = _loss(ora, wl, G_tau, G_drag)
    gu, gv, gw, glz = ora.stage_vjp(wl, G_tau, r["div"], r["ustar"], G_drag)
    assert np.abs(glz).max() > 0
    eps = 1e-6
    for _ in range(8):
        d = [rng.standard_normal(g.shape) for _ in range(4)]
        jp, _ = _loss(ora, _perturbed(wl, eps, d), G_tau, G_drag)
        jm, _ = _loss(ora, _perturbed(wl, -eps, d), G_tau, G_drag)
        fd = (jp - jm) / (2 * eps)
        an = float((gu * d[0]).sum() + (gv * d[1]).sum() + (gw * d[2]).sum() + (glz * d[3]).sum())
        assert abs(fd - an) <= 1e-6 * (abs(an) + 1.0), (fd, an)


def test_reverse_mode_log_z0_only(ora):
    """Perturbing log z0 alone moves only band stresses; the reverse mode must see it.
    The forced-velocity term is left out of the loss so that its large,
    log z0-independent value does not swamp the difference quotient."""
    wl = configs.fractal(16, 12, 12, rms=2.0, seed_offset=3)
    g = wl.grid
    rng = np.random.default_rng(99)
    J0, r = _loss(ora, wl, None, np.array([1.0, 0.0, 0.0]), 0.0)
    gu, gv, gw, glz = ora.stage_vjp(wl, None, r["div"], [0 * a for a in r["ustar"]],
                                    [1.0, 0.0, 0.0])
    eps = 1e-6
    zero = np.zeros(g.shape)
    for _ in range(4):
        d = [zero, zero, zero, rng.standard_normal(g.shape)]
        jp, _ = _loss(ora, _perturbed(wl, eps, d), None, np.array([1.0, 0.0, 0.0]), 0.0)
        jm, _ = _loss(ora, _perturbed(wl, -eps, d), None, np.array([1.0, 0.0, 0.0]), 0.0)
        fd = (jp - jm) / (2 * eps)
        an = float((glz * d[3]).sum())
        assert abs(fd - an) <= 1e-6 * (abs(an) + 1e-3), (fd, an)
