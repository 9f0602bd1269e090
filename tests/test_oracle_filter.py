"""Pins of the radial filter of the oracle (the exponential filter exp(-36 eta^36)
applied to the Chebyshev expansion in r; used for the shell experiment of
Sect. 5.3, whose radial discontinuity the paper treats by finite differences).

* a Chebyshev polynomial T_k(x(r)) (written as cos(k arccos x)) is scaled by
  exp(-36 (k / (n_r - 1))^36), constants are kept;
* the transposed filter used by the adjoint passes the dot-product test, alone
  and through a whole RK4 step with the filter on.
"""

import numpy as np
import pytest

from oracle import grid as og, ops, step, adjoint


@pytest.mark.parametrize("n_r", [5, 9, 17, 33])
def test_chebyshev_modes_scaled(n_r):
    g = og.make_grid(1, n_r, 2, 4, 2, 4)
    x = (2.0 * g.r - g.r_in - g.r_out) / (g.r_out - g.r_in)
    for k in range(n_r):
        Tk = np.cos(k * np.arccos(np.clip(x, -1.0, 1.0)))
        F = np.broadcast_to(Tk[None, :, None, None, None, None], g.shape).copy()
        want = np.exp(-36.0 * (k / (n_r - 1.0)) ** 36) * F
        got = ops.apply_filter(F, g, radial=True)
        np.testing.assert_allclose(got, want, atol=1e-13 * n_r)


def test_transpose_and_step_adjoint():
    g = og.make_grid(2, 9, 4, 8, 4, 8)
    rng = np.random.default_rng(0)
    x = rng.normal(size=g.shape)
    y = rng.normal(size=g.shape)
    assert np.sum(ops.apply_filter(x, g, radial=True) * y) == pytest.approx(
        np.sum(x * ops.apply_filter_T(y, g, radial=True)), rel=1e-13)
    kappa, sigma, eta = (rng.uniform(0.2, 1.5, size=g.shape[:4]) for _ in range(3))
    p = step.Physics(kappa, sigma, 0 * eta, bc=True, scattering=True, filt=True, filt_r=True)
    dt = g.dt_default()
    y0 = rng.normal(size=g.shape)
    lin = step.rk4_step(y0 + x, g, p, dt) - step.rk4_step(y0, g, p, dt)
    lam = rng.normal(size=g.shape)
    lam_prev = adjoint.adjoint_step(y0, lam, g, p, dt)[0]
    assert np.sum(lin * lam) == pytest.approx(np.sum(x * lam_prev), rel=1e-11)
