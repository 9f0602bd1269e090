"""Pins of the radially implicit split step of the oracle (the backward-Euler
Chebyshev advection of App. B for the radial term, RK4 for the rest).

* The backward-Euler collocation solve against exact polynomial algebra: with
  u the data (degree < n_r) and w(r) = prod over the non-inflow nodes of
  (r - r_j), the collocation solution is the polynomial q with
  q + dt c q' = u + alpha w, q = sum_k (-dt c)^k (u + alpha w)^(k) (a finite
  Neumann series), and alpha fixed by q(inflow) = u(inflow).
* A step from data depending on r only (L reduces to the radial term, the
  explicit part vanishes in vacuum) equals the solve alone.
* A uniform state is kept exactly.
"""

import numpy as np
from numpy.polynomial import Chebyshev
import pytest

from oracle import grid as og, ops, step


def _backward_euler_poly(r_nodes, u, dtc, inflow, domain):
    """Exact polynomial solution of the collocated backward-Euler equation (u a
    Chebyshev series on the shell, for conditioning)."""
    others = [x for j, x in enumerate(r_nodes) if j != inflow]
    w = Chebyshev.fromroots(others, domain=domain)

    def neumann(c):
        out, term, k = c * 0.0, c, 0
        while term.degree() >= 0 and k <= c.degree() + 1:
            out = out + (-dtc) ** k * term
            if term.degree() == 0:
                break
            term = term.deriv()
            k += 1
        return out

    qu, qw = neumann(u), neumann(w)
    r0 = r_nodes[inflow]
    alpha = (u(r0) - qu(r0)) / qw(r0)
    return lambda r: qu(r) + alpha * qw(r)


@pytest.mark.parametrize("n_r", [5, 9, 17])
def test_backward_euler_solve_polynomial_exact(n_r):
    g = og.make_grid(1, n_r, 2, 4, 4, 8)
    dt = 0.05
    B = ops.radial_implicit_matrices(g, dt)
    rng = np.random.default_rng(n_r)
    dom = [g.r_in, g.r_out]
    u = Chebyshev(rng.normal(size=n_r - 1), domain=dom)  # degree n_r - 2
    vals = u(g.r)
    for i, Th in enumerate(g.Theta):
        c = np.cos(Th)
        inflow = 0 if c > 0 else n_r - 1
        q = _backward_euler_poly(g.r, u, dt * c, inflow, dom)
        np.testing.assert_allclose(B[i] @ vals, q(g.r), rtol=0, atol=1e-12 * np.max(np.abs(vals)))


def test_radial_data_step_is_the_solve():
    g = og.make_grid(1, 9, 4, 8, 4, 8)
    rng = np.random.default_rng(0)
    f = rng.normal(size=g.n_r)
    F = np.broadcast_to(f[None, :, None, None, None, None], g.shape).copy()
    z = np.zeros(g.shape[:4])
    p = step.Physics(z, z, z, bc=True, scattering=False, radial_implicit=True)
    dt = 0.07
    got = step.rk4_step(F, g, p, dt)
    np.testing.assert_allclose(got, ops.apply_radial_implicit(F, g, dt), atol=1e-13)


def test_constant_state_is_kept():
    g = og.make_grid(2, 9, 4, 8, 4, 8)
    z = np.zeros(g.shape[:4])
    p = step.Physics(z, z, z, bc=True, scattering=False, radial_implicit=True)
    F = np.full(g.shape, 2.5)
    np.testing.assert_allclose(step.run(F, g, p, 0.1, 5), F, atol=1e-13)


@pytest.mark.parametrize("n_r", [9, 33])
def test_backward_euler_radial_step_has_no_step_limit(n_r):
    # App. B: the implicit radial solve sets no Courant limit.  With the inflow
    # value held, the rest of the line evolves by the non-inflow block of B_i,
    # whose eigenvalues 1 / (1 + dt lambda) lie inside the unit disc for every dt
    # (lambda: eigenvalues of cos(Theta_i) D_r with the inflow node removed, in
    # the right half plane); far beyond the explicit limit it damps hard.
    g = og.make_grid(1, n_r, 2, 4, 8, 16)
    for dt in (1e-3, 1e-1, 10.0, 1e3):
        B = ops.radial_implicit_matrices(g, dt)
        for i, b in enumerate(B):
            j = 0 if np.cos(g.Theta[i]) > 0 else n_r - 1
            keep = [k for k in range(n_r) if k != j]
            rho = np.max(np.abs(np.linalg.eigvals(b[np.ix_(keep, keep)])))
            assert rho < 1.0, (dt, i, rho)
            if dt >= 1e3:
                assert rho < 0.01
            # the inflow row is the identity
            e = np.zeros(n_r)
            e[j] = 1.0
            np.testing.assert_allclose(b[j], e, rtol=0, atol=1e-13)


def test_backward_euler_front_speed_app_b():
    # App. B's 1D experiment: a step profile entering the shell at r_in with
    # speed C (here C = cos Theta_0), 65 Chebyshev points, dt = 8 (R2 - R1) /
    # (C N_r^2) (the paper's Delta t_opt).  The paper reports the right
    # propagation speed: the half-height point sits at r_in + C t.
    n_r = 65
    g = og.make_grid(1, n_r, 2, 4, 8, 16)
    C = np.cos(g.Theta[0])
    dt = 8.0 * (g.r_out - g.r_in) / (C * n_r ** 2)
    B = ops.radial_implicit_matrices(g, dt)[0]
    u = np.zeros(n_r)
    u[0] = 1.0
    nsteps = int(round(1.0 / dt))
    for _ in range(nsteps):
        u = B @ u
    t = nsteps * dt
    x = np.linspace(g.r_in, g.r_out, 2001)
    prof = np.polynomial.chebyshev.Chebyshev.fit(g.r, u, n_r - 1, domain=[g.r_in, g.r_out])(x)
    front = x[np.argmax(prof < 0.5)]
    assert abs(front - (g.r_in + C * t)) < 0.05
    # the profile stays bounded (no growth) and is 1 behind the front
    assert np.max(np.abs(u)) < 1.3
    assert abs(u[0] - 1.0) < 1e-12  # the inflow value is held (up to the rounding of the inverse)
