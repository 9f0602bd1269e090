"""Oracle time stepping: classical RK4 on dF/dt = -L_sph F + C(F), and the
paper's own second-order Adams-Bashforth scheme (Sect. 5.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper advances its spectral coefficients with second-order Adams-Bashforth
(Sect. 5.1); this hot path uses classical fourth-order Runge-Kutta instead.
Inflow data are constant in time, so the stages carry no explicit time.
The optional filter (ops.apply_filter, angular lines and optionally r) is applied
after each full step; with the inflow conditions on, the inflow nodes are then
set back to their prescribed values (Sect. 4.2: F is imposed there; a filter
that moved them would break the boundary condition, and it makes long filtered
runs with inflow unstable).
"""

from dataclasses import dataclass

import numpy as np

from . import energy, ops


@dataclass
class Physics:
    """Coefficient fields [eps][r][theta][phi] and switches."""

    kappa: np.ndarray
    sigma: np.ndarray
    eta: np.ndarray
    bc: bool = True
    scattering: bool = True
    filt: bool = False
    # with filt: also filter the radial (Chebyshev) lines
    filt_r: bool = False
    # split step: RK4 on everything but the radial term, then a backward-Euler
    # radial substep (the implicit scheme of App. B)
    radial_implicit: bool = False
    # phase function p(mu) = (1 - c2/3) + c1 mu + c2 mu^2 as (c1, c2); None = isotropic
    kernel: tuple = None
    # inflow planes [eps][theta][phi][Theta][Phi] at r_in and r_out (None = zero),
    # re-imposed after the filter
    g_in: np.ndarray = None
    g_out: np.ndarray = None
    # Fokker-Planck energy coupling (energy.fp_source) as (gamma_min, gamma_max,
    # alpha), the groups being the Chebyshev nodes of gamma; None = off
    energy: tuple = None

    @staticmethod
    def vacuum(g, bc=True):
        z = np.zeros((g.n_eps, g.n_r, g.n_theta, g.n_phi))
        return Physics(z, z.copy(), z.copy(), bc=bc, scattering=False)


def filter_step(y, g, p):
    """The filter after a step (ops.apply_filter), then, with the inflow
    conditions on, the prescribed values at the inflow nodes."""
    y = ops.apply_filter(y, g, radial=p.filt_r)
    if p.bc:
        y = ops.project_inflow(y, g, p.g_in, p.g_out)
    return y


def rhs(F, g, p):
    out = ops.rhs(F, g, p.kappa, p.sigma, p.eta, bc=p.bc, scattering=p.scattering, kernel=p.kernel,
                  radial=not p.radial_implicit)
    if p.energy is not None:
        # the coupling's isotropic source sigma S(F), zero at the inflow nodes
        s = p.sigma if p.scattering else np.zeros_like(np.asarray(p.sigma, np.float64))
        src = energy.fp_source(F, g, s, *p.energy)[..., None, None]
        out = out + (src * ops.inflow_mask(g) if p.bc else src)
    return out


def rk4_stages(y, g, p, dt):
    """The four stage inputs Y_s and slopes k_s of one classical RK4 step."""
    Y1 = y
    k1 = rhs(Y1, g, p)
    Y2 = y + 0.5 * dt * k1
    k2 = rhs(Y2, g, p)
    Y3 = y + 0.5 * dt * k2
    k3 = rhs(Y3, g, p)
    Y4 = y + dt * k3
    k4 = rhs(Y4, g, p)
    return (Y1, Y2, Y3, Y4), (k1, k2, k3, k4)


def rk4_step(y, g, p, dt):
    """y_{n+1} = y + dt/6 (k1 + 2 k2 + 2 k3 + k4), then (radial_implicit) the
    backward-Euler radial substep, then the filter if enabled."""
    _, (k1, k2, k3, k4) = rk4_stages(y, g, p, dt)
    y1 = y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    if p.radial_implicit:
        y1 = ops.apply_radial_implicit(y1, g, dt, bc=p.bc)
    if p.filt:
        y1 = filter_step(y1, g, p)
    return y1


def run(y, g, p, dt, n_steps, callback=None):
    """n_steps RK4 steps from y; callback(n, y) after each step if given."""
    for n in range(n_steps):
        y = rk4_step(y, g, p, dt)
        if callback is not None:
            callback(n + 1, y)
    return y


def ab2_run(y, g, p, dt, n_steps, k_prev=None):
    """n_steps of second-order Adams-Bashforth (the scheme of Sect. 5.1):
    y_{n+1} = y_n + dt (3/2 k_n - 1/2 k_{n-1}), k_n = rhs(y_n).  Without a
    previous slope (k_prev None) the first step takes k_{-1} = k_0, i.e. forward
    Euler (the paper does not state its start).  The filter, if enabled, acts
    on the state and on the stored slope after every step (with the inflow
    conditions on, the state then takes its inflow values again and the slope is
    zero at the inflow nodes, as the right-hand side is).  Returns (y, k) with k
    the stored slope, to continue a run."""
    for _ in range(n_steps):
        k = rhs(y, g, p)
        kp = k if k_prev is None else k_prev
        y = y + dt * (1.5 * k - 0.5 * kp)
        if p.filt:
            y = filter_step(y, g, p)
            k = ops.apply_filter(k, g, radial=p.filt_r)
            if p.bc:
                k = k * ops.inflow_mask(g)
        k_prev = k
    return y, k_prev
