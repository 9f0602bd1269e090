"""Closed-form solutions and invariants used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* omega(theta, phi, Theta, Phi): the Cartesian components of the direction,
  Eqs. (omegax)-(omegaz), Sect. 4.1.
* Free streaming: particles travel in straight lines between collisions
  (Sect. 2.1), so with c = 1 and no collisions F(t, x, omega) = F0(x - t omega, omega).
* Homogeneous emitting/absorbing sphere of radius R_s with uniform kappa and
  eta = kappa B: along each ray the stationary transport equation
  dI/ds = kappa (B - I) with I = 0 where the ray enters the sphere gives
  I = B (1 - exp(-kappa s)), s = r mu + sqrt(R_s^2 - r^2 (1 - mu^2)), mu = cos Theta.
* B(eps, T) = 2 eps^2 / (exp(eps/T) - 1): the steady state of Eq. (Bose) at zero
  chemical potential, in the same F = gamma^2 f normalisation (Sect. 3.2).
"""

import numpy as np


def omega(th, ph, Th, Ph):
    """(omega_x, omega_y, omega_z), Eqs. (omegax)-(omegaz)."""
    ox = (np.cos(Th) * np.sin(th) * np.cos(ph) + np.sin(Th) * np.cos(Ph) * np.cos(th) * np.cos(ph)
          - np.sin(Th) * np.sin(Ph) * np.sin(ph))
    oy = (np.cos(Th) * np.sin(th) * np.sin(ph) + np.sin(Th) * np.cos(Ph) * np.cos(th) * np.sin(ph)
          + np.sin(Th) * np.sin(Ph) * np.cos(ph))
    oz = np.cos(Th) * np.cos(th) - np.sin(Th) * np.cos(Ph) * np.sin(th)
    return ox, oy, oz


def position(r, th, ph):
    return r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)


def on_grid(g, fn):
    """Evaluate fn(x, y, z, ox, oy, oz) on every node of g (all energy groups equal)."""
    r, th, ph, Th, Ph = g.mesh()
    x, y, z = position(r, th, ph)
    ox, oy, oz = omega(th, ph, Th, Ph)
    return np.broadcast_to(fn(x, y, z, ox, oy, oz), g.shape).astype(np.float64).copy()


def free_streaming(g, fn, t):
    """F(t) = F0(x - t omega, omega) on the nodes of g."""
    return on_grid(g, lambda x, y, z, ox, oy, oz: fn(x - t * ox, y - t * oy, z - t * oz, ox, oy, oz))


def planck_like(eps, T):
    """B(eps, T) = 2 eps^2 / (exp(eps / T) - 1)."""
    return 2.0 * eps ** 2 / np.expm1(eps / T)


def homogeneous_sphere(g, kappa, B, R_s):
    """Stationary I = B (1 - exp(-kappa s)) on the nodes of g for a uniform sphere
    of radius R_s >= r_out; kappa and B are arrays over eps."""
    r, th, ph, Th, Ph = g.mesh()
    mu = np.cos(Th)
    s = r * mu + np.sqrt(R_s ** 2 - r ** 2 * (1.0 - mu ** 2))
    k = np.asarray(kappa, np.float64).reshape(-1, 1, 1, 1, 1, 1)
    b = np.asarray(B, np.float64).reshape(-1, 1, 1, 1, 1, 1)
    return np.broadcast_to(b * (1.0 - np.exp(-k * s)), g.shape).copy()
