"""Closed-form solutions and invariants used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* omega(theta, phi, Theta, Phi): the Cartesian components of the direction,
  Eqs. (omegax)-(omegaz), Sect. 4.1.
* Free streaming: particles travel in straight lines between collisions
  (Sect. 2.1), so with c = 1 and no collisions F(t, x, omega) = F0(x - t omega, omega);
  in the shell with zero inflow, zero where that segment crosses a boundary.
* Homogeneous emitting/absorbing sphere of radius R_s with uniform kappa and
  eta = kappa B: along each ray the stationary transport equation
  dI/ds = kappa (B - I) with I = 0 where the ray enters the sphere gives
  I = B (1 - exp(-kappa s)), s = r mu + sqrt(R_s^2 - r^2 (1 - mu^2)), mu = cos Theta.
* Isotropisation in a uniform scattering medium (the experiment of Sect. 5.2,
  with smooth data): a spatially uniform F(omega) has L F = 0, and the scattering
  term multiplies its spherical-harmonic part of degree l by -sigma (1 - lambda_l),
  lambda_l = (1/2) int p(mu) P_l(mu) dmu (Funk-Hecke); classical RK4 multiplies
  that part by R(-sigma (1 - lambda_l) dt) per step, R(z) = 1 + z + z^2/2 + z^3/6
  + z^4/24.
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


def free_streaming_shell(g, fn, t):
    """Free streaming in the shell r_in <= |x| <= r_out with zero inflow: the
    particle at (x, omega) at time t came from x - t omega if the straight segment
    x - s omega, 0 <= s <= t, stays inside the shell (Sect. 2.1), else it entered
    through a boundary, where the inflow is zero (Sect. 4.2).  |x - s omega|^2 is
    convex in s, so the segment leaves through r_out only if its start does, and
    through r_in if its smallest radius, at s = clip(x . omega, 0, t), is below
    r_in."""
    def f(x, y, z, ox, oy, oz):
        sx, sy, sz = x - t * ox, y - t * oy, z - t * oz
        s_min = np.clip(x * ox + y * oy + z * oz, 0.0, t)
        r_min2 = (x - s_min * ox) ** 2 + (y - s_min * oy) ** 2 + (z - s_min * oz) ** 2
        inside = (sx * sx + sy * sy + sz * sz <= g.r_out ** 2) & (r_min2 >= g.r_in ** 2)
        return np.where(inside, fn(sx, sy, sz, ox, oy, oz), 0.0)

    return on_grid(g, f)


def homogeneous_sphere(g, kappa, B, R_s):
    """Stationary I = B (1 - exp(-kappa s)) on the nodes of g for a uniform sphere
    of radius R_s >= r_out; kappa and B are arrays over eps."""
    r, th, ph, Th, Ph = g.mesh()
    mu = np.cos(Th)
    s = r * mu + np.sqrt(R_s ** 2 - r ** 2 * (1.0 - mu ** 2))
    k = np.asarray(kappa, np.float64).reshape(-1, 1, 1, 1, 1, 1)
    b = np.asarray(B, np.float64).reshape(-1, 1, 1, 1, 1, 1)
    return np.broadcast_to(b * (1.0 - np.exp(-k * s)), g.shape).copy()


def rk4_amplification(z):
    """Growth factor of one classical RK4 step on y' = lambda y, z = lambda dt."""
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def funk_hecke(kernel):
    """Eigenvalues (lambda_0, lambda_1, lambda_2) of the in-scattering operator for
    p(mu) = c0 + c1 mu + c2 mu^2, c0 = 1 - c2/3 (kernel = (c1, c2))."""
    c1, c2 = kernel
    c0 = 1.0 - c2 / 3.0
    return c0 + c2 / 3.0, c1 / 3.0, 2.0 * c2 / 15.0


def isotropisation(g, a, b, Q, sigma, kernel, dt, n):
    """F after n RK4 steps from the uniform F0 = a + b . omega + omega . Q . omega
    (Q symmetric) with kappa = eta = 0, uniform sigma and no inflow mask."""
    lam = funk_hecke(kernel)
    R = [rk4_amplification(-sigma * (1.0 - l) * dt) ** n for l in lam]
    Q = np.asarray(Q, np.float64)
    tr = np.trace(Q) / 3.0
    Q2 = Q - tr * np.eye(3)

    def fn(x, y, z, ox, oy, oz):
        o = (ox, oy, oz)
        quad = sum(Q2[i, j] * o[i] * o[j] for i in range(3) for j in range(3))
        return (a + tr) * R[0] + (b[0] * ox + b[1] * oy + b[2] * oz) * R[1] + quad * R[2]

    return on_grid(g, fn)


def isotropisation_ab2(g, a, b, Q, sigma, kernel, dt, n):
    """The uniform-medium problem of isotropisation() advanced by the
    Adams-Bashforth scheme with a forward-Euler first step: each degree-l part
    follows the scalar recurrence u_1 = (1 + z) u_0, u_{n+1} = u_n + z (3/2 u_n -
    1/2 u_{n-1}), z = -sigma (1 - lambda_l) dt."""
    lam = funk_hecke(kernel)
    R = []
    for l in lam:
        z = -sigma * (1.0 - l) * dt
        u_prev, u = 1.0, 1.0
        for step in range(n):
            if step == 0:
                u_prev, u = u, (1.0 + z) * u
            else:
                u_prev, u = u, u + z * (1.5 * u - 0.5 * u_prev)
        R.append(u)
    Q = np.asarray(Q, np.float64)
    tr = np.trace(Q) / 3.0
    Q2 = Q - tr * np.eye(3)

    def fn(x, y, z, ox, oy, oz):
        o = (ox, oy, oz)
        quad = sum(Q2[i, j] * o[i] * o[j] for i in range(3) for j in range(3))
        return (a + tr) * R[0] + (b[0] * ox + b[1] * oy + b[2] * oz) * R[1] + quad * R[2]

    return on_grid(g, fn)
