"""Oracle: the Liouville operator in the conservative (flux) form of App. A.

TEST INFRASTRUCTURE ONLY (see the package docstring).

App. A (Eq. Cohercons) multiplies the transport equation by the phase-space
volume element V = r^2 sin(theta) sin(Theta); every streaming term then becomes
the derivative of a flux:

    V L F = d_r(cos Theta F^) + d_theta(c_th F^) + d_phi(c_ph F^)
            - (1/r) d_Theta(sin Theta F^) - (sin Theta cos theta / (r sin theta)) d_Phi(sin Phi F^),

F^ = V F (App. B, Eq. flux), with c_th = sin Theta cos Phi / r and c_ph =
sin Theta sin Phi / (r sin theta) the coefficients of Eq. (Liouvsph), which do
not vary along their own lines.  Integrated over the phase space, every term but
the radial one is the integral of a derivative over a full period, so
dN/dt = -(J_R2 - J_R1) (Eq. Cons).

Two discrete forms are built here, both with the collocation matrices of the
hot path:

* apply_L_flux: the form above, differentiating each flux along its line.  F^
  changes sign across the position pole (sin(-theta) = -sin(theta)), so the
  theta DFS line of F^ takes the partner half with the opposite sign (the
  coefficient c_th stays outside the derivative); the Theta flux
  sin(Theta) F^ = r^2 sin(theta) sin^2(Theta) F does not change sign across
  Theta = 0, pi, so its DFS line is the ordinary one.
* apply_L_hybrid: F itself with the radial and Phi terms in flux form,
  (cos Theta / r^2) D_r(r^2 F) and -(sin Theta cos theta / (r sin theta)) D_Phi(sin Phi F),
  and the two terms they add to the operator removed again explicitly:
  -2 cos Theta F / r (which the Theta term's flux form would cancel) and
  + sin Theta cos theta cos Phi F / (r sin theta) (which the theta term's would);
  the theta, phi and Theta terms as in ops.apply_L.

All three forms (with ops.apply_L) are the same continuous operator; they differ
in which parts of the discrete sum over the grid cancel exactly.
"""

import numpy as np

from . import ops


def volume(g):
    """V = r^2 sin(theta) sin(Theta), rank-6 broadcastable."""
    r, th, ph, Th, Ph = g.mesh()
    return r ** 2 * np.sin(th) * np.sin(Th) + 0.0 * (ph + Ph)


def _d_theta_odd(G, g):
    """DFS derivative along theta of a field that changes sign across the pole:
    the partner half of each line is the negated value at (phi + pi, Phi + pi)."""
    ext = ops.dfs_extend_theta(G, g)
    n = g.n_theta
    sign = np.concatenate([np.ones(n), -np.ones(n)]).reshape(1, 1, 2 * n, 1, 1, 1)
    D = ops.apply_along(g.D_theta, ext * sign, ops.AX_TH)
    return np.take(D, np.arange(n), axis=ops.AX_TH)


def apply_L_flux(F, g):
    """L F from the flux form of Eq. (Cohercons): (1/V) times the sum of the five
    flux derivatives of F^ = V F."""
    r, th, ph, Th, Ph = g.mesh()
    c_r, c_th, c_ph, _, _ = ops.liouville_coefficients(g)
    V = volume(g)
    Fh = V * F
    total = (c_r * ops.d_r(Fh, g)
             + c_th * _d_theta_odd(Fh, g)
             + c_ph * ops.d_phi(Fh, g)
             - (1.0 / r) * ops.d_Theta(np.sin(Th) * Fh, g)
             - (np.sin(Th) * np.cos(th) / (r * np.sin(th))) * ops.d_Phi(np.sin(Ph) * Fh, g))
    return total / V


def apply_L_hybrid(F, g):
    """L F with the radial and Phi terms in flux form and their added terms
    removed explicitly; theta, phi and Theta terms as in Eq. (Liouvsph)."""
    r, th, ph, Th, Ph = g.mesh()
    c_r, c_th, c_ph, c_Th, _ = ops.liouville_coefficients(g)
    radial = c_r * ops.d_r(r ** 2 * F, g) / r ** 2 - 2.0 * np.cos(Th) * F / r
    Phi = (-(np.sin(Th) * np.cos(th) / (r * np.sin(th))) * ops.d_Phi(np.sin(Ph) * F, g)
           + np.sin(Th) * np.cos(th) * np.cos(Ph) * F / (r * np.sin(th)))
    return radial + c_th * ops.d_theta(F, g) + c_ph * ops.d_phi(F, g) + c_Th * ops.d_Theta(F, g) + Phi


def conservation_residual(LF, F, g):
    """The discrete Eq. (Cons) for dF/dt = -L F at one instant: dN/dt + J_R2 - J_R1
    with N and J from the quadratures of the diagnostics, per energy group, and
    its scale |J_R2| + |J_R1|."""
    from . import diagnostics
    dN = diagnostics.particle_number(-LF, g)
    _, J_in, J_out = diagnostics.fluxes(F, g)
    return dN + J_out - J_in, np.abs(J_out) + np.abs(J_in)
