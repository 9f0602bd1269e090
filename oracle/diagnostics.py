"""Oracle diagnostics: particle number N, boundary fluxes J, outgoing-flux map.

TEST INFRASTRUCTURE ONLY (see the package docstring).

App. A defines the particle number (Eq. Npho) as the integral of F over
r^2 dr sin(theta) dtheta dphi sin(Theta) dTheta dPhi, and the flux through a
sphere of radius R (Eq. Flux) as R^2 times the integral of F cos(Theta) over the
same angles; Eq. (Cons) states dN/dt + J_R2 - J_R1 = 0.  The quadratures are
this build's choice (the paper gives none): Clenshaw-Curtis in r, Fejer's
first rule in cos(theta) and cos(Theta), the trapezoid rule in phi and Phi.
"""

import numpy as np


def _angle_weights(g):
    """Weights over (theta, phi, Theta, Phi), shape (n_theta, n_phi, n_Theta, n_Phi)."""
    wth = g.w_theta[:, None, None, None]
    wph = np.full((1, g.n_phi, 1, 1), 2.0 * np.pi / g.n_phi)
    wTh = g.w_Theta[None, None, :, None]
    wPh = np.full((1, 1, 1, g.n_Phi), 2.0 * np.pi / g.n_Phi)
    return wth * wph * wTh * wPh


def particle_number(F, g):
    """N per energy group, Eq. (Npho)."""
    w = _angle_weights(g)[None, None] * (g.w_r * g.r ** 2)[None, :, None, None, None, None]
    return np.sum(F * w, axis=(1, 2, 3, 4, 5))


def boundary_flux(F, g, j):
    """J at r = r_j per energy group, Eq. (Flux): r_j^2 * sum w cos(Theta) F(r_j)."""
    w = _angle_weights(g) * np.cos(g.Theta)[None, None, :, None]
    return g.r[j] ** 2 * np.sum(F[:, j] * w[None], axis=(1, 2, 3, 4))


def fluxes(F, g):
    """(N, J_in, J_out) per energy group."""
    return particle_number(F, g), boundary_flux(F, g, 0), boundary_flux(F, g, g.n_r - 1)


def outgoing_flux_map(F, g):
    """j(eps, theta, phi) = sum over cos(Theta_i) > 0 and Phi_m of
    w_i (2 pi / n_Phi) cos(Theta_i) F(r_out, theta, phi, Theta_i, Phi_m)."""
    cT = np.cos(g.Theta)
    w = np.where(cT > 0, g.w_Theta * cT, 0.0)[:, None] * (2.0 * np.pi / g.n_Phi)
    return np.sum(F[:, g.n_r - 1] * w, axis=(3, 4))


def outgoing_flux_map_T(jbar, g):
    """Transpose of outgoing_flux_map: a full-shape array that is zero except at
    r_out."""
    cT = np.cos(g.Theta)
    w = np.where(cT > 0, g.w_Theta * cT, 0.0)[:, None] * (2.0 * np.pi / g.n_Phi)
    out = np.zeros(g.shape)
    out[:, g.n_r - 1] = jbar[:, :, :, None, None] * w
    return out
