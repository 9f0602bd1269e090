"""Oracle: Fokker-Planck energy coupling of the transport equation (Sect. 3.2,
Eq. Transpfp), on a Chebyshev energy axis.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With the coupling on, the n_eps energy groups are the Chebyshev-Gauss-Lobatto
nodes gamma_k of [gamma_min, gamma_max] (ascending, grid.cgl_nodes), and the
right-hand side of every (eps, r, theta, phi) plane gains the isotropic source

    sigma * S(gamma),
    S = (1/4pi) d/dgamma [ alpha gamma^2 dM0/dgamma + (gamma^2 - 2 alpha gamma) M0 ]
        + (3 / (128 pi^2)) d/dgamma Q,
    M0 = int F dw,
    Q  = int int [1 - mu + mu^2 - mu^3] F(w') F(w'') dw' dw'',   mu = w' . w'',

where sigma (the plane's scattering coefficient) stands for n sigma_Th.  With the
Thomson phase function p(mu) = (3/4)(1 + mu^2) in the scattering term (ops), the
right-hand side is that of Eq. (Transpfp): -sigma F + sigma (K F) + sigma S.  S
is added to the emissivity eta of the plane, so it is set to zero at the inflow
nodes with the rest of the right-hand side.

Readings of the paper (listed in the design notes):

* Sign.  Eq. (Kompa) as printed, dF/dt = -n sigma d/dgamma [flux], makes the
  energy diffusion alpha gamma^2 d2F/dgamma2 run backwards in time (ill-posed);
  the linear part of Eq. (Transpfp) has the well-posed sign.  The induced
  (F^2) term of Eq. (Transpfp), with its printed factor -3/(128 pi^2), reduces
  for an isotropic F to -(1/2) dF^2/dgamma; the steady state the paper gives,
  the Bose distribution of Eq. (Bose), cancels the flux
  alpha gamma^2 F' + (gamma^2 - 2 alpha gamma) F + F^2/2 only with +F^2/2.  The
  oracle therefore takes dF/dt = +n sigma d/dgamma [flux] for an isotropic F,
  i.e. the factor +3/(128 pi^2) in front of the induced term.
* The double angular integral is evaluated through the moments of F,
  Mk = int w (x) ... (x) w F dw (rank 0 to 3, the plane quadrature of ops:
  Fejer in cos Theta, uniform in Phi): the kernel 1 - mu + mu^2 - mu^3 gives
  Q = M0^2 - M1.M1 + M2:M2 - M3:.M3 (full contractions).  A test checks this
  against the double sum over the quadrature nodes.
* The energy derivative is the collocation matrix of the CGL nodes
  (grid.cheb_diff_matrix on [gamma_min, gamma_max]), applied to the flux with no
  boundary condition: the number of particles, sum over the Clenshaw-Curtis
  weights of the energy nodes (Eq. Cosph), changes by the flux difference
  between the two ends, which vanishes when F does.
"""

import numpy as np

from . import grid as _grid
from . import ops


def energy_nodes(n_eps, gamma_min, gamma_max):
    """The energy of each group: CGL nodes of [gamma_min, gamma_max], ascending."""
    return _grid.cgl_nodes(n_eps, gamma_min, gamma_max)


def _quadrature(g):
    """Weights of int dw over one (Theta, Phi) plane, shape (n_Theta, n_Phi)."""
    return np.repeat((g.w_Theta * (2.0 * np.pi / g.n_Phi))[:, None], g.n_Phi, axis=1)


def moments(F, g):
    """Angular moments of F over each plane: M0 [..], M1 [.., 3], M2 [.., 3, 3],
    M3 [.., 3, 3, 3], with the leading axes (eps, r, theta, phi)."""
    w = _quadrature(g)
    om = ops.plane_directions(g).reshape(g.n_Theta, g.n_Phi, 3)
    wF = F * w
    M0 = wF.sum(axis=(4, 5))
    M1 = np.einsum("...ij,ija->...a", wF, om)
    M2 = np.einsum("...ij,ija,ijb->...ab", wF, om, om)
    M3 = np.einsum("...ij,ija,ijb,ijc->...abc", wF, om, om, om)
    return M0, M1, M2, M3


def induced_Q(F, g):
    """Q = int int [1 - mu + mu^2 - mu^3] F(w') F(w'') dw' dw'' per plane, from
    the moments."""
    M0, M1, M2, M3 = moments(F, g)
    return (M0 * M0 - np.einsum("...a,...a->...", M1, M1) + np.einsum("...ab,...ab->...", M2, M2)
            - np.einsum("...abc,...abc->...", M3, M3))


def fp_source(F, g, sigma, gamma_min, gamma_max, alpha):
    """sigma * S per plane, shape (n_eps, n_r, n_theta, n_phi) (module docstring)."""
    gam = energy_nodes(g.n_eps, gamma_min, gamma_max)
    D = _grid.cheb_diff_matrix(g.n_eps, gamma_min, gamma_max)
    M0 = moments(F, g)[0]
    Q = induced_Q(F, g)
    dM0 = np.tensordot(D, M0, axes=(1, 0))
    gc = gam.reshape(-1, 1, 1, 1)
    flux = alpha * gc * gc * dM0 + (gc * gc - 2.0 * alpha * gc) * M0
    S = np.tensordot(D, flux, axes=(1, 0)) / (4.0 * np.pi) + (3.0 / (128.0 * np.pi ** 2)) * np.tensordot(D, Q, axes=(1, 0))
    return np.asarray(sigma, np.float64).reshape(S.shape) * S


def fp_rhs_T(Y, X, g, sigma, gamma_min, gamma_max, alpha, bc=True):
    """Transpose of the linearisation at Y of the coupling's part of the
    right-hand side, F -> M sigma S(F) (broadcast over each plane, M the inflow
    mask), applied to X (rank 6):

        u  = sigma sum_w (M X)                    per plane
        a0 = L1^T u,  aQ = 3/(128 pi^2) D^T u     along gamma, with
        L1 = (1/4pi) D [diag(alpha gamma^2) D + diag(gamma^2 - 2 alpha gamma)]
        A0 = a0 + 2 aQ M0,  A1 = -2 aQ M1,  A2 = 2 aQ M2,  A3 = -2 aQ M3
        result(w) = wq(w) [A0 + A1.w + A2:ww + A3:.www]

    (dQ = 2 (M0 dM0 - M1.dM1 + M2:dM2 - M3:.dM3); Mk the moments of Y; wq the
    plane quadrature weight of the direction)."""
    Xm = X * ops.inflow_mask(g) if bc else X
    u = np.asarray(sigma, np.float64).reshape(Xm.shape[:4]) * Xm.sum(axis=(4, 5))
    gam = energy_nodes(g.n_eps, gamma_min, gamma_max)
    D = _grid.cheb_diff_matrix(g.n_eps, gamma_min, gamma_max)
    L1 = D @ (np.diag(alpha * gam * gam) @ D + np.diag(gam * gam - 2.0 * alpha * gam)) / (4.0 * np.pi)
    a0 = np.tensordot(L1.T, u, axes=(1, 0))
    aQ = (3.0 / (128.0 * np.pi ** 2)) * np.tensordot(D.T, u, axes=(1, 0))
    M0, M1, M2, M3 = moments(Y, g)
    A0 = a0 + 2.0 * aQ * M0
    A1 = -2.0 * aQ[..., None] * M1
    A2 = 2.0 * aQ[..., None, None] * M2
    A3 = -2.0 * aQ[..., None, None, None] * M3
    om = ops.plane_directions(g).reshape(g.n_Theta, g.n_Phi, 3)
    poly = (A0[..., None, None] + np.einsum("...a,ija->...ij", A1, om)
            + np.einsum("...ab,ija,ijb->...ij", A2, om, om)
            + np.einsum("...abc,ija,ijb,ijc->...ij", A3, om, om, om))
    return poly * _quadrature(g)


def kompaneets_flux(F, gam, dF, alpha):
    """The flux of Eq. (Kompa) for an isotropic, homogeneous F(gamma) given with
    its derivative dF: alpha gamma^2 F' + (gamma^2 - 2 alpha gamma) F + F^2/2."""
    return alpha * gam * gam * dF + (gam * gam - 2.0 * alpha * gam) * F + 0.5 * F * F
