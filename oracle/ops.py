"""Oracle operators: Liouville operator, collision term, inflow mask, right-hand side,
spectral filter, and the exact transposes used by the discrete adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Array layout: F[eps][r][theta][phi][Theta][Phi] (axes 0..5), FP64.

Readings of the paper used here (each is listed in the design notes):

* Eq. (sing) in Sect. 4.1 prints cos(Phi) in front of the singular phi and Phi
  derivatives; Eq. (Liouvsph) and the conservative form of App. A
  (Eq. Cohercons) have sin(Phi), and only sin(Phi) gives L omega_i = 0
  (Eq. prop2).  The operator below follows Eq. (Liouvsph).
* theta and Theta derivatives use double-Fourier-sphere lines: the point
  (-theta, phi, Theta, Phi) is the point (theta, phi + pi, Theta, Phi + pi), and
  the direction (-Theta, Phi) is the direction (Theta, Phi + pi) (both follow
  from Eqs. omegax-omegaz).  Nodes are half-shifted, so no node sits on a pole
  or on Theta = pi/2.
* The collision term is Eq. (Transp) with coherent scattering
  (Eq. sigmadif), the density absorbed into kappa = n sigma_a, sigma = n x (total
  scattering cross section), eta = n S, and without the induced-process factors
  (they make the equation nonlinear):
      C(F) = eta - (kappa + sigma) F + sigma (K F),
      (K F)(omega) = sum_{omega'} wq(omega') p(omega . omega') F(omega'),
      wq(Theta_i, Phi_m) = w_i (2pi/n_Phi) / (4pi)   (Fejer in cos Theta),
  with the phase function p(mu) = c0 + c1 mu + c2 mu^2 normalised by
  c0 = 1 - c2/3 (its mean over the sphere is one, so sigma is the total
  scattering opacity).  Isotropic scattering (Eq. sigman with B = 0) is
  c1 = c2 = 0, where K F is the angular mean <F>; Eq. sigman gives c1 = B/A
  (-1/3 and -1/10 for the neutron and proton kernels, Eqs. crossnun, crossnup);
  Thomson scattering, Eq. sigmaTh, is p = (3/4)(1 + mu^2): its printed
  prefactor is garbled, and this normalisation is the one of the azimuthally
  integrated kernel (3/8)(1 + cos^2 cos'^2 + sin^2 sin'^2 / 2) of App. B
  (Eq. speccons).  Directions are omega = (cos Theta, sin Theta cos Phi,
  sin Theta sin Phi) in the local orthonormal frame of the position; omega .
  omega' does not depend on that frame.
* Inflow (Sect. 4.2, Eq. Sphedif): F is imposed at r = r_in where
  cos(Theta) > 0 and at r = r_out where cos(Theta) < 0; the right-hand side is
  set to zero there (a collocation analogue of the paper's Tau imposition).
"""

import numpy as np

AX_EPS, AX_R, AX_TH, AX_PH, AX_TTH, AX_TPH = range(6)


def apply_along(D, F, axis):
    """(D F) along one axis: out[..., i, ...] = sum_k D[i, k] F[..., k, ...]."""
    out = np.tensordot(D, F, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


# ---------------------------------------------------------------------------
# the five 1D derivatives


def d_r(F, g):
    """Chebyshev collocation derivative along r."""
    return apply_along(g.D_r, F, AX_R)


def d_phi(F, g):
    """Fourier derivative along phi (periodic, n_phi points)."""
    return apply_along(g.D_phi, F, AX_PH)


def d_Phi(F, g):
    """Fourier derivative along Phi (periodic, n_Phi points)."""
    return apply_along(g.D_Phi, F, AX_TPH)


def dfs_extend_theta(F, g):
    """Build the 2 n_theta periodic DFS line in theta for every (phi_k, Phi_m).

    Entry i < n_theta is F(theta_i, phi_k, Phi_m); entry 2 n_theta - 1 - i is the
    value at colatitude -theta_i, i.e. F(theta_i, phi_k + pi, Phi_m + pi).
    """
    partner = np.roll(np.roll(F, -(g.n_phi // 2), axis=AX_PH), -(g.n_Phi // 2), axis=AX_TPH)
    return np.concatenate([F, np.flip(partner, axis=AX_TH)], axis=AX_TH)


def dfs_extend_theta_T(G, g):
    """Transpose of dfs_extend_theta: fold the 2 n_theta line back onto F's shape."""
    n = g.n_theta
    head = np.take(G, np.arange(n), axis=AX_TH)
    tail = np.flip(np.take(G, np.arange(n, 2 * n), axis=AX_TH), axis=AX_TH)
    back = np.roll(np.roll(tail, g.n_phi // 2, axis=AX_PH), g.n_Phi // 2, axis=AX_TPH)
    return head + back


def dfs_extend_Theta(F, g):
    """Build the 2 n_Theta periodic DFS line in Theta for every Phi_m.

    Entry i < n_Theta is F(Theta_i, Phi_m); entry 2 n_Theta - 1 - i is the value
    at -Theta_i, i.e. F(Theta_i, Phi_m + pi).
    """
    partner = np.roll(F, -(g.n_Phi // 2), axis=AX_TPH)
    return np.concatenate([F, np.flip(partner, axis=AX_TTH)], axis=AX_TTH)


def dfs_extend_Theta_T(G, g):
    n = g.n_Theta
    head = np.take(G, np.arange(n), axis=AX_TTH)
    tail = np.flip(np.take(G, np.arange(n, 2 * n), axis=AX_TTH), axis=AX_TTH)
    return head + np.roll(tail, g.n_Phi // 2, axis=AX_TPH)


def d_theta(F, g):
    """DFS Fourier derivative along theta: differentiate the 2 n_theta line, keep
    the first n_theta entries (the derivative at theta_i for this (phi_k, Phi_m))."""
    G = apply_along(g.D_theta, dfs_extend_theta(F, g), AX_TH)
    return np.take(G, np.arange(g.n_theta), axis=AX_TH)


def d_Theta(F, g):
    """DFS Fourier derivative along Theta (within each (Theta, Phi) plane)."""
    G = apply_along(g.D_Theta, dfs_extend_Theta(F, g), AX_TTH)
    return np.take(G, np.arange(g.n_Theta), axis=AX_TTH)


def _pad_half(X, axis, n):
    """Transpose of 'keep the first n of 2n entries': zero-pad to length 2n."""
    shape = list(X.shape)
    shape[axis] = n
    return np.concatenate([X, np.zeros(shape)], axis=axis)


def d_theta_T(X, g):
    """Exact transpose of d_theta."""
    G = _pad_half(X, AX_TH, g.n_theta)
    return dfs_extend_theta_T(apply_along(g.D_theta.T, G, AX_TH), g)


def d_Theta_T(X, g):
    """Exact transpose of d_Theta."""
    G = _pad_half(X, AX_TTH, g.n_Theta)
    return dfs_extend_Theta_T(apply_along(g.D_Theta.T, G, AX_TTH), g)


# ---------------------------------------------------------------------------
# the Liouville operator, Eq. (Liouvsph)


def liouville_coefficients(g):
    """Pointwise coefficients of the five terms of Eq. (Liouvsph), rank-6 broadcastable:
        c_r   = cos Theta
        c_th  = sin Theta cos Phi / r
        c_ph  = sin Theta sin Phi / (r sin theta)
        c_Th  = -sin Theta / r
        c_Ph  = -sin Theta sin Phi cos theta / (r sin theta)
    """
    r, th, ph, Th, Ph = g.mesh()
    c_r = np.cos(Th) + 0.0 * r
    c_th = np.sin(Th) * np.cos(Ph) / r
    c_ph = np.sin(Th) * np.sin(Ph) / (r * np.sin(th))
    c_Th = -np.sin(Th) / r + 0.0 * Ph
    c_Ph = -np.sin(Th) * np.sin(Ph) * np.cos(th) / (r * np.sin(th))
    return c_r, c_th, c_ph, c_Th, c_Ph


def apply_L(F, g):
    """L_sph F, Eq. (Liouvsph): the sum of the r, theta, phi, Theta, Phi terms."""
    c_r, c_th, c_ph, c_Th, c_Ph = liouville_coefficients(g)
    return (c_r * d_r(F, g) + c_th * d_theta(F, g) + c_ph * d_phi(F, g)
            + c_Th * d_Theta(F, g) + c_Ph * d_Phi(F, g))


def apply_L_angular(F, g):
    """L_sph F without the radial term (the four angular terms of Eq. Liouvsph)."""
    _, c_th, c_ph, c_Th, c_Ph = liouville_coefficients(g)
    return c_th * d_theta(F, g) + c_ph * d_phi(F, g) + c_Th * d_Theta(F, g) + c_Ph * d_Phi(F, g)


def radial_implicit_matrices(g, dt, bc=True):
    """Backward-Euler radial advection (the implicit scheme of App. B): for each
    Theta node, F_new solves (I + dt cos(Theta_i) D_r) F_new = F along every r
    line, with the inflow row (r_in for cos Theta > 0, r_out for cos Theta < 0)
    replaced by F_new = F there when bc is True.  Returns the inverses, shape
    (n_Theta, n_r, n_r)."""
    out = np.empty((g.n_Theta, g.n_r, g.n_r))
    for i, Th in enumerate(g.Theta):
        c = np.cos(Th)
        A = np.eye(g.n_r) + dt * c * g.D_r
        if bc:
            row = 0 if c > 0 else g.n_r - 1
            A[row] = 0.0
            A[row, row] = 1.0
        out[i] = np.linalg.inv(A)
    return out


def apply_radial_implicit(F, g, dt, bc=True):
    """F_new = B_i F along r for every Theta node i (radial_implicit_matrices)."""
    B = radial_implicit_matrices(g, dt, bc)
    out = np.empty_like(F)
    for i in range(g.n_Theta):
        out[:, :, :, :, i, :] = apply_along(B[i], F[:, :, :, :, i, :], AX_R)
    return out


def apply_LT(G, g):
    """Exact transpose of apply_L (as a matrix on the nodal values):
    sum over directions of D_dir^T (c_dir * G)."""
    c_r, c_th, c_ph, c_Th, c_Ph = liouville_coefficients(g)
    return (apply_along(g.D_r.T, c_r * G, AX_R)
            + d_theta_T(c_th * G, g)
            + apply_along(g.D_phi.T, c_ph * G, AX_PH)
            + d_Theta_T(c_Th * G, g)
            + apply_along(g.D_Phi.T, c_Ph * G, AX_TPH))


# ---------------------------------------------------------------------------
# collision term and boundary mask


def angular_mean(F, g):
    """<F> = (1/4pi) sum_i sum_m w_i (2pi/n_Phi) F[..., i, m], kept as a rank-6
    array of shape (..., 1, 1)."""
    w = g.w_Theta[:, None] * (2.0 * np.pi / g.n_Phi) / (4.0 * np.pi)
    return np.sum(F * w, axis=(AX_TTH, AX_TPH), keepdims=True)


def angular_mean_T(X, g):
    """Transpose of F -> broadcast(<F>): sum X over the plane, times the weights."""
    w = g.w_Theta[:, None] * (2.0 * np.pi / g.n_Phi) / (4.0 * np.pi)
    return np.sum(X, axis=(AX_TTH, AX_TPH), keepdims=True) * w


def plane_directions(g):
    """Unit vectors omega of the (Theta, Phi) nodes in the local frame, shape
    (n_Theta n_Phi, 3), rows in C order over (i, m)."""
    Th, Ph = np.meshgrid(g.Theta, g.Phi, indexing="ij")
    om = np.stack([np.cos(Th), np.sin(Th) * np.cos(Ph), np.sin(Th) * np.sin(Ph)], axis=-1)
    return om.reshape(-1, 3)


def scattering_matrix(g, kernel):
    """Dense in-scattering matrix of one (Theta, Phi) plane for the phase
    function p(mu) = c0 + c1 mu + c2 mu^2, kernel = (c1, c2), c0 = 1 - c2/3:
    K[a, b] = wq(b) p(omega_a . omega_b), rows and columns in C order over (i, m)."""
    c1, c2 = kernel
    c0 = 1.0 - c2 / 3.0
    om = plane_directions(g)
    mu = om @ om.T
    wq = np.repeat(g.w_Theta * (2.0 * np.pi / g.n_Phi) / (4.0 * np.pi), g.n_Phi)
    return (c0 + c1 * mu + c2 * mu * mu) * wq[None, :]


def is_isotropic(kernel):
    return kernel is None or (kernel[0] == 0.0 and kernel[1] == 0.0)


def scatter_in(F, g, kernel=None):
    """K F over every (Theta, Phi) plane (the angular mean <F>, broadcastable,
    for the isotropic kernel)."""
    if is_isotropic(kernel):
        return angular_mean(F, g)
    K = scattering_matrix(g, kernel)
    n = g.n_Theta * g.n_Phi
    return (F.reshape(-1, n) @ K.T).reshape(F.shape)


def scatter_in_T(X, g, kernel=None):
    """Transpose of F -> K F."""
    if is_isotropic(kernel):
        return angular_mean_T(X, g)
    K = scattering_matrix(g, kernel)
    n = g.n_Theta * g.n_Phi
    X = np.broadcast_to(X, X.shape[:4] + (g.n_Theta, g.n_Phi))
    return (X.reshape(-1, n) @ K).reshape(X.shape)


def expand_coeff(c, g):
    """Isotropic coefficient field [eps][r][theta][phi] -> rank-6 broadcastable."""
    c = np.asarray(c, dtype=np.float64)
    return c.reshape(g.n_eps, g.n_r, g.n_theta, g.n_phi, 1, 1)


def collision(F, g, kappa, sigma, eta, kernel=None):
    """C(F) = eta - (kappa + sigma) F + sigma K F  (see the module docstring)."""
    k = expand_coeff(kappa, g)
    s = expand_coeff(sigma, g)
    e = expand_coeff(eta, g)
    return e - (k + s) * F + s * scatter_in(F, g, kernel)


def inflow_mask(g):
    """1 where F evolves, 0 at the inflow nodes (r_in, cos Theta > 0) and
    (r_out, cos Theta < 0); shape (1, n_r, 1, 1, n_Theta, 1)."""
    m = np.ones((1, g.n_r, 1, 1, g.n_Theta, 1))
    cT = np.cos(g.Theta)
    m[0, 0, 0, 0, cT > 0, 0] = 0.0
    m[0, g.n_r - 1, 0, 0, cT < 0, 0] = 0.0
    return m


def project_inflow(F, g, g_in=None, g_out=None):
    """Set F to the inflow values at the inflow nodes (zero where g_* is None).
    g_in, g_out: [eps][theta][phi][Theta][Phi]."""
    F = F.copy()
    cT = np.cos(g.Theta)
    pin = np.zeros(F[:, 0].shape) if g_in is None else np.asarray(g_in, np.float64)
    pout = np.zeros(F[:, -1].shape) if g_out is None else np.asarray(g_out, np.float64)
    for i in range(g.n_Theta):
        if cT[i] > 0:
            F[:, 0, :, :, i, :] = pin[:, :, :, i, :]
        elif cT[i] < 0:
            F[:, -1, :, :, i, :] = pout[:, :, :, i, :]
    return F


def rhs(F, g, kappa, sigma, eta, bc=True, scattering=True, kernel=None, radial=True):
    """Right-hand side dF/dt = -L_sph F + C(F) (Eqs. Transpfpsph, Transp), set to
    zero at the inflow nodes when bc is True; without the radial term of L_sph
    when radial is False (the explicit part of the radially implicit split)."""
    s = sigma if scattering else np.zeros_like(np.asarray(sigma, np.float64))
    LF = apply_L(F, g) if radial else apply_L_angular(F, g)
    out = -LF + collision(F, g, kappa, s, eta, kernel)
    if bc:
        out = out * inflow_mask(g)
    return out


def rhs_linear_T(X, g, kappa, sigma, bc=True, scattering=True, kernel=None):
    """Transpose of the linear part of rhs (A^T X, with A = M(-L - (k+s) + s K))."""
    if bc:
        X = X * inflow_mask(g)
    k = expand_coeff(kappa, g)
    s = expand_coeff(sigma, g) if scattering else 0.0 * k
    return -apply_LT(X, g) - (k + s) * X + scatter_in_T(s * X, g, kernel)


# ---------------------------------------------------------------------------
# spectral filter


def filter_matrix(n):
    """Grid-space form of the exponential filter exp(-36 (|k|/(n/2))^36) on a
    periodic line of n points (the paper only mentions adding viscosity in
    coefficient space, App. B; the filter shape is this build's reading).
    Returns the symmetric n x n matrix F_jl = (1/n) sum_k s(k) cos(k (x_j - x_l))
    over k = -n/2 .. n/2 - 1, with the Nyquist term taken as a cosine."""
    j = np.arange(n)
    M = np.zeros((n, n))
    for k in range(-(n // 2), n // 2):
        s = np.exp(-36.0 * (abs(k) / (n / 2.0)) ** 36)
        M += s * np.cos(2.0 * np.pi * k * (j[:, None] - j[None, :]) / n)
    return M / n


def radial_filter_matrix(g):
    """Nodal form of the same exponential filter on the Chebyshev expansion in r:
    F = sum_k a_k T_k(x) (interpolation on the CGL nodes, x in [-1, 1]) is mapped
    to sum_k s(k / (n_r - 1)) a_k T_k(x), s(eta) = exp(-36 eta^36).  With the
    Vandermonde matrix V_jk = T_k(x_j): M = V diag(s) V^-1.  (The paper filters
    nothing radially; it treats the radial discontinuity of its shell experiment
    with finite differences, Sect. 5.3.)"""
    n = g.n_r
    x = -np.cos(np.pi * np.arange(n) / (n - 1))
    V = np.polynomial.chebyshev.chebvander(x, n - 1)
    s = np.exp(-36.0 * (np.arange(n) / (n - 1.0)) ** 36)
    return V @ np.diag(s) @ np.linalg.inv(V)


def apply_filter(F, g, radial=False):
    """Filter every theta (DFS), phi, Theta (DFS) and Phi line, in that order,
    then (radial=True) every r line."""
    Ft = filter_matrix(2 * g.n_theta)
    G = apply_along(Ft, dfs_extend_theta(F, g), AX_TH)
    F = np.take(G, np.arange(g.n_theta), axis=AX_TH)
    F = apply_along(filter_matrix(g.n_phi), F, AX_PH)
    FT = filter_matrix(2 * g.n_Theta)
    G = apply_along(FT, dfs_extend_Theta(F, g), AX_TTH)
    F = np.take(G, np.arange(g.n_Theta), axis=AX_TTH)
    F = apply_along(filter_matrix(g.n_Phi), F, AX_TPH)
    if radial:
        F = apply_along(radial_filter_matrix(g), F, AX_R)
    return F


def apply_filter_T(X, g, radial=False):
    """Transpose of apply_filter: the angular line filters are symmetric and act
    on other axes than the radial one (their partner maps are shifts by pi, which
    commute with the circulant filters), so the transpose is the radial matrix
    transposed, then the angular filters."""
    if radial:
        X = apply_along(radial_filter_matrix(g).T, X, AX_R)
    return apply_filter(X, g)


# ---------------------------------------------------------------------------
# single-point evaluation (for sampled checks of large grids)


def rhs_at(F, g, kappa, sigma, eta, idx, bc=True, scattering=True, kernel=None):
    """The right-hand side at a single node idx = (e, j, l, k, i, m), computed
    from the five lines through that node and its (Theta, Phi) plane only.
    F may be any array-like indexable by numpy (e.g. a memory map)."""
    e, j, l, k, i, m = idx
    nth, nph, nTh, nPh = g.n_theta, g.n_phi, g.n_Theta, g.n_Phi
    kp, mp = (k + nph // 2) % nph, (m + nPh // 2) % nPh
    r, th, Th, Ph = g.r[j], g.theta[l], g.Theta[i], g.Phi[m]
    line_r = np.asarray(F[e, :, l, k, i, m], np.float64)
    dr = g.D_r[j] @ line_r
    th_line = np.concatenate([np.asarray(F[e, j, :, k, i, m], np.float64),
                              np.asarray(F[e, j, :, kp, i, mp], np.float64)[::-1]])
    dth = g.D_theta[l] @ th_line
    dph = g.D_phi[k] @ np.asarray(F[e, j, l, :, i, m], np.float64)
    plane = np.asarray(F[e, j, l, k], np.float64)
    Th_line = np.concatenate([plane[:, m], plane[:, mp][::-1]])
    dTh = g.D_Theta[i] @ Th_line
    dPh = g.D_Phi[m] @ plane[i, :]
    LF = (np.cos(Th) * dr + np.sin(Th) * np.cos(Ph) / r * dth
          + np.sin(Th) * np.sin(Ph) / (r * np.sin(th)) * dph
          - np.sin(Th) / r * dTh
          - np.sin(Th) * np.sin(Ph) * np.cos(th) / (r * np.sin(th)) * dPh)
    ka, si, et = (float(np.asarray(c)[e, j, l, k]) for c in (kappa, sigma, eta))
    if not scattering:
        si = 0.0
    if is_isotropic(kernel):
        inscat = np.sum(plane * g.w_Theta[:, None]) * (2.0 * np.pi / nPh) / (4.0 * np.pi)
    else:
        inscat = scattering_matrix(g, kernel)[i * nPh + m] @ plane.reshape(-1)
    out = -LF + et - (ka + si) * plane[i, m] + si * inscat
    if bc:
        cT = np.cos(Th)
        if (j == 0 and cT > 0) or (j == g.n_r - 1 and cT < 0):
            out = 0.0
    return out
