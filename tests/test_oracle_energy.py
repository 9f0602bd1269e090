"""Pins of the oracle's Fokker-Planck energy coupling (oracle/energy.py; Sect. 3.2,
Eqs. Transpfp, Kompa, Cosph, Bose), each against something other than the
oracle itself:

* an isotropic, homogeneous F(gamma) reduces Eq. (Transpfp) to the Kompaneets
  operator d/dgamma [alpha gamma^2 F' + (gamma^2 - 2 alpha gamma) F + F^2/2],
  exact on polynomials (numpy.polynomial arithmetic and derivative);
* the induced-scattering double integral from the moments equals the double sum
  over the quadrature nodes of its kernel 1 - mu + mu^2 - mu^3 (brute force);
* the Bose distribution of Eq. (Bose) is a steady state, to spectral accuracy
  that improves with the number of energy nodes;
* the source is an exact derivative in gamma: its Clenshaw-Curtis integral is
  the difference of the flux at the two ends (particle number, Eq. Cosph).
"""

import numpy as np
import pytest

from oracle import energy, grid, ops


def _grid(n_eps, n_Theta=4, n_Phi=8):
    return grid.make_grid(n_eps, 3, 2, 4, n_Theta, n_Phi)


def _isotropic(g, f_of_gamma, gam):
    F = np.empty((g.n_eps, g.n_r, g.n_theta, g.n_phi, g.n_Theta, g.n_Phi))
    F[...] = f_of_gamma(gam).reshape(-1, 1, 1, 1, 1, 1)
    return F


def test_isotropic_reduction_is_kompaneets():
    g = _grid(8)
    gmin, gmax, alpha = 0.0, 2.0, 0.3
    gam = energy.energy_nodes(g.n_eps, gmin, gmax)
    P = np.polynomial.Polynomial([1.0, 0.5, -0.2])
    x = np.polynomial.Polynomial([0.0, 1.0])
    flux = alpha * x * x * P.deriv() + (x * x - 2.0 * alpha * x) * P + 0.5 * P * P
    want = flux.deriv()(gam)
    F = _isotropic(g, P, gam)
    src = energy.fp_source(F, g, np.ones(F.shape[:4]), gmin, gmax, alpha)
    err = np.max(np.abs(src - want.reshape(-1, 1, 1, 1))) / np.max(np.abs(want))
    assert err <= 1e-12, err
    # sigma scales the source plane by plane
    s = np.random.default_rng(0).uniform(0.5, 2.0, F.shape[:4])
    assert np.allclose(energy.fp_source(F, g, s, gmin, gmax, alpha), s * src, rtol=1e-14, atol=0.0)


def test_induced_Q_matches_double_sum():
    g = _grid(2)
    rng = np.random.default_rng(1)
    F = rng.normal(size=(g.n_eps, g.n_r, g.n_theta, g.n_phi, g.n_Theta, g.n_Phi))
    # directions and weights written out from the node definitions
    dirs, wts = [], []
    for i, T in enumerate(g.Theta):
        for m, Ph in enumerate(g.Phi):
            dirs.append((np.cos(T), np.sin(T) * np.cos(Ph), np.sin(T) * np.sin(Ph)))
            wts.append(g.w_Theta[i] * 2.0 * np.pi / g.n_Phi)
    dirs, wts = np.array(dirs), np.array(wts)
    Q = energy.induced_Q(F, g)
    flat = F.reshape(F.shape[:4] + (-1,))
    for idx in np.ndindex(*F.shape[:4]):
        f = flat[idx]
        q = 0.0
        for a in range(len(wts)):
            for b in range(len(wts)):
                mu = float(dirs[a] @ dirs[b])
                q += wts[a] * wts[b] * (1.0 - mu + mu ** 2 - mu ** 3) * f[a] * f[b]
        assert abs(Q[idx] - q) <= 1e-12 * max(abs(q), 1.0), (idx, Q[idx], q)


@pytest.mark.parametrize("n_eps", [24, 32])
def test_bose_distribution_is_steady(n_eps):
    # the distribution has a pole at gamma = mu; with mu = -1 it lies far enough
    # from [0, 2] for the Chebyshev interpolant to converge quickly
    gmin, gmax, alpha, mu = 0.0, 2.0, 0.2, -1.0

    def bose(x):
        return 2.0 * x * x / np.expm1((x - mu) / alpha)

    def residual(n):
        g = _grid(n)
        gam = energy.energy_nodes(n, gmin, gmax)
        F = _isotropic(g, bose, gam)
        src = energy.fp_source(F, g, np.ones(F.shape[:4]), gmin, gmax, alpha)
        # scale: the energy drift term alone, d/dgamma (gamma^2 F)
        D = grid.cheb_diff_matrix(n, gmin, gmax)
        drift = D @ (gam * gam * bose(gam))
        return np.max(np.abs(src)) / np.max(np.abs(drift))

    r = residual(n_eps)
    bound = {24: 1e-5, 32: 1e-9}[n_eps]
    assert r <= bound, r
    if n_eps == 32:
        assert r < 1e-3 * residual(24)


def test_induced_sign_against_a_degenerate_bose_distribution():
    """Near degeneracy (mu close to 0) the F^2/2 part of the flux matters: the
    Bose distribution is steady with the sign taken here, and with the printed
    sign of the induced term (-F^2/2 in the flux) its source would be
    -d(F^2)/dgamma, a tenth of the energy drift."""
    n, gmin, gmax, alpha, mu = 64, 0.0, 2.0, 0.2, -0.2
    g = _grid(n)
    gam = energy.energy_nodes(n, gmin, gmax)
    b = 2.0 * gam * gam / np.expm1((gam - mu) / alpha)
    F = _isotropic(g, lambda x: 2.0 * x * x / np.expm1((x - mu) / alpha), gam)
    D = grid.cheb_diff_matrix(n, gmin, gmax)
    src = energy.fp_source(F, g, np.ones(F.shape[:4]), gmin, gmax, alpha)
    scale = np.max(np.abs(D @ (gam * gam * b)))
    printed = src - (D @ b ** 2).reshape(-1, 1, 1, 1)
    assert np.max(np.abs(src)) <= 1e-9 * scale
    assert np.max(np.abs(printed)) >= 5e-2 * scale


def test_source_integrates_to_the_end_fluxes():
    g = _grid(9)
    gmin, gmax, alpha = 0.5, 2.5, 0.15
    rng = np.random.default_rng(2)
    F = rng.normal(size=(g.n_eps, g.n_r, g.n_theta, g.n_phi, g.n_Theta, g.n_Phi))
    sigma = np.ones(F.shape[:4])
    src = energy.fp_source(F, g, sigma, gmin, gmax, alpha)
    W = 0.5 * (gmax - gmin) * grid.clenshaw_curtis_weights(g.n_eps)
    lhs = np.tensordot(W, src, axes=(0, 0))
    # the flux at the two end nodes, from the moments there
    gam = energy.energy_nodes(g.n_eps, gmin, gmax)
    D = grid.cheb_diff_matrix(g.n_eps, gmin, gmax)
    M0 = energy.moments(F, g)[0]
    dM0 = np.tensordot(D, M0, axes=(1, 0))
    Q = energy.induced_Q(F, g)
    end = []
    for k in (0, g.n_eps - 1):
        lin = alpha * gam[k] ** 2 * dM0[k] + (gam[k] ** 2 - 2.0 * alpha * gam[k]) * M0[k]
        end.append(lin / (4.0 * np.pi) + 3.0 / (128.0 * np.pi ** 2) * Q[k])
    want = end[1] - end[0]
    assert np.max(np.abs(lhs - want)) <= 1e-11 * np.max(np.abs(want))


def test_rhs_adds_the_source_to_eta():
    from oracle import step
    g = _grid(5)
    rng = np.random.default_rng(3)
    F = rng.normal(size=(g.n_eps, g.n_r, g.n_theta, g.n_phi, g.n_Theta, g.n_Phi))
    k, s, e = (rng.uniform(0.1, 1.0, F.shape[:4]) for _ in range(3))
    p0 = step.Physics(k, s, e, kernel=(0.0, 0.75))
    p1 = step.Physics(k, s, e, kernel=(0.0, 0.75), energy=(0.1, 1.1, 0.05))
    src = energy.fp_source(F, g, s, 0.1, 1.1, 0.05)
    want = step.rhs(F, g, p0) + ops.expand_coeff(src, g) * ops.inflow_mask(g)
    assert np.max(np.abs(step.rhs(F, g, p1) - want)) <= 1e-12 * np.max(np.abs(want))


def _coupled_case(seed, kernel=(0.0, 0.75)):
    from oracle import step
    g = _grid(5)
    rng = np.random.default_rng(seed)
    shp6 = (g.n_eps, g.n_r, g.n_theta, g.n_phi, g.n_Theta, g.n_Phi)
    Y = 0.3 * rng.normal(size=shp6)
    k, s, e = (rng.uniform(0.1, 1.0, shp6[:4]) for _ in range(3))
    p = step.Physics(k, s, e, kernel=kernel, energy=(0.1, 1.1, 0.05))
    return g, rng, shp6, Y, p


@pytest.mark.parametrize("kernel", [None, (0.0, 0.75)], ids=["isotropic", "thomson"])
def test_jacobian_transpose_by_complex_step(kernel):
    """<X, J(Y) d> with J d = Im rhs(Y + i h d) / h (exact: the right-hand side is
    analytic in F) equals <J(Y)^T X, d> from the linear transpose plus
    fp_rhs_T."""
    from oracle import step
    g, rng, shp6, Y, p = _coupled_case(4, kernel)
    d, X = rng.normal(size=shp6), rng.normal(size=shp6)
    h = 1e-30
    Jd = np.imag(step.rhs(Y + 1j * h * d, g, p)) / h
    JT = ops.rhs_linear_T(X, g, p.kappa, p.sigma, kernel=p.kernel) + energy.fp_rhs_T(Y, X, g, p.sigma, *p.energy)
    lhs, rhs = np.sum(X * Jd), np.sum(JT * d)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.sum(np.abs(X * Jd))), (lhs, rhs)


def test_adjoint_step_by_complex_step_and_differences():
    """The adjoint RK4 step with the coupling: dLoss/dy against the complex-step
    derivative of the step, and the sigma, kappa and eta gradients against central
    differences (the coefficient fields enter through real-valued helpers)."""
    from oracle import adjoint, step
    g, rng, shp6, y, p = _coupled_case(5)
    dt = 0.02
    lam = rng.normal(size=shp6)
    lam_prev, gk, ge, gs = adjoint.adjoint_step(y, lam, g, p, dt)
    d = rng.normal(size=shp6)
    h = 1e-30
    dir_y = np.sum(lam * np.imag(step.rk4_step(y + 1j * h * d, g, p, dt))) / h
    assert abs(dir_y - np.sum(lam_prev * d)) <= 1e-11 * np.sum(np.abs(lam_prev * d))
    import dataclasses
    for name, grad in (("sigma", gs), ("kappa", gk), ("eta", ge)):
        dc = rng.normal(size=shp6[:4])
        eps = 1e-6

        def J(sign):
            q = dataclasses.replace(p, **{name: getattr(p, name) + sign * eps * dc})
            return np.sum(lam * step.rk4_step(y, g, q, dt))
        fd = (J(1.0) - J(-1.0)) / (2.0 * eps)
        assert abs(fd - np.sum(grad * dc)) <= 1e-6 * max(abs(fd), 1e-12), (name, fd, np.sum(grad * dc))
