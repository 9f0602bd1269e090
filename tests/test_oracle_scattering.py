"""Pins of the oracle's anisotropic in-scattering operator K (phase function
p(mu) = c0 + c1 mu + c2 mu^2 with c0 = 1 - c2/3; Eqs. sigmadif, sigman, sigmaTh
and the azimuthally integrated Thomson kernel of App. B, Eq. speccons).

* K keeps constants and conserves the particle number (the normalisation of p,
  with a quadrature exact for quadratics in omega);
* Funk-Hecke: spherical harmonics of degree l are eigenfunctions with
  eigenvalue (1/2) int p(mu) P_l(mu) dmu: c0 + c2/3, c1/3, 2 c2/15 for l = 0, 1, 2;
* Thomson: for Phi-independent F, K reduces to the kernel printed in App. B;
* brute force: the dense right-hand side, RK4 step and adjoint assembled by
  explicit loops over direction pairs (tests/_brute.py).
"""

import math

import numpy as np
import pytest

from oracle import grid as og, ops, step, adjoint
from tests import _brute

KERNELS = {"thomson": (0.0, 0.75), "neutron": (-1.0 / 3.0, 0.0), "proton": (-0.1, 0.0),
           "mixed": (0.4, -0.6)}


def dirs(g):
    Th, Ph = np.meshgrid(g.Theta, g.Phi, indexing="ij")
    return np.cos(Th), np.sin(Th) * np.cos(Ph), np.sin(Th) * np.sin(Ph)


@pytest.mark.parametrize("name", list(KERNELS))
@pytest.mark.parametrize("nT", [4, 8, 16])
def test_constants_and_number(name, nT):
    g = og.make_grid(1, 3, 2, 4, nT, 2 * nT)
    K = ops.scattering_matrix(g, KERNELS[name])
    wq = np.repeat(g.w_Theta * (2 * np.pi / g.n_Phi) / (4 * np.pi), g.n_Phi)
    np.testing.assert_allclose(K @ np.ones(K.shape[0]), 1.0, atol=1e-14)
    np.testing.assert_allclose(wq @ K, wq, atol=1e-15)


@pytest.mark.parametrize("name", list(KERNELS))
def test_funk_hecke_eigenvalues(name):
    c1, c2 = KERNELS[name]
    c0 = 1 - c2 / 3
    g = og.make_grid(1, 3, 2, 4, 8, 16)
    K = ops.scattering_matrix(g, (c1, c2))
    x, y, z = (a.reshape(-1) for a in dirs(g))
    cases = [(np.ones_like(x), c0 + c2 / 3), (x, c1 / 3), (y, c1 / 3), (z, c1 / 3),
             (x * y, 2 * c2 / 15), (y * z, 2 * c2 / 15), (x * x - z * z, 2 * c2 / 15),
             (3 * x * x - 1, 2 * c2 / 15)]
    for f, lam in cases:
        np.testing.assert_allclose(K @ f, lam * f, atol=2e-15)


def test_thomson_reduces_to_azimuthally_integrated_kernel():
    g = og.make_grid(1, 3, 2, 4, 8, 16)
    rng = np.random.default_rng(0)
    f = rng.normal(size=g.n_Theta)
    F = np.repeat(f, g.n_Phi)
    got = (ops.scattering_matrix(g, KERNELS["thomson"]) @ F).reshape(g.n_Theta, g.n_Phi)
    c, s = np.cos(g.Theta), np.sin(g.Theta)
    want = np.array([sum(g.w_Theta[j] * 0.375 * (1 + (c[i] * c[j]) ** 2 + 0.5 * (s[i] * s[j]) ** 2) * f[j]
                         for j in range(g.n_Theta)) for i in range(g.n_Theta)])
    np.testing.assert_allclose(got, np.repeat(want[:, None], g.n_Phi, axis=1), atol=1e-14)


def test_isotropic_kernel_is_the_angular_mean():
    g = og.make_grid(2, 3, 2, 4, 4, 8)
    F = np.random.default_rng(1).normal(size=g.shape)
    K = ops.scattering_matrix(g, (0.0, 0.0))
    got = (F.reshape(-1, 32) @ K.T).reshape(g.shape)
    np.testing.assert_allclose(got, np.broadcast_to(ops.angular_mean(F, g), g.shape), atol=1e-15)


@pytest.mark.parametrize("name", ["thomson", "neutron", "mixed"])
def test_scattering_conserves_number_pointwise(name):
    g = og.make_grid(2, 3, 2, 4, 8, 16)
    F = np.random.default_rng(2).normal(size=g.shape)
    sig = np.ones(g.shape[:4])
    C = ops.collision(F, g, 0 * sig, sig, 0 * sig, KERNELS[name])
    w = g.w_Theta[:, None] * (2 * np.pi / g.n_Phi)
    assert np.max(np.abs(np.sum(C * w, axis=(4, 5)))) <= 1e-14 * np.max(np.abs(F))


def test_transpose_dot_product():
    g = og.make_grid(2, 5, 4, 8, 8, 16)
    rng = np.random.default_rng(5)
    x = rng.normal(size=g.shape)
    y = rng.normal(size=g.shape)
    kappa, sigma = (rng.uniform(0.2, 1.5, size=g.shape[:4]) for _ in range(2))
    for kern in KERNELS.values():
        lin = ops.rhs(x, g, kappa, sigma, 0 * kappa, kernel=kern)
        assert np.sum(lin * y) == pytest.approx(np.sum(x * ops.rhs_linear_T(y, g, kappa, sigma, kernel=kern)),
                                                rel=1e-13)


@pytest.mark.parametrize("name", ["thomson", "neutron"])
def test_brute_force_rhs_step_adjoint(name):
    # n_Theta = 4: unequal quadrature weights, so K is not symmetric
    kern = KERNELS[name]
    g = og.make_grid(1, 3, 2, 4, 4, 8)
    rng = np.random.default_rng(3)
    kappa, sigma, eta = (rng.uniform(0.2, 1.5, size=(1, 3, 2, 4)) for _ in range(3))
    p = step.Physics(kappa, sigma, eta, bc=True, scattering=True, kernel=kern)
    A = _brute.assemble(g, kappa, sigma, bc=True, kernel=kern)
    b = _brute.source(g, eta, bc=True)
    y = rng.normal(size=g.shape)
    np.testing.assert_allclose(step.rhs(y, g, p).ravel(), A @ y.ravel() + b, atol=1e-12)
    dt = 0.05
    P, Q = _brute.rk4_polys(dt * A)
    np.testing.assert_allclose(step.rk4_step(y, g, p, dt).ravel(), P @ y.ravel() + dt * Q @ b, atol=1e-12)
    lam = rng.normal(size=g.shape)
    lam_prev, gk, ge, gs = adjoint.adjoint_step(y, lam, g, p, dt)
    np.testing.assert_allclose(lam_prev.ravel(), P.T @ lam.ravel(), atol=1e-12)
    h = 1e-30
    for q in [(0, 0, 0, 0), (0, 2, 1, 3), (0, 1, 1, 1)]:
        sc = sigma.astype(complex)
        sc[q] += 1j * h
        Pc, Qc = _brute.rk4_polys(dt * _brute.assemble(g, kappa, sc, bc=True, dtype=complex, kernel=kern))
        d = np.imag(lam.ravel() @ (Pc @ y.ravel() + dt * Qc @ b)) / h
        assert gs[q] == pytest.approx(d, rel=1e-11, abs=1e-13), q


def test_rhs_at_with_kernel():
    g = og.make_grid(2, 5, 4, 8, 4, 8)
    rng = np.random.default_rng(4)
    F = rng.normal(size=g.shape)
    kappa, sigma, eta = (rng.uniform(0.2, 1.5, size=g.shape[:4]) for _ in range(3))
    full = ops.rhs(F, g, kappa, sigma, eta, kernel=KERNELS["thomson"])
    for idx in [(0, 0, 0, 0, 0, 0), (1, 4, 3, 7, 3, 7), (1, 2, 1, 5, 2, 3)]:
        v = ops.rhs_at(F, g, kappa, sigma, eta, idx, kernel=KERNELS["thomson"])
        assert v == pytest.approx(full[idx], rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("name", ["isotropic", "thomson", "neutron", "mixed"])
def test_isotropisation_closed_form(name):
    """Sect. 5.2's uniform-medium experiment with smooth data: the RK4 solution is
    the Funk-Hecke/RK4 closed form (L F = 0 for F depending on omega only)."""
    from oracle import closed_forms as cf
    kern = (0.0, 0.0) if name == "isotropic" else KERNELS[name]
    g = og.make_grid(1, 5, 4, 8, 8, 16)
    a, b = 1.0, (0.5, -0.3, 0.2)
    Q = np.array([[0.4, 0.1, -0.2], [0.1, -0.1, 0.3], [-0.2, 0.3, 0.25]])
    F0 = cf.isotropisation(g, a, b, Q, 0.0, kern, 0.0, 0)
    dt, n = g.dt_default(), 10  # a stable step for the Liouville part
    sig = 0.5 / dt              # sigma dt = 0.5
    z = np.zeros(g.shape[:4])
    p = step.Physics(z, z + sig, z, bc=False, scattering=True, kernel=kern)
    got = step.run(F0, g, p, dt, n)
    want = cf.isotropisation(g, a, b, Q, sig, kern, dt, n)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # the isotropic part is conserved; the anisotropic parts decay
    assert np.max(np.abs(want - F0)) > 1e-3


@pytest.mark.parametrize("name", ["isotropic", "thomson"])
def test_ab2_isotropisation_closed_form(name):
    """Adams-Bashforth (Sect. 5.1) on the uniform-medium problem: each degree-l
    part follows the scalar AB2 recurrence with the Funk-Hecke rate; continuing a
    run from its returned slope equals one longer run."""
    from oracle import closed_forms as cf
    kern = (0.0, 0.0) if name == "isotropic" else KERNELS[name]
    g = og.make_grid(1, 5, 4, 8, 8, 16)
    a, b = 1.0, (0.5, -0.3, 0.2)
    Q = np.array([[0.4, 0.1, -0.2], [0.1, -0.1, 0.3], [-0.2, 0.3, 0.25]])
    F0 = cf.isotropisation(g, a, b, Q, 0.0, kern, 0.0, 0)
    dt = g.dt_default()
    sig = 0.3 / dt
    z = np.zeros(g.shape[:4])
    p = step.Physics(z, z + sig, z, bc=False, scattering=True, kernel=kern)
    got, _ = step.ab2_run(F0, g, p, dt, 12)
    want = cf.isotropisation_ab2(g, a, b, Q, sig, kern, dt, 12)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    y5, k5 = step.ab2_run(F0, g, p, dt, 5)
    y12, _ = step.ab2_run(y5, g, p, dt, 7, k_prev=k5)
    assert np.max(np.abs(y12 - got)) <= 1e-14 * np.max(np.abs(got))
