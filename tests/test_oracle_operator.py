"""Pins of the oracle's operator, collision term, time step, diagnostics and
adjoint: closed forms and invariants from the paper (Eqs. prop1, prop2, propf,
free streaming, Eq. Cons), exactness cases, and brute force on tiny grids."""

import os

import numpy as np
import pytest

import synth
from oracle import grid as og, ops, step, diagnostics, adjoint, closed_forms as cf
from tests import _brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_value(key):
    with open(os.path.join(GOLD, "paper_values.txt")) as f:
        for line in f:
            if line.startswith(key + " "):
                return np.array([float(v) for v in line.split()[1:]])
    raise KeyError(key)


def nrm(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.fixture(scope="module")
def g1():
    return og.make_grid(1, 17, 8, 16, 8, 16)


def test_omega_unit_and_two_derivations_agree(g1):
    r, th, ph, Th, Ph = g1.mesh()
    ox, oy, oz = cf.omega(th, ph, Th, Ph)
    np.testing.assert_allclose(ox ** 2 + oy ** 2 + oz ** 2, 1.0, atol=1e-15)  # Eq. (prop1)
    # the input generator builds omega from the local frame; the oracle from Eqs. (omegax-z)
    cfg = synth.config(1)
    nodes = synth.fields.nodes(cfg)
    _, om = synth.fields._cart(nodes[0][:, None, None, None, None], nodes[1][None, :, None, None, None],
                                nodes[2][None, None, :, None, None], nodes[3][None, None, None, :, None],
                                nodes[4][None, None, None, None, :])
    for a, b in zip(om, (ox[0], oy[0], oz[0])):
        np.testing.assert_allclose(np.broadcast_to(a, np.broadcast_shapes(a.shape, b.shape)),
                                   np.broadcast_to(b, np.broadcast_shapes(a.shape, b.shape)), atol=1e-15)


def test_L_of_position_is_omega(g1):
    # L x_i = omega . grad x_i = omega_i (the Cartesian form of the operator, Eq. Tra1)
    for comp in range(3):
        F = cf.on_grid(g1, lambda x, y, z, ox, oy, oz: (x, y, z)[comp])
        want = cf.on_grid(g1, lambda x, y, z, ox, oy, oz: (ox, oy, oz)[comp])
        assert nrm(ops.apply_L(F, g1), want) <= 1e-13


def test_L_of_omega_vanishes(g1):
    # Eq. (prop2)
    for comp in range(3):
        F = cf.on_grid(g1, lambda x, y, z, ox, oy, oz: (ox, oy, oz)[comp])
        assert np.max(np.abs(ops.apply_L(F, g1))) <= 1e-13


def test_L_of_paper_uniform_distribution_vanishes(g1):
    # Eq. (propf) on the Sect. 5.2 initial distribution (without the hemisphere cut)
    c = _paper_value("uniform_test_coeffs")
    F = cf.on_grid(g1, lambda x, y, z, ox, oy, oz: (c[0] + c[1] * ox + c[2] * oy + c[3] * oz) ** 4)
    assert np.max(np.abs(ops.apply_L(F, g1))) <= 1e-12 * np.max(np.abs(F))


def test_dfs_consistency_of_generators():
    # A field consistent with the DFS identities has band-limited DFS lines: the
    # smooth random field only carries |k| <= 10 per angle, so every theta and
    # Theta DFS line (length 32 here) must have no energy above mode 10.
    cfg = synth.config(2).scaled(n_r=5, n_eps=1)
    g = og.make_grid(*cfg.shape)
    G = synth.fields.smooth_random_G(cfg)[None]
    for ext, ax in ((ops.dfs_extend_theta, 2), (ops.dfs_extend_Theta, 4)):
        spec = np.abs(np.fft.fft(ext(G, g), axis=ax))
        n = spec.shape[ax]
        k = np.abs(np.fft.fftfreq(n, 1.0 / n))
        high = np.take(spec, np.where(k > 10)[0], axis=ax)
        assert np.max(high) <= 1e-12 * np.max(spec)
    # a non-symmetrised field fails the same check (the check has teeth)
    bad = G * np.cos(g.mesh()[4])  # times cos(Phi), which flips sign under Phi -> Phi + pi
    spec = np.abs(np.fft.fft(ops.dfs_extend_Theta(bad, g), axis=4))
    assert np.max(spec[..., 12:20, :]) > 1e-3 * np.max(spec)


def test_free_streaming_exact_for_polynomials(g1):
    # F0 = P(x) Q(omega) with x-degree 2: L^3 F0 = 0, so RK4 is exact and matches
    # F0(x - t omega, omega) (straight-line propagation, Sect. 2.1).
    rng = np.random.default_rng(5)
    cx = rng.normal(size=10)
    co = rng.normal(size=4)

    def f0(x, y, z, ox, oy, oz):
        P = (cx[0] + cx[1] * x + cx[2] * y + cx[3] * z + cx[4] * x * x + cx[5] * y * y
             + cx[6] * z * z + cx[7] * x * y + cx[8] * y * z + cx[9] * x * z)
        Q = co[0] + co[1] * ox + co[2] * oy + co[3] * oz * ox
        return P * Q

    F = cf.on_grid(g1, f0)
    p = step.Physics.vacuum(g1, bc=False)
    dt = g1.dt_default()
    y = step.run(F, g1, p, dt, 10)
    want = cf.free_streaming(g1, f0, 10 * dt)
    assert nrm(y, want) <= 1e-12


def test_brute_force_operator_and_transpose():
    g = og.make_grid(1, 5, 2, 4, 2, 4)
    A = _brute.assemble(g, bc=False)
    rng = np.random.default_rng(0)
    x = rng.normal(size=g.shape)
    y = rng.normal(size=g.shape)
    np.testing.assert_allclose(-ops.apply_L(x, g).ravel(), A @ x.ravel(), atol=1e-12)
    np.testing.assert_allclose(-ops.apply_LT(y, g).ravel(), A.T @ y.ravel(), atol=1e-12)


def test_brute_force_rhs_step_and_adjoint():
    g = og.make_grid(2, 5, 2, 4, 2, 4)
    rng = np.random.default_rng(1)
    kappa, sigma, eta = (rng.uniform(0.2, 1.5, size=(2, 5, 2, 4)) for _ in range(3))
    p = step.Physics(kappa, sigma, eta, bc=True, scattering=True)
    A = _brute.assemble(g, kappa, sigma, bc=True)
    b = _brute.source(g, eta, bc=True)
    y = rng.normal(size=g.shape)
    np.testing.assert_allclose(step.rhs(y, g, p).ravel(), A @ y.ravel() + b, atol=1e-12)
    dt = 0.05
    P, Q = _brute.rk4_polys(dt * A)
    np.testing.assert_allclose(step.rk4_step(y, g, p, dt).ravel(), P @ y.ravel() + dt * Q @ b, atol=1e-12)
    lam = rng.normal(size=g.shape)
    lam_prev, gk, ge, gs = adjoint.adjoint_step(y, lam, g, p, dt)
    np.testing.assert_allclose(lam_prev.ravel(), P.T @ lam.ravel(), atol=1e-12)
    # coefficient gradients by complex-step differentiation of the brute-force step
    h = 1e-30
    for name, grad in (("kappa", gk), ("eta", ge), ("sigma", gs)):
        for q in [(0, 0, 0, 0), (1, 2, 1, 3), (0, 4, 1, 1), (1, 1, 0, 2)]:
            kc = kappa.astype(complex)
            sc = sigma.astype(complex)
            ec = eta.astype(complex)
            {"kappa": kc, "eta": ec, "sigma": sc}[name][q] += 1j * h
            Ac = _brute.assemble(g, kc, sc, bc=True, dtype=complex)
            bc_ = _brute.source(g, ec, bc=True)
            Pc, Qc = _brute.rk4_polys(dt * Ac)
            y1 = Pc @ y.ravel() + dt * Qc @ bc_
            d = np.imag(lam.ravel() @ y1) / h
            assert grad[q] == pytest.approx(d, rel=1e-11, abs=1e-13), (name, q)


def test_adjoint_dot_product_per_pass():
    g = og.make_grid(2, 7, 4, 8, 4, 8)
    rng = np.random.default_rng(2)
    x = rng.normal(size=g.shape)
    y = rng.normal(size=g.shape)
    for fwd, bwd in ((ops.d_theta, ops.d_theta_T), (ops.d_Theta, ops.d_Theta_T)):
        assert np.sum(fwd(x, g) * y) == pytest.approx(np.sum(x * bwd(y, g)), rel=1e-13)
    assert np.sum(ops.apply_L(x, g) * y) == pytest.approx(np.sum(x * ops.apply_LT(y, g)), rel=1e-13)
    m = ops.angular_mean(x, g)
    assert np.sum(np.broadcast_to(m, g.shape) * y) == pytest.approx(np.sum(x * ops.angular_mean_T(y, g)), rel=1e-13)
    kappa, sigma, eta = (rng.uniform(0.2, 1.5, size=g.shape[:4]) for _ in range(3))
    lin = lambda v: ops.rhs(v, g, kappa, sigma, 0 * eta)  # noqa: E731
    assert np.sum(lin(x) * y) == pytest.approx(np.sum(x * ops.rhs_linear_T(y, g, kappa, sigma)), rel=1e-13)


def test_scattering_quadrature_and_number_conservation(g1):
    one = np.ones(g1.shape)
    np.testing.assert_allclose(ops.angular_mean(one, g1), 1.0, atol=1e-15)
    for comp in range(3):
        F = cf.on_grid(g1, lambda x, y, z, ox, oy, oz: (ox, oy, oz)[comp])
        assert np.max(np.abs(ops.angular_mean(F, g1))) <= 1e-15
    # scattering alone conserves the particle number (detailed balance, App. A)
    cfg = synth.config(1)
    F = synth.fields.beam(cfg)
    sig = np.random.default_rng(0).uniform(0.5, 1.0, size=g1.shape[:4])
    S = np.broadcast_to(sig[..., None, None], g1.shape) * (ops.angular_mean(F, g1) - F)
    N = diagnostics.particle_number(np.abs(F), g1)
    assert abs(diagnostics.particle_number(S, g1)[0]) <= 1e-15 * N[0]


def test_conservation_law_polynomial(g1):
    # Eq. (Cons): dN/dt = -(J_R2 - J_R1) exactly when every quadrature is exact
    f0 = lambda x, y, z, ox, oy, oz: (1 + x * ox + 0.3 * y * y) * (2 + oz + 0.5 * ox * oy)  # noqa: E731
    F = cf.on_grid(g1, f0)
    dN = diagnostics.particle_number(-ops.apply_L(F, g1), g1)
    _, Jin, Jout = diagnostics.fluxes(F, g1)
    assert dN[0] == pytest.approx(-(Jout[0] - Jin[0]), rel=1e-13, abs=1e-12)


def test_conservation_over_rk4_run_beam(g1):
    # Discrete Eq. (Cons) over a run: N(t) - N(0) + sum dt sum_s b_s (J_out - J_in)(Y_s)
    # with bc off; spectrally small for the beam (report-level bound)
    cfg = synth.config(1)
    F = synth.fields.beam(cfg)
    p = step.Physics.vacuum(g1, bc=False)
    dt = g1.dt_default()
    N0 = diagnostics.particle_number(F, g1)[0]
    acc = 0.0
    y = F
    for _ in range(5):
        Ys, _ = step.rk4_stages(y, g1, p, dt)
        for b, Y in zip((1 / 6, 1 / 3, 1 / 3, 1 / 6), Ys):
            _, Jin, Jout = diagnostics.fluxes(Y, g1)
            acc += dt * b * (Jout[0] - Jin[0])
        y = step.rk4_step(y, g1, p, dt)
    res = diagnostics.particle_number(y, g1)[0] - N0 + acc
    assert abs(res) <= 1e-3 * abs(N0)


def test_uniform_isotropic_preserved():
    g = og.make_grid(2, 9, 4, 8, 4, 8)
    c = 0.7
    F = np.full(g.shape, c)
    p = step.Physics.vacuum(g, bc=True)
    y = step.run(F, g, p, 0.01, 5)
    np.testing.assert_allclose(y, c, atol=1e-14)
    rng = np.random.default_rng(0)
    kappa = rng.uniform(0.5, 2, size=g.shape[:4])
    sigma = rng.uniform(0, 1, size=g.shape[:4])
    p2 = step.Physics(kappa, sigma, kappa * c, bc=True, scattering=True)
    y = step.run(F, g, p2, 0.01, 5)
    np.testing.assert_allclose(y, c, atol=1e-14)


def test_filter_single_mode():
    # Fourier modes that are smooth on both spheres (their theta and Theta parities
    # match the DFS identities) are multiplied by exp(-36 (k / (n/2))^36) per line.
    g = og.make_grid(1, 5, 4, 16, 4, 16)
    r, th, ph, Th, Ph = g.mesh()
    s = lambda k, n: np.exp(-36.0 * (k / (n / 2.0)) ** 36)  # noqa: E731
    z = 0 * (r + th + ph + Th + Ph)
    cases = [
        (np.cos(6 * ph) + z, s(6, 16)),
        (np.cos(4 * Ph) + z, s(4, 16)),
        (np.cos(3 * th) + z, s(3, 8)),
        (np.sin(th) * np.sin(Th) * np.cos(3 * Ph) + z, s(1, 8) * s(1, 8) * s(3, 16)),
        (np.sin(th) * np.cos(7 * ph) + z, s(1, 8) * s(7, 16)),
    ]
    for F, fac in cases:
        F = np.broadcast_to(F, g.shape).copy()
        np.testing.assert_allclose(ops.apply_filter(F, g), fac * F, atol=1e-14)


def test_homogeneous_sphere_stationary_converges():
    # Formal solution I = B (1 - exp(-kappa s)) of a uniform sphere of radius 4 with
    # analytic inflow on both radial boundaries: the RHS at the analytic state is a
    # pure discretisation error and must fall with resolution.
    res = []
    for (n_r, n_a) in ((9, 8), (17, 16)):
        g = og.make_grid(1, n_r, n_a // 2, n_a, n_a // 2, n_a)
        kap, B = np.array([0.7]), np.array([1.3])
        I = cf.homogeneous_sphere(g, kap, B, 4.0)
        z = np.zeros(g.shape[:4])
        p = step.Physics(z + kap[0], z, z + kap[0] * B[0], bc=True, scattering=False)
        res.append(np.max(np.abs(step.rhs(I, g, p))) / (kap[0] * B[0]))
    assert res[1] < 0.2 * res[0]
    assert res[1] < 2e-3


def test_flux_loss_gradient_fd():
    # the loss is quadratic in F0, so central differences are exact up to rounding
    cfg = synth.config(4).scaled(n_eps=2, n_r=7, n_theta=2, n_phi=4, n_Theta=4, n_Phi=4)
    g = og.make_grid(*cfg.shape)
    kappa, sigma, eta = synth.fields.coefficients(cfg)
    p = step.Physics(kappa, sigma, eta, bc=True, scattering=False)
    F0 = synth.fields.random_state(cfg, 3)
    jt = np.random.default_rng(4).normal(size=(2, 2, 4))
    dt = 0.02
    loss, gF, gk, ge, _ = adjoint.loss_and_grads(F0, g, p, dt, 6, jt, checkpoint_every=4)
    rng = np.random.default_rng(1)
    for _ in range(3):
        d = rng.normal(size=g.shape)
        h = 1e-3
        lp = adjoint.flux_loss(step.run(F0 + h * d, g, p, dt, 6), g, jt)
        lm = adjoint.flux_loss(step.run(F0 - h * d, g, p, dt, 6), g, jt)
        assert np.sum(gF * d) == pytest.approx((lp - lm) / (2 * h), rel=1e-9)
    for _ in range(2):
        dk = rng.normal(size=kappa.shape)
        h = 1e-6
        pp = step.Physics(kappa + h * dk, sigma, eta, bc=True, scattering=False)
        pm = step.Physics(kappa - h * dk, sigma, eta, bc=True, scattering=False)
        lp = adjoint.flux_loss(step.run(F0, g, pp, dt, 6), g, jt)
        lm = adjoint.flux_loss(step.run(F0, g, pm, dt, 6), g, jt)
        assert np.sum(gk * dk) == pytest.approx((lp - lm) / (2 * h), rel=1e-6)


def test_rhs_at_matches_full(g1):
    cfg = synth.config(3).scaled(n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8)
    g = og.make_grid(*cfg.shape)
    F = synth.fields.random_state(cfg, 7)
    kappa, sigma, eta = synth.fields.random_coeffs(cfg, 8)
    full = ops.rhs(F, g, kappa, sigma, eta)
    rng = np.random.default_rng(0)
    for _ in range(20):
        idx = tuple(int(rng.integers(0, s)) for s in g.shape)
        assert ops.rhs_at(F, g, kappa, sigma, eta, idx) == pytest.approx(full[idx], rel=1e-12, abs=1e-12)
    for idx in [(0, 0, 0, 0, 0, 0), (1, 8, 3, 7, 3, 7), (0, 0, 1, 2, 3, 4)]:
        assert ops.rhs_at(F, g, kappa, sigma, eta, idx) == pytest.approx(full[idx], rel=1e-12, abs=1e-12)


def test_project_inflow_sets_only_incoming_half():
    g = og.make_grid(2, 5, 2, 4, 4, 8)
    rng = np.random.default_rng(0)
    F = rng.normal(size=g.shape)
    gi = rng.normal(size=(2, 2, 4, 4, 8))
    go = rng.normal(size=(2, 2, 4, 4, 8))
    P = ops.project_inflow(F, g, gi, go)
    cT = np.cos(g.Theta)
    for i in range(g.n_Theta):
        np.testing.assert_array_equal(P[:, 0, :, :, i], gi[:, :, :, i] if cT[i] > 0 else F[:, 0, :, :, i])
        np.testing.assert_array_equal(P[:, -1, :, :, i], go[:, :, :, i] if cT[i] < 0 else F[:, -1, :, :, i])
    np.testing.assert_array_equal(P[:, 1:-1], F[:, 1:-1])


def test_outgoing_flux_map_against_boundary_flux():
    # App. A, Eq. (Flux): for F that vanishes on the incoming half at r_out
    # (cos Theta < 0), the flux map integrated over the position sphere with the
    # same theta/phi weights is J_out / R2^2.  A map over the wrong hemisphere
    # gives 0, one without the cos Theta weight a different sum.
    g = og.make_grid(2, 7, 4, 8, 6, 12)
    rng = np.random.default_rng(21)
    F = rng.normal(size=g.shape)
    cT = np.cos(g.Theta)
    F[:, -1][:, :, :, cT < 0] = 0.0
    j = diagnostics.outgoing_flux_map(F, g)
    w_pos = g.w_theta[:, None] * np.full(g.n_phi, 2.0 * np.pi / g.n_phi)[None, :]
    J_out = diagnostics.boundary_flux(F, g, g.n_r - 1)
    got = np.sum(j * w_pos[None], axis=(1, 2))
    np.testing.assert_allclose(got, J_out / g.r_out ** 2, rtol=1e-13)


def test_outgoing_flux_map_closed_form():
    # F = cos(Theta) g(theta, phi) at r_out: the half-range sum of w_i cos^2 Theta_i
    # is half the full one (the half-shifted nodes are symmetric about pi/2), and
    # Fejer's rule integrates mu^2 exactly: (1/2)(2/3); the trapezoid sum over Phi
    # gives 2 pi.  So j = (2 pi / 3) g(theta, phi) for every position node.
    g = og.make_grid(1, 5, 4, 8, 8, 16)
    r, th, ph, Th, Ph = g.mesh()
    gpos = 1.0 + 0.3 * np.cos(th) + 0.2 * np.sin(th) * np.sin(ph)
    F = np.broadcast_to(np.cos(Th) * gpos + 0.0 * Ph + 0.0 * r, g.shape).copy()
    j = diagnostics.outgoing_flux_map(F, g)
    want = (2.0 * np.pi / 3.0) * np.broadcast_to(gpos, (1, 1, g.n_theta, g.n_phi, 1, 1))[:, 0, :, :, 0, 0]
    np.testing.assert_allclose(j, want, rtol=1e-14)
    # the transpose is exact against the map (dot-product test)
    jbar = np.random.default_rng(3).normal(size=j.shape)
    X = np.random.default_rng(4).normal(size=g.shape)
    assert np.sum(diagnostics.outgoing_flux_map(X, g) * jbar) == pytest.approx(
        np.sum(X * diagnostics.outgoing_flux_map_T(jbar, g)), rel=1e-13)


def test_L_angular_of_paper_uniform_distribution_vanishes(g1):
    # Eq. (propf): F(omega) does not depend on position, so L F = 0 and, as F has
    # no r dependence in these coordinates, the angular part alone vanishes too.
    c = _paper_value("uniform_test_coeffs")
    F = cf.on_grid(g1, lambda x, y, z, ox, oy, oz: (c[0] + c[1] * ox + c[2] * oy + c[3] * oz) ** 4)
    assert np.max(np.abs(ops.apply_L_angular(F, g1))) <= 1e-12 * np.max(np.abs(F))


def test_L_angular_plus_radial_is_L():
    # on unstructured data: the angular part plus cos(Theta) D_r F is the whole
    # operator of Eq. (Liouvsph) (pinned above by Eqs. prop1/prop2/propf and
    # brute force); and for F = x_i (no omega dependence) the angular part is
    # omega_i - cos(Theta) dx_i/dr
    g = og.make_grid(2, 9, 4, 8, 4, 8)
    F = np.random.default_rng(22).normal(size=g.shape)
    c_r = ops.liouville_coefficients(g)[0]
    np.testing.assert_allclose(ops.apply_L_angular(F, g) + c_r * ops.d_r(F, g), ops.apply_L(F, g),
                               rtol=0, atol=1e-12 * np.max(np.abs(ops.apply_L(F, g))))
    gq = og.make_grid(1, 9, 8, 16, 8, 16)
    r, th, ph, Th, Ph = gq.mesh()
    for comp in range(3):
        F = cf.on_grid(gq, lambda x, y, z, ox, oy, oz: (x, y, z)[comp])
        om = cf.on_grid(gq, lambda x, y, z, ox, oy, oz: (ox, oy, oz)[comp])
        # d x_i / dr = x_i / r on the ray of fixed (theta, phi)
        want = om - np.cos(Th) * F / r
        assert nrm(ops.apply_L_angular(F, gq), want) <= 1e-13


def test_free_streaming_shell_brute_force():
    # the inside/outside decision of the shell closed form against a brute-force
    # walk along each backward segment (2001 points)
    g = og.make_grid(1, 5, 4, 8, 4, 8)
    t = 0.9
    one = lambda x, y, z, ox, oy, oz: 1.0 + 0.0 * (x + ox)  # noqa: E731
    got = cf.free_streaming_shell(g, one, t)
    r, th, ph, Th, Ph = g.mesh()
    X = np.broadcast_arrays(*cf.position(r, th, ph))
    O = np.broadcast_arrays(*cf.omega(th, ph, Th, Ph))
    shp = np.broadcast_shapes(X[0].shape, O[0].shape)
    X = [np.broadcast_to(a, shp) for a in X]
    O = [np.broadcast_to(a, shp) for a in O]
    inside = np.ones(shp, bool)
    for s in np.linspace(0.0, t, 2001):
        rr = np.sqrt(sum((X[a] - s * O[a]) ** 2 for a in range(3)))
        inside &= (rr >= g.r_in - 1e-12) & (rr <= g.r_out + 1e-12)
    np.testing.assert_array_equal(got[0], np.where(inside, 1.0, 0.0)[0])
    assert 0.2 < inside.mean() < 0.9  # both outcomes occur


def test_config1_closed_form_report():
    # Config 1 as specified (zero inflow, 10 steps): the oracle against
    # F0(x - t omega, omega) in the shell.  Resolution limited (17 x 8 x 16 x 8 x 16
    # for a w = 0.5 beam with a C^3 lobe): a report with a loose bound.
    cfg = synth.config(1)
    g = og.make_grid(*cfg.shape)
    f0 = synth.fields.beam_function(cfg)
    F = ops.project_inflow(synth.fields.beam(cfg), g)
    y = step.run(F, g, step.Physics.vacuum(g), cfg.dt, cfg.steps)
    want = cf.free_streaming_shell(g, f0, cfg.steps * cfg.dt)
    mr = nrm(y, want)
    l2 = np.linalg.norm((y - want).ravel()) / np.linalg.norm(want.ravel())
    print(f"config 1 oracle vs closed form after {cfg.steps} steps: max-rel {mr:.3e} L2-rel {l2:.3e}")
    assert l2 < 0.15 and mr < 0.3


def test_flux_forms_are_the_same_operator():
    # Eq. (Cohercons) is the transport equation times V: on data the grid
    # represents exactly (x-degree 2, angular degree 2), the flux form of every
    # term and the hybrid form equal Eq. (Liouvsph)
    from oracle import conservative as cons
    F = synth.fields.polynomial_state(synth.config(1).scaled(n_r=9), seed=3, deg_x=2, deg_om=2)
    g = og.make_grid(*F.shape)
    L = ops.apply_L(F, g)
    assert nrm(cons.apply_L_hybrid(F, g), L) <= 1e-12
    assert nrm(cons.apply_L_flux(F, g), L) <= 1e-12


def test_flux_form_radial_phi_Phi_balance_exactly():
    # the parts of the flux form that cancel for any nodal data: the sum of
    # D_r(cos Theta F^) with Clenshaw-Curtis weights is the boundary difference of
    # cos Theta F^ (the quadrature is exact on the derivative of the interpolant);
    # Fourier derivatives along phi and Phi sum to zero over a period
    g = og.make_grid(1, 9, 4, 8, 4, 8)
    X = np.random.default_rng(23).normal(size=g.shape)
    cT = np.cos(g.mesh()[3])
    rsum = np.tensordot(g.w_r, ops.d_r(cT * X, g), axes=([0], [1]))
    np.testing.assert_allclose(rsum, (cT * X)[:, -1] - (cT * X)[:, 0], atol=1e-12)
    assert np.max(np.abs(ops.d_phi(X, g).sum(axis=3))) <= 1e-12
    assert np.max(np.abs(ops.d_Phi(X, g).sum(axis=5))) <= 1e-12


def test_conservation_residual_of_the_three_forms():
    # Eq. (Cons) at one instant on the workload-1 beam (no inflow mask): the
    # residual dN/dt + J_R2 - J_R1 relative to |J_R2| + |J_R1| for Eq. (Liouvsph)
    # as built, the full flux form of Eq. (Cohercons) and the hybrid (radial and
    # Phi terms in flux form).  Measured on this grid (17 x 8 x 16 x 8 x 16):
    # 5.40e-3, 3.78e-2 and 5.40e-3.  The hybrid equals the form as built to
    # rounding: Clenshaw-Curtis integrates the radial terms of both exactly (the
    # interpolant's r^2 p' + 2 r p has degree n_r, one more than the rule's
    # guaranteed n_r - 1, but the symmetric rule is exact there too) and the
    # trapezoid rule the Phi terms, so the whole residual comes from the theta and
    # Theta DFS lines.  The full flux form is worse there: the theta line of
    # F^ = V F is odd across the pole.  Neither form is built on the GPU.
    from oracle import conservative as cons
    cfg = synth.config(1)
    g = og.make_grid(*cfg.shape)
    F = synth.fields.beam(cfg)
    res = {}
    for name, fn in (("liouvsph", ops.apply_L), ("flux", cons.apply_L_flux), ("hybrid", cons.apply_L_hybrid)):
        r, s = cons.conservation_residual(fn(F, g), F, g)
        res[name] = float(abs(r[0]) / s[0])
    print("Eq. (Cons) relative residual on the beam: " + ", ".join(f"{k} {v:.2e}" for k, v in res.items()))
    assert 4e-3 < res["liouvsph"] < 7e-3
    assert abs(res["hybrid"] - res["liouvsph"]) <= 1e-10
    assert res["flux"] > 5 * res["liouvsph"]
