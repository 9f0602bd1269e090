"""Oracle discrete adjoint of the RK4 step, and the outgoing-flux misfit loss.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The right-hand side is affine in F: rhs(Y) = A Y + M eta with
A = M (-L - (kappa + sigma) I + sigma K), M the inflow mask and K the
in-scattering operator (the broadcast angular mean for isotropic scattering).  For y1 = y + dt/6 (k1 + 2 k2 + 2 k3 + k4) with
k_s = rhs(Y_s), the exact transpose of the step is (lam = dLoss/dy1):

    kb4 = dt/6 lam
    kb3 = dt/3 lam + dt   A^T kb4
    kb2 = dt/3 lam + dt/2 A^T kb3
    kb1 = dt/6 lam + dt/2 A^T kb2
    dLoss/dy = lam + sum_s A^T kb_s

and the coefficient gradients are sum_s (d rhs(Y_s) / d coeff)^T kb_s, which need
the stage inputs Y_s (recomputed from y).  With the energy coupling on the
right-hand side is no longer affine: A^T is then the transpose of its Jacobian
at each stage input, A^T + (M sigma S'(Y_s))^T (energy.fp_rhs_T), and sigma's
gradient gains S(Y_s) summed against M kb_s.  With the filter on, lam is first
set to zero at the inflow nodes (when the inflow conditions are on: the step
re-imposes the inflow values after the filter) and mapped by the filter's
transpose (the angular line filters are symmetric, the radial one is not).
"""

import numpy as np

from . import energy, ops, step, diagnostics


def adjoint_step(y, lam, g, p, dt):
    """One adjoint RK4 step.

    y: the state at the start of the step; lam: dLoss/dy_{n+1}.
    Returns (dLoss/dy_n, grad_kappa, grad_eta, grad_sigma), the gradients as
    [eps][r][theta][phi] arrays for this step only.
    """
    if p.radial_implicit:
        raise NotImplementedError("no adjoint of the radially implicit split step")
    if p.filt:
        # the filter step is y -> (I - P) Filter y + P g (P: the inflow nodes), whose
        # linear part transposes to Filter^T (I - P)
        if p.bc:
            lam = lam * ops.inflow_mask(g)
        lam = ops.apply_filter_T(lam, g, radial=p.filt_r)
    (Y1, Y2, Y3, Y4), _ = step.rk4_stages(y, g, p, dt)
    s_eff = p.sigma if p.scattering else np.zeros_like(np.asarray(p.sigma, np.float64))

    def AT(x, Ys):
        # the transpose of the right-hand side's Jacobian at the stage input Ys
        out = ops.rhs_linear_T(x, g, p.kappa, p.sigma, bc=p.bc, scattering=p.scattering, kernel=p.kernel)
        if p.energy is not None:
            out = out + energy.fp_rhs_T(Ys, x, g, s_eff, *p.energy, bc=p.bc)
        return out

    kb4 = (dt / 6.0) * lam
    a4 = AT(kb4, Y4)
    kb3 = (dt / 3.0) * lam + dt * a4
    a3 = AT(kb3, Y3)
    kb2 = (dt / 3.0) * lam + 0.5 * dt * a3
    a2 = AT(kb2, Y2)
    kb1 = (dt / 6.0) * lam + 0.5 * dt * a2
    a1 = AT(kb1, Y1)
    lam_prev = lam + a1 + a2 + a3 + a4

    M = ops.inflow_mask(g) if p.bc else 1.0
    gk = np.zeros((g.n_eps, g.n_r, g.n_theta, g.n_phi))
    ge = np.zeros_like(gk)
    gs = np.zeros_like(gk)
    for Ys, kb in ((Y1, kb1), (Y2, kb2), (Y3, kb3), (Y4, kb4)):
        mk = M * kb
        gk -= np.sum(mk * Ys, axis=(4, 5))
        ge += np.sum(mk, axis=(4, 5))
        if p.scattering:
            gs += np.sum(mk * (ops.scatter_in(Ys, g, p.kernel) - Ys), axis=(4, 5))
            if p.energy is not None:
                # the coupling's source is sigma S(Ys)
                gs += np.sum(mk, axis=(4, 5)) * energy.fp_source(Ys, g, np.ones(gs.shape), *p.energy)
    return lam_prev, gk, ge, gs


def flux_loss(F, g, j_target):
    """Squared misfit of the outgoing-flux map: sum (j - j*)^2 (no 1/2, no area
    weights)."""
    d = diagnostics.outgoing_flux_map(F, g) - j_target
    return float(np.sum(d * d))


def flux_loss_grad_F(F, g, j_target):
    d = diagnostics.outgoing_flux_map(F, g) - j_target
    return diagnostics.outgoing_flux_map_T(2.0 * d, g)


def loss_and_grads(F0, g, p, dt, n_steps, j_target, checkpoint_every=None):
    """Run n_steps forward, evaluate the flux loss, and back-propagate with the
    discrete adjoint.  States are kept every checkpoint_every steps and the
    steps in between are recomputed on the way back.

    Returns (loss, dLoss/dF0, dLoss/dkappa, dLoss/deta, dLoss/dsigma)."""
    K = checkpoint_every or n_steps
    ckpt = {0: F0}
    y = F0
    for n in range(n_steps):
        y = step.rk4_step(y, g, p, dt)
        if (n + 1) % K == 0 and n + 1 < n_steps:
            ckpt[n + 1] = y
    loss = flux_loss(y, g, j_target)
    lam = flux_loss_grad_F(y, g, j_target)
    gk = np.zeros((g.n_eps, g.n_r, g.n_theta, g.n_phi))
    ge = np.zeros_like(gk)
    gs = np.zeros_like(gk)
    seg_starts = sorted(ckpt)
    for s0 in reversed(seg_starts):
        s1 = min(s0 + K, n_steps)
        states = [ckpt[s0]]
        for _ in range(s0, s1 - 1):
            states.append(step.rk4_step(states[-1], g, p, dt))
        for yn in reversed(states):
            lam, a, b, c = adjoint_step(yn, lam, g, p, dt)
            gk += a
            ge += b
            gs += c
    return loss, lam, gk, ge, gs
