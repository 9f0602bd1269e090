"""Differentiable transport: gradients of the outgoing-flux misfit with respect to
the opacity field kappa_s(r, theta, phi) and the initial state, through
TransportRK4 (checkpoint every K steps, recompute, discrete adjoint on the GPU).

Parameterisation (workload 4): kappa = kappa0 (eps/10)^2 kappa_s, eta = kappa B(eps,
T0/r), sigma = 0; loss = sum (j - j*)^2 with j the outgoing-flux map at r_out.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og, step, adjoint
from tests.gpu_util import need_gpu, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def factors(cfg):
    """c_eps [eps] and B [eps][r][theta][phi] with kappa = c_eps kappa_s, eta = kappa B."""
    shp = (cfg.n_r, cfg.n_theta, cfg.n_phi)
    kappa, _, eta = synth.fields.coefficients(cfg, kappa_s=np.ones(shp))
    c_eps = kappa[:, 0, 0, 0].copy()
    return c_eps, eta / kappa


def base_kappa_s(cfg):
    r = synth.fields.nodes(cfg)[0]
    return np.ascontiguousarray(np.broadcast_to((r ** -2.0)[:, None, None], (cfg.n_r, cfg.n_theta, cfg.n_phi)))


class Model:
    def __init__(self, cfg, K):
        from paper_1104_5330_amd import Sp6Grid
        self.cfg, self.K = cfg, K
        self.G = Sp6Grid.from_config(cfg, scattering=False)
        c_eps, B = factors(cfg)
        dev = torch.device("cuda")
        self.c = torch.as_tensor(c_eps, device=dev).view(-1, 1, 1, 1)
        self.B = torch.as_tensor(B, device=dev)

    def loss(self, kappa_s, F0, jt, n):
        from paper_1104_5330_amd.autograd import transport, outgoing_flux
        kappa = self.c * kappa_s.unsqueeze(0)
        eta = kappa * self.B
        sigma = torch.zeros_like(kappa)
        F = transport(self.G, F0, kappa, sigma, eta, self.cfg.dt, n, self.K)
        j = outgoing_flux(self.G, F)
        return ((j - jt) ** 2).sum()


def test_autograd_matches_oracle_adjoint():
    cfg = synth.config(4).scaled(n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8)
    n, K = 20, 5
    dev = torch.device("cuda")
    m = Model(cfg, K)
    ks = base_kappa_s(cfg)
    F0 = synth.fields.shell_state(cfg)
    jt = np.random.default_rng(3).normal(size=(cfg.n_eps, cfg.n_theta, cfg.n_phi)) * 0.01
    kst = torch.tensor(ks, device=dev, requires_grad=True)
    F0t = torch.tensor(F0, device=dev, requires_grad=True)
    L = m.loss(kst, F0t, torch.as_tensor(jt, device=dev), n)
    L.backward()
    # oracle: discrete adjoint with the same checkpointing, chained to kappa_s by hand
    g = og.make_grid(*cfg.shape)
    c_eps, B = factors(cfg)
    kappa = c_eps[:, None, None, None] * ks[None]
    p = step.Physics(kappa, np.zeros_like(kappa), kappa * B, scattering=False)
    loss, gF, gk, ge, _ = adjoint.loss_and_grads(F0, g, p, cfg.dt, n, jt, checkpoint_every=K)
    gks = np.sum(c_eps[:, None, None, None] * (gk + ge * B), axis=0)
    e_loss = abs(L.item() - loss) / abs(loss)
    e_F = np.max(np.abs(F0t.grad.cpu().numpy() - gF)) / np.max(np.abs(gF))
    e_k = np.max(np.abs(kst.grad.cpu().numpy() - gks)) / np.max(np.abs(gks))
    banner(f"autograd vs oracle adjoint: loss {e_loss:.1e}, dF0 {e_F:.1e}, dkappa_s {e_k:.1e}")
    assert e_loss <= 1e-12 and e_F <= 1e-10 and e_k <= 1e-10


def test_workload4_gradient_vs_finite_differences():
    cfg = synth.config(4)
    n, K = cfg.steps, 20
    dev = torch.device("cuda")
    m = Model(cfg, K)
    ks = torch.as_tensor(base_kappa_s(cfg), device=dev)
    rho = torch.as_tensor(synth.fields.low_mode_position_field(cfg, seed=0), device=dev)
    F0 = synth.fields.shell_state(cfg, device=dev)
    with torch.no_grad():
        from paper_1104_5330_amd.autograd import transport, outgoing_flux
        ks_star = ks * (1.0 + 0.2 * rho)
        kap = m.c * ks_star.unsqueeze(0)
        jt = outgoing_flux(m.G, transport(m.G, F0, kap, torch.zeros_like(kap), kap * m.B, cfg.dt, n, K)).clone()
    kst = ks.clone().requires_grad_(True)
    F0t = F0.clone().requires_grad_(True)
    L = m.loss(kst, F0t, jt, n)
    L.backward()
    gk, gF = kst.grad.detach(), F0t.grad.detach()
    rng = np.random.default_rng(1)
    hk = 1e-5 * ks.abs().max().item()
    hF = 1e-5 * F0.abs().max().item()
    worst = 0.0
    with torch.no_grad():
        for it in range(16):
            # each block normalised to unit max-norm, so that h is the largest
            # perturbation of any entry: 1e-5 of that block's largest value
            dk = torch.as_tensor(rng.normal(size=ks.shape), device=dev)
            dk /= dk.abs().max()
            dF = torch.as_tensor(rng.normal(size=F0.shape), device=dev)
            dF /= dF.abs().max()
            Lp = m.loss(ks + hk * dk, F0 + hF * dF, jt, n).item()
            Lm = m.loss(ks - hk * dk, F0 - hF * dF, jt, n).item()
            fd = (Lp - Lm) / 2.0
            pred = hk * torch.sum(gk * dk).item() + hF * torch.sum(gF * dF).item()
            rel = abs(pred - fd) / max(abs(fd), 1e-30)
            worst = max(worst, rel)
            print(f"[gpu-test] direction {it}: adjoint {pred:.10e} fd {fd:.10e} rel {rel:.2e}", flush=True)
    banner(f"workload 4 ({n} steps, checkpoint {K}): worst |adjoint - FD| / |FD| = {worst:.2e}")
    assert worst <= 1e-6


@pytest.mark.parametrize("filt", [0, 2])
def test_stored_stages_match_recomputed(filt):
    # sp6_step_stages advances F exactly as sp6_step and its stages are the RK4
    # stage inputs; the adjoint step reading them equals the one recomputing them
    from paper_1104_5330_amd import Sp6Grid
    cfg = synth.config(3).scaled(n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8)
    G = Sp6Grid.from_config(cfg, filter=filt)
    rng = np.random.default_rng(5)
    F = synth.fields.random_state(cfg, 5)
    k, s, e = synth.fields.random_coeffs(cfg, 6)
    dev = torch.device("cuda")
    G.set_coefficients(*(torch.as_tensor(a, device=dev) for a in (k, s, e)))
    Fa = torch.as_tensor(F, device=dev)
    Fb = Fa.clone()
    Ys = torch.empty((3,) + cfg.shape, dtype=torch.float64, device=dev)
    G.step(Fa, cfg.dt, 1)
    G.step_stages(Fb, cfg.dt, Ys)
    assert torch.equal(Fa, Fb)
    g = og.make_grid(*cfg.shape)
    p = step.Physics(k, s, e, filt=bool(filt), filt_r=filt == 2)
    Y_or, _ = step.rk4_stages(F, g, p, cfg.dt)
    for i in range(3):
        want = Y_or[i + 1]
        err = np.max(np.abs(Ys[i].cpu().numpy() - want)) / np.max(np.abs(want))
        assert err <= 1e-12, (i, err)
    lam = torch.as_tensor(rng.normal(size=cfg.shape), device=dev)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device=dev)
    la, lb = lam.clone(), lam.clone()
    ga = [z.clone() for _ in range(3)]
    gb = [z.clone() for _ in range(3)]
    F0 = torch.as_tensor(F, device=dev)
    G.adjoint_step(F0, cfg.dt, la, *ga)
    G.adjoint_step_stages(F0, Ys, cfg.dt, lb, *gb)
    assert torch.equal(la, lb)
    for x, y in zip(ga, gb):
        assert torch.equal(x, y)


def test_autograd_keep_stages_is_the_same():
    from paper_1104_5330_amd.autograd import transport, outgoing_flux
    cfg = synth.config(4).scaled(n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8)
    m = Model(cfg, 4)
    dev = torch.device("cuda")
    ks = torch.tensor(base_kappa_s(cfg), device=dev)
    F0 = torch.tensor(synth.fields.shell_state(cfg), device=dev)
    grads = []
    for keep in (True, False):
        kst = ks.clone().requires_grad_(True)
        F0t = F0.clone().requires_grad_(True)
        kappa = m.c * kst.unsqueeze(0)
        F = transport(m.G, F0t, kappa, torch.zeros_like(kappa), kappa * m.B, cfg.dt, 10, 4, keep_stages=keep)
        L = (outgoing_flux(m.G, F) ** 2).sum()
        L.backward()
        grads.append((kst.grad.clone(), F0t.grad.clone()))
    assert torch.equal(grads[0][0], grads[1][0])
    assert torch.equal(grads[0][1], grads[1][1])
