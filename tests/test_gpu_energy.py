"""Fokker-Planck energy coupling on the GPU (sp6_set_energy_coupling; Sect. 3.2,
Eq. Transpfp) against the FP64 oracle (oracle/energy.py): right-hand sides and
RK4 steps element by element at 1e-12 on every plane kernel (2 x 4, 16 x 32 and
32 x 64 planes) with the isotropic and the Thomson phase function, the split
step, Adams-Bashforth, the step without allocation, the adjoint step and its
gradients, the mixed path (at its stated bounds), the refusals, and at full
angular size a property that holds at any size: a homogeneous isotropic Bose
distribution (Eq. Bose) is steady to the accuracy of the energy collocation."""

import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import energy, grid as og, step
from tests.gpu_util import need_gpu, maxrel, to_dev, to_host, oracle_grid, small, banner, stable_dt

pytestmark = pytest.mark.gpu

TOL = 1e-12
GAMMA = (0.0, 1.0, 0.05)  # gamma_min, gamma_max, alpha
THOMSON = (0.0, 0.75)

SHAPES = {
    "tiny": small(3, n_eps=4, n_r=5, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4),
    "planes16": small(3, n_eps=6, n_r=5, n_theta=4, n_phi=8, n_Theta=16, n_Phi=32),
    "planes32": small(3, n_eps=3, n_r=3, n_theta=2, n_phi=4, n_Theta=32, n_Phi=64),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def setup(cfg, kernel, seed=0, energy_on=True):
    from paper_1104_5330_amd import Sp6Grid
    G = Sp6Grid.from_config(cfg, scattering=True)
    if kernel is not None:
        G.set_scattering_kernel(*kernel)
    F = synth.fields.random_state(cfg, seed)
    k, s, e = synth.fields.random_coeffs(cfg, seed + 1)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    if energy_on:
        G.set_energy_coupling(*GAMMA)
    p = step.Physics(k, s, e, bc=True, scattering=True, kernel=kernel, energy=GAMMA if energy_on else None)
    return G, F, p


@pytest.mark.parametrize("kernel", [None, THOMSON], ids=["isotropic", "thomson"])
@pytest.mark.parametrize("name", list(SHAPES))
def test_rhs(name, kernel):
    cfg = SHAPES[name]
    G, F, p = setup(cfg, kernel, seed=3)
    g = oracle_grid(cfg)
    got = to_host(G.rhs(to_dev(F)))
    want = step.rhs(F, g, p)
    err = maxrel(got, want)
    banner(f"energy rhs {name} {kernel}: max-rel {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("name", list(SHAPES))
def test_steps(name):
    cfg = SHAPES[name]
    G, F, p = setup(cfg, THOMSON, seed=5)
    g = oracle_grid(cfg)
    dt = 0.25 * stable_dt(cfg)
    want = step.run(F, g, p, dt, 3)
    Fd = to_dev(F)
    G.step(Fd, dt, 3)
    err = maxrel(to_host(Fd), want)
    banner(f"energy steps {name}: max-rel {err:.2e}")
    assert err <= TOL


def test_split_step_and_noalloc():
    cfg = SHAPES["planes16"]
    G, F, p = setup(cfg, THOMSON, seed=7)
    g = oracle_grid(cfg)
    dt = 0.25 * stable_dt(cfg)
    p.radial_implicit = True
    want = step.run(F, g, p, dt, 2)
    Fd = to_dev(F)
    G.step_radial_implicit(Fd, dt, 2)
    assert maxrel(to_host(Fd), want) <= TOL
    A, B = to_dev(F), to_dev(F)
    G.step(A, dt, 2)
    G.step_noalloc(B, dt, 2)
    torch.cuda.synchronize()
    assert torch.equal(A, B)


def test_adams_bashforth():
    cfg = SHAPES["planes16"]
    G, F, p = setup(cfg, THOMSON, seed=11)
    g = oracle_grid(cfg)
    dt = 0.25 * stable_dt(cfg)
    want, _ = step.ab2_run(F, g, p, dt, 3)
    Fd, H = to_dev(F), torch.empty(cfg.shape, dtype=torch.float64, device="cuda")
    G.step_ab2(Fd, H, dt, 3, start=True)
    err = maxrel(to_host(Fd), want)
    banner(f"energy AB2 planes16: max-rel {err:.2e}")
    assert err <= TOL


def test_mixed_path():
    """FP32 line passes and split-bf16 radial matrix, the source formed in FP64
    from the FP32 stage copies: within the mixed path's stated bounds (operator
    level 2e-5 per 32 points of the longest line, steps 1e-5)."""
    from paper_1104_5330_amd import Sp6Grid
    cfg = SHAPES["planes16"]
    G = Sp6Grid.from_config(cfg, scattering=True, precision="mixed")
    G.set_scattering_kernel(*THOMSON)
    F = synth.fields.shell_state(cfg)
    k, s, e = synth.fields.random_coeffs(cfg, 12)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    G.set_energy_coupling(*GAMMA)
    p = step.Physics(k, s, e, bc=True, scattering=True, kernel=THOMSON, energy=GAMMA)
    g = oracle_grid(cfg)
    op = 2e-5 * max(cfg.n_phi, 2 * cfg.n_theta, cfg.n_Phi, 2 * cfg.n_Theta, 32) / 32
    err_rhs = maxrel(to_host(G.rhs(to_dev(F))), step.rhs(F, g, p))
    dt = 0.25 * stable_dt(cfg)
    Fd = to_dev(F)
    G.step(Fd, dt, 3)
    err_step = maxrel(to_host(Fd), step.run(F, g, p, dt, 3))
    banner(f"energy mixed planes16: rhs max-rel {err_rhs:.2e}, 3 steps max-rel {err_step:.2e}")
    assert err_rhs <= op
    assert err_step <= 1e-5
    G.close()


@pytest.mark.parametrize("name", list(SHAPES))
def test_adjoint_step(name):
    """The adjoint RK4 step with the coupling (the transpose of the step's
    linearisation at its stage inputs) and the kappa, eta, sigma gradients against
    the oracle, with the stage inputs recomputed and with them stored."""
    from oracle import adjoint
    cfg = SHAPES[name]
    G, F, p = setup(cfg, THOMSON, seed=13)
    g = oracle_grid(cfg)
    dt = 0.25 * stable_dt(cfg)
    lam = synth.fields.random_state(cfg, 14)
    lam_prev, gk, ge, gs = adjoint.adjoint_step(F, lam, g, p, dt)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device="cuda")
    for stored in (False, True):
        lam_d, gkd, ged, gsd = to_dev(lam), z.clone(), z.clone(), z.clone()
        if stored:
            Ys = torch.empty((3,) + cfg.shape, dtype=torch.float64, device="cuda")
            G.step_stages(to_dev(F), dt, Ys)
            G.adjoint_step_stages(to_dev(F), Ys, dt, lam_d, gkd, ged, gsd)
        else:
            G.adjoint_step(to_dev(F), dt, lam_d, gkd, ged, gsd)
        errs = [maxrel(to_host(lam_d), lam_prev), maxrel(to_host(gkd), gk), maxrel(to_host(ged), ge),
                maxrel(to_host(gsd), gs)]
        banner(f"energy adjoint {name} stored={stored}: lam {errs[0]:.2e} gk {errs[1]:.2e} ge {errs[2]:.2e} "
               f"gs {errs[3]:.2e}")
        assert errs[0] <= TOL and max(errs[1:]) <= 1e-11


def test_refusals_and_switching_off():
    from paper_1104_5330_amd import Sp6Grid, _lib
    cfg = SHAPES["tiny"]
    G, F, _ = setup(cfg, None, seed=9, energy_on=False)
    lib, h = G.lib, G._h
    Fd = to_dev(F)
    plain = G.rhs(Fd).clone()
    call = lambda *a: lib.sp6_set_energy_coupling(h, ctypes.c_int32(1), *(ctypes.c_double(v) for v in a))
    assert call(1.0, 1.0, 0.1) == _lib.SP6_ERR_ARG
    assert call(-0.5, 1.0, 0.1) == _lib.SP6_ERR_ARG
    assert call(0.0, 1.0, -0.1) == _lib.SP6_ERR_ARG
    assert call(0.0, float("inf"), 0.1) == _lib.SP6_ERR_ARG
    G.set_energy_coupling(*GAMMA)
    on = G.rhs(Fd).clone()
    assert not torch.equal(on, plain)
    G.set_energy_coupling(enable=False)
    off = G.rhs(Fd)
    torch.cuda.synchronize()
    assert torch.equal(off, plain)
    G.close()
    # handles that cannot take it
    H2 = Sp6Grid.from_config(cfg, scattering=False)
    st = H2.lib.sp6_set_energy_coupling(H2._h, ctypes.c_int32(1), ctypes.c_double(0.0), ctypes.c_double(1.0),
                                        ctypes.c_double(0.1))
    assert st == _lib.SP6_ERR_STATE
    H2.close()
    one = Sp6Grid.from_config(small(3, n_eps=1, n_r=5, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4))
    st = one.lib.sp6_set_energy_coupling(one._h, ctypes.c_int32(1), ctypes.c_double(0.0), ctypes.c_double(1.0),
                                         ctypes.c_double(0.1))
    assert st == _lib.SP6_ERR_SHAPE
    one.close()


def test_bose_distribution_is_steady_full_angular_size():
    """Workload 2's spatial and angular grid (33 x 16 x 32 x 16 x 32) with 32
    energy nodes: a homogeneous isotropic Bose distribution, Thomson scattering,
    no absorption or emission.  Streaming and scattering leave it unchanged and
    the energy flux vanishes, so the right-hand side is zero up to the energy
    collocation error (the oracle's own Bose test: 4e-11 of the drift term)."""
    from paper_1104_5330_amd import Sp6Grid
    n, (gmin, gmax, alpha, mu) = 32, (0.0, 2.0, 0.2, -1.0)
    cfg = small(2, n_eps=n)
    gam = energy.energy_nodes(n, gmin, gmax)
    bose = 2.0 * gam * gam / np.expm1((gam - mu) / alpha)
    D = og.cheb_diff_matrix(n, gmin, gmax)
    scale = np.max(np.abs(D @ (gam * gam * bose)))
    G = Sp6Grid.from_config(cfg, scattering=True)
    G.set_scattering_kernel(*THOMSON)
    shp = (cfg.n_eps, cfg.n_r, cfg.n_theta, cfg.n_phi)
    z = torch.zeros(shp, dtype=torch.float64, device="cuda")
    G.set_coefficients(z, z + 1.0, z)
    G.set_energy_coupling(gmin, gmax, alpha)
    F = torch.as_tensor(bose, device="cuda").view(-1, 1, 1, 1, 1, 1).expand(cfg.shape).contiguous()
    G.set_inflow(F[:, 0].contiguous(), F[:, -1].contiguous())
    r = G.rhs(F)
    torch.cuda.synchronize()
    rel = float(r.abs().max()) / scale
    banner(f"Bose state on {cfg.shape}: max |rhs| / drift scale = {rel:.2e}")
    assert rel <= 1e-9
    G.close()


def test_autograd_through_the_coupled_step_vs_finite_differences():
    """torch.autograd through 12 coupled RK4 steps (checkpoints every 5, stage
    inputs kept): the gradient of an outgoing-flux misfit with respect to the
    initial state, kappa and sigma against central differences along 8 random
    joint directions, each block scaled to unit max-norm and stepped by 1e-5 of
    its largest value."""
    from paper_1104_5330_amd.autograd import transport, outgoing_flux
    cfg = SHAPES["planes16"]
    G, _, _ = setup(cfg, THOMSON, seed=15)
    dev = torch.device("cuda")
    F0 = 0.3 * synth.fields.shell_state(cfg, device=dev)
    k, s, e = (to_dev(a) for a in synth.fields.random_coeffs(cfg, 16))
    dt, n, K = 0.25 * stable_dt(cfg), 12, 5
    with torch.no_grad():
        jt = 0.9 * outgoing_flux(G, transport(G, F0, k, s, e, dt, n, K)).clone()

    def loss(F, kk, ss):
        return ((outgoing_flux(G, transport(G, F, kk, ss, e, dt, n, K)) - jt) ** 2).sum()

    Ft, kt, st = (x.clone().requires_grad_(True) for x in (F0, k, s))
    L = loss(Ft, kt, st)
    L.backward()
    rng = np.random.default_rng(17)
    worst = 0.0
    with torch.no_grad():
        for it in range(8):
            dirs = []
            for x in (F0, k, s):
                dx = torch.as_tensor(rng.normal(size=x.shape), device=dev)
                dirs.append((dx / dx.abs().max(), 1e-5 * x.abs().max().item()))
            (dF, hF), (dk, hk), (ds, hs) = dirs
            Lp = loss(F0 + hF * dF, k + hk * dk, s + hs * ds).item()
            Lm = loss(F0 - hF * dF, k - hk * dk, s - hs * ds).item()
            fd = (Lp - Lm) / 2.0
            pred = (hF * torch.sum(Ft.grad * dF) + hk * torch.sum(kt.grad * dk) + hs * torch.sum(st.grad * ds)).item()
            rel = abs(pred - fd) / max(abs(fd), 1e-30)
            worst = max(worst, rel)
    banner(f"coupled autograd ({n} steps, checkpoint {K}): worst |adjoint - FD| / |FD| = {worst:.2e}")
    assert worst <= 1e-6


def test_without_inflow_conditions():
    """bc = 0: the source and its transpose apply at every node (no mask)."""
    from paper_1104_5330_amd import Sp6Grid
    from oracle import adjoint
    cfg = SHAPES["planes16"]
    G = Sp6Grid.from_config(cfg, scattering=True, bc=False)
    G.set_scattering_kernel(*THOMSON)
    F = synth.fields.random_state(cfg, 18)
    k, s, e = synth.fields.random_coeffs(cfg, 19)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    G.set_energy_coupling(*GAMMA)
    p = step.Physics(k, s, e, bc=False, scattering=True, kernel=THOMSON, energy=GAMMA)
    g = oracle_grid(cfg)
    assert maxrel(to_host(G.rhs(to_dev(F))), step.rhs(F, g, p)) <= TOL
    dt = 0.25 * stable_dt(cfg)
    lam = synth.fields.random_state(cfg, 20)
    lam_prev, gk, ge, gs = adjoint.adjoint_step(F, lam, g, p, dt)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device="cuda")
    lam_d, gkd, ged, gsd = to_dev(lam), z.clone(), z.clone(), z.clone()
    G.adjoint_step(to_dev(F), dt, lam_d, gkd, ged, gsd)
    assert maxrel(to_host(lam_d), lam_prev) <= TOL
    assert max(maxrel(to_host(gkd), gk), maxrel(to_host(ged), ge), maxrel(to_host(gsd), gs)) <= 1e-11
    G.close()
