"""Adams-Bashforth stepping (the scheme of Sect. 5.1) on the GPU against the
oracle: several steps from a forward-Euler start, continuation across calls
through the history buffer, with the filter, the uniform-medium closed form, and
the handle checks (FP64 only)."""

import numpy as np
import pytest
import torch

import synth
from oracle import step
from tests.gpu_util import need_gpu, maxrel, to_dev, to_host, oracle_grid, small, banner

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def setup(cfg, filt=0, seed=0):
    from paper_1104_5330_amd import Sp6Grid
    G = Sp6Grid.from_config(cfg, scattering=True, filter=filt)
    F = synth.fields.random_state(cfg, seed)
    k, s, e = synth.fields.random_coeffs(cfg, seed + 1)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    return G, F, (k, s, e)


@pytest.mark.parametrize("name,shape,filt", [
    ("tiny", dict(n_eps=1, n_r=5, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4), 0),
    ("small", dict(n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8), 0),
    ("w3_reduced", dict(n_eps=1, n_r=9), 0),
    ("filtered", dict(n_eps=1, n_r=17, n_theta=4, n_phi=8, n_Theta=8, n_Phi=16), 2),
])
def test_ab2_steps_and_continuation(name, shape, filt):
    cfg = small(3, **shape)
    G, F, (k, s, e) = setup(cfg, filt)
    g = oracle_grid(cfg)
    p = step.Physics(k, s, e, bc=True, scattering=True, filt=bool(filt), filt_r=filt == 2)
    dt = cfg.dt
    want, kw = step.ab2_run(F, g, p, dt, 6)
    Fd, Hd = to_dev(F), torch.empty(cfg.shape, dtype=torch.float64, device="cuda")
    G.step_ab2(Fd, Hd, dt, 2, start=True)
    G.step_ab2(Fd, Hd, dt, 4, start=False)
    err = maxrel(to_host(Fd), want)
    # the history buffer is F_n - dt/2 k_{n-1}
    herr = maxrel(to_host(Hd), want - 0.5 * dt * kw)
    banner(f"AB2 {name}: 6 steps (2 + 4) {err:.2e}, history {herr:.2e}")
    assert err <= TOL and herr <= TOL


def test_ab2_uniform_medium_closed_form():
    from oracle import closed_forms as cf
    from paper_1104_5330_amd import Sp6Grid
    cfg = small(3, n_eps=1, n_r=9, n_theta=8, n_phi=16, n_Theta=8, n_Phi=16)
    g = oracle_grid(cfg)
    a, b = 1.0, (0.5, -0.3, 0.2)
    Q = np.array([[0.4, 0.1, -0.2], [0.1, -0.1, 0.3], [-0.2, 0.3, 0.25]])
    kern = (0.0, 0.75)
    F0 = cf.isotropisation(g, a, b, Q, 0.0, kern, 0.0, 0)
    dt = cfg.dt
    sig = 0.3 / dt
    G = Sp6Grid.from_config(cfg, bc=False, scattering=True)
    G.set_scattering_kernel(*kern)
    z = np.zeros(cfg.shape[:4])
    G.set_coefficients(to_dev(z), to_dev(z + sig), to_dev(z))
    Fd, Hd = to_dev(F0), torch.empty(cfg.shape, dtype=torch.float64, device="cuda")
    G.step_ab2(Fd, Hd, dt, 12)
    err = maxrel(to_host(Fd), cf.isotropisation_ab2(g, a, b, Q, sig, kern, dt, 12))
    banner(f"AB2 uniform medium (Thomson) vs closed form: {err:.2e}")
    assert err <= TOL


def test_ab2_handle_checks():
    from paper_1104_5330_amd import Sp6Grid, Sp6Error
    cfg = small(3, n_eps=1, n_r=5, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4)
    G = Sp6Grid.from_config(cfg, precision="mixed")
    k, s, e = synth.fields.random_coeffs(cfg, 1)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    F = to_dev(synth.fields.random_state(cfg, 0))
    H = torch.empty_like(F)
    with pytest.raises(Sp6Error) as ei:
        G.step_ab2(F, H, cfg.dt, 1)
    assert ei.value.status == 5  # SP6_ERR_STATE
    G64, F2, _ = setup(cfg)
    Fd = to_dev(F2)
    with pytest.raises(Sp6Error) as ei:
        G64.step_ab2(Fd, Fd, cfg.dt, 1)  # H must be distinct from F
    assert ei.value.status == 1
