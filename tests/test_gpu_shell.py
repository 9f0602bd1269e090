"""The 5D shell problem of Sect. 5.3 (coherent scattering in a shell with a
density profile, Lambert inflow at r_in, radial and angular filters) and the
radial filter on the GPU, against the FP64 oracle: the filter alone, RK4 steps
with the filter after each step, the adjoint step with the transposed filter,
the mixed path, and two full-size steps of the shell workload."""

import numpy as np
import pytest
import torch

import synth
from oracle import ops, step, adjoint
from tests.gpu_util import need_gpu, maxrel, to_dev, to_host, oracle_grid, small, banner, stable_dt

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


@pytest.mark.parametrize("shape", [
    dict(n_eps=1, n_r=5, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4),
    dict(n_eps=2, n_r=17, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8),
    dict(n_eps=1, n_r=33, n_theta=4, n_phi=8, n_Theta=8, n_Phi=16),
    dict(n_eps=1, n_r=65, n_theta=2, n_phi=4, n_Theta=4, n_Phi=8),
    dict(n_eps=1, n_r=23, n_theta=2, n_phi=4, n_Theta=4, n_Phi=8),
], ids=["r5", "r17", "r33", "r65", "r23"])
def test_radial_filter(shape):
    from paper_1104_5330_amd import Sp6Grid
    cfg = small(6, **shape)
    G = Sp6Grid.from_config(cfg, filter=2)
    F = synth.fields.random_state(cfg, 0)
    Fd = to_dev(F)
    G.apply_filter(Fd)
    err = maxrel(to_host(Fd), ops.apply_filter(F, oracle_grid(cfg), radial=True))
    banner(f"radial filter {cfg.shape}: {err:.2e}")
    assert err <= TOL


def setup(cfg, precision="fp64"):
    from paper_1104_5330_amd import Sp6Grid
    G = Sp6Grid.from_config(cfg, scattering=True, filter=2, precision=precision)
    k, s, e = synth.fields.coefficients(cfg)
    g_in, g_out = synth.fields.lambert_inflow(cfg)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    G.set_inflow(to_dev(g_in), to_dev(g_out))
    # a seeded interior plus the projected inflow (the shell experiment starts empty)
    F = ops.project_inflow(0.1 * synth.fields.polynomial_state(cfg, seed=1), oracle_grid(cfg), g_in, g_out)
    return G, F, (k, s, e), (g_in, g_out)


# the 32 x 64 position sphere: the stage buffers in the paired in-plane order,
# the state in the plain one between steps (the filter runs on it)
SHELL_SHAPES = {"small": dict(n_r=17, n_theta=4, n_phi=8, n_Theta=8, n_Phi=16),
                "sphere64": dict(n_r=5, n_theta=32, n_phi=64, n_Theta=8, n_Phi=16)}


@pytest.mark.parametrize("name", list(SHELL_SHAPES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shell_steps(precision, name):
    cfg = small(6, **SHELL_SHAPES[name])
    G, F, (k, s, e), (gi, go) = setup(cfg, precision)
    g = oracle_grid(cfg)
    p = step.Physics(k, s, e, bc=True, scattering=True, filt=True, filt_r=True, g_in=gi, g_out=go)
    dt = stable_dt(cfg)
    Fd = to_dev(F)
    G.step(Fd, dt, 5)
    err = maxrel(to_host(Fd), step.run(F, g, p, dt, 5))
    banner(f"shell {precision}: 5 steps with radial + angular filters: {err:.2e}")
    assert err <= (TOL if precision == "fp64" else 1e-5)


def test_shell_adjoint():
    cfg = small(6, n_r=17, n_theta=4, n_phi=8, n_Theta=8, n_Phi=16)
    G, F, (k, s, e), (gi, go) = setup(cfg)
    g = oracle_grid(cfg)
    p = step.Physics(k, s, e, bc=True, scattering=True, filt=True, filt_r=True, g_in=gi, g_out=go)
    lam = synth.fields.random_state(cfg, 4)
    lam_prev, gk, ge, gs = adjoint.adjoint_step(F, lam, g, p, cfg.dt)
    lam_d = to_dev(lam)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device="cuda")
    gsd = z.clone()
    G.adjoint_step(to_dev(F), cfg.dt, lam_d, None, None, gsd)
    e1, e2 = maxrel(to_host(lam_d), lam_prev), maxrel(to_host(gsd), gs)
    banner(f"shell adjoint with the transposed filter: lam {e1:.2e}, grad sigma {e2:.2e}")
    assert e1 <= TOL and e2 <= 1e-11


def test_shell_full_size_two_steps():
    """The shell workload at full size (33 x 16 x 32 x 16 x 32, optical depth 5):
    two steps against the oracle."""
    from paper_1104_5330_amd import Sp6Grid
    cfg = synth.config(6)
    g = oracle_grid(cfg)
    k, s, e = synth.fields.coefficients(cfg)
    g_in, g_out = synth.fields.lambert_inflow(cfg)
    G = Sp6Grid.from_config(cfg, scattering=True, filter=2)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    G.set_inflow(to_dev(g_in), to_dev(g_out))
    F = ops.project_inflow(np.zeros(cfg.shape), g, g_in, g_out)
    Fd = to_dev(F)
    G.step(Fd, cfg.dt, 2)
    p = step.Physics(k, s, e, bc=True, scattering=True, filt=True, filt_r=True, g_in=g_in, g_out=g_out)
    err = maxrel(to_host(Fd), step.run(F, g, p, cfg.dt, 2))
    banner(f"{cfg.name}: 2 full-size steps vs oracle: {err:.2e}")
    assert err <= TOL
