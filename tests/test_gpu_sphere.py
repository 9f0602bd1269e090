"""The fused theta-phi pass on 16 x 32 (theta, phi) grids (the workload's sphere):
theta + phi terms, the right-hand side and RK4 steps against the oracle for
several (n_eps, n_r), i.e. several tiles per (eps, r) slab and tile counts
from 96 to 672, and the rejection of a state that is not 16-byte aligned."""

import numpy as np
import pytest
import torch

import synth
from oracle import ops, step
from tests.gpu_util import need_gpu, maxrel, to_dev, to_host, oracle_grid, small, banner

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


SPHERE = dict(n_theta=16, n_phi=32, n_Theta=2, n_Phi=4)


def setup(cfg, seed):
    from paper_1104_5330_amd import Sp6Grid
    G = Sp6Grid.from_config(cfg)
    F = synth.fields.random_state(cfg, seed)
    k, s, e = synth.fields.random_coeffs(cfg, seed + 1)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    return G, F, (k, s, e)


@pytest.mark.parametrize("n_eps,n_r", [(1, 3), (2, 5), (3, 7), (1, 17)])
def test_theta_phi_terms(n_eps, n_r):
    cfg = small(3, n_eps=n_eps, n_r=n_r, **SPHERE)
    banner(f"sphere {cfg.shape}")
    G, F, _ = setup(cfg, n_r)
    g = oracle_grid(cfg)
    _, c_th, c_ph, _, _ = ops.liouville_coefficients(g)
    want = c_th * ops.d_theta(F, g) + c_ph * ops.d_phi(F, g)
    got = to_host(G.apply_L_terms(6, to_dev(F)))
    assert maxrel(got, want) <= TOL


@pytest.mark.parametrize("n_eps,n_r", [(2, 5), (1, 9)])
def test_rhs_and_steps(n_eps, n_r):
    cfg = small(3, n_eps=n_eps, n_r=n_r, n_theta=16, n_phi=32, n_Theta=4, n_Phi=8)
    G, F, (k, s, e) = setup(cfg, 20 + n_r)
    g = oracle_grid(cfg)
    assert maxrel(to_host(G.rhs(to_dev(F))), ops.rhs(F, g, k, s, e)) <= TOL
    want = step.run(F, g, step.Physics(k, s, e), cfg.dt, 2)
    Fd = to_dev(F)
    G.step(Fd, cfg.dt, 2)
    assert maxrel(to_host(Fd), want) <= TOL


def test_unaligned_input_is_rejected():
    # states must be 16-byte aligned
    from paper_1104_5330_amd._lib import Sp6Error
    cfg = small(3, n_eps=1, n_r=5, **SPHERE)
    G, F, _ = setup(cfg, 30)
    buf = torch.zeros(F.size + 1, dtype=torch.float64, device="cuda")
    Fu = buf[1:].view(cfg.shape)  # 8 bytes past a 16-byte boundary
    assert Fu.data_ptr() % 16 == 8
    with pytest.raises(Sp6Error):
        G.apply_L_terms(6, Fu)
