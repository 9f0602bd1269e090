"""The homogeneous emitting and absorbing sphere (uniform kappa, eta = kappa B, no
scattering) run to its stationary state on the GPU from an empty shell, with
the exact intensity I = B (1 - exp(-kappa s)) imposed as inflow (s the path
length back to the surface of a sphere of radius 4 > r_out).  Unfiltered, the
stationary state matches I to a discretisation error that falls fast with
resolution; on the workload's 33 x 16 x 32 x 16 x 32 grid the run is made with
the angular and radial filters (which re-impose the inflow values after every
step) and stays at the discretisation error through t = 14."""

import math

import numpy as np
import pytest
import torch

from oracle import closed_forms as cf
from tests.gpu_util import need_gpu, to_dev, to_host, oracle_grid, small, banner

pytestmark = pytest.mark.gpu

KAPPA, B, R_S = 0.7, 1.3, 4.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def run_to_steady(n_r, n_a, filt=0, t_end=14.0, chunks=2):
    from paper_1104_5330_amd import Sp6Grid
    cfg = small(2, n_eps=1, n_r=n_r, n_theta=n_a, n_phi=2 * n_a, n_Theta=n_a, n_Phi=2 * n_a)
    g = oracle_grid(cfg)
    I = cf.homogeneous_sphere(g, [KAPPA], [B], R_S)
    G = Sp6Grid.from_config(cfg, scattering=False, filter=filt)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device="cuda")
    G.set_coefficients(z + KAPPA, z, z + KAPPA * B)
    G.set_inflow(to_dev(I[:, 0]), to_dev(I[:, -1]))
    F = torch.zeros(cfg.shape, dtype=torch.float64, device="cuda")
    G.project_inflow(F)
    n = math.ceil(t_end / cfg.dt / chunks)
    errs = []
    for _ in range(chunks):
        G.step(F, cfg.dt, n)
        errs.append(float(np.max(np.abs(to_host(F) - I)) / B))
    banner(f"homogeneous sphere {cfg.shape} filter {filt}: {chunks} x {n} steps, max |F - I| / B = "
           + ", ".join(f"{e:.2e}" for e in errs))
    return errs


def test_homogeneous_sphere_steady_state():
    e_lo = run_to_steady(9, 4)[-1]
    e_hi = run_to_steady(17, 8)[-1]
    assert e_hi < 0.1 * e_lo and e_hi < 1e-3
    e_w = run_to_steady(33, 16, filt=2)
    assert e_w[-1] < 1e-3
    assert e_w[-1] <= 1.5 * e_w[0]  # no slow growth once stationary
