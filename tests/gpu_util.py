"""Shared helpers of the GPU parity tests."""

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def maxrel(a, b):
    """max |a - b| / max |b| (normwise relative error)."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def l2rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def to_dev(x):
    # a writable C-order copy (read-only views, e.g. broadcasts, are copied too)
    return torch.from_numpy(np.array(x, dtype=np.float64, order="C")).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_grid(cfg):
    return og.make_grid(*cfg.shape, r_in=cfg.r_in, r_out=cfg.r_out)


def small(cfg_id, **kw):
    return synth.config(cfg_id).scaled(**kw)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def stable_dt(cfg):
    """The workload rule dt = 0.2 (r_1 - r_0), capped so that the stiffest angular
    term stays inside RK4's stability interval on the imaginary axis (about 2.8):
    the phi and Phi derivatives carry 1/sin(theta), and at the first half-shifted
    node theta_0 = pi / (2 n_theta) with r = r_in their rate is (n / 2) / (r_in
    sin theta_0).  Every workload's own dt is below the cap; small test grids that
    pair a short radial line with fine angles are not."""
    import math
    s0 = math.sin(math.pi / (2 * cfg.n_theta))
    lam = max(cfg.n_phi, cfg.n_Phi) / 2 / (cfg.r_in * s0)
    return min(cfg.dt, 0.5 / lam)
