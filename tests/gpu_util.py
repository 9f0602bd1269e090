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
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_grid(cfg):
    return og.make_grid(*cfg.shape, r_in=cfg.r_in, r_out=cfg.r_out)


def small(cfg_id, **kw):
    return synth.config(cfg_id).scaled(**kw)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
