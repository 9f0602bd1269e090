"""Full-size checks in the launch configuration the benchmark times.

* Workload 2 (8 groups, (33, 16, 32, 16, 32)): the right-hand side at sampled
  nodes against the oracle's single-node evaluation, and one whole RK4 step of
  one energy group against the oracle (groups are independent, so the group
  slab of the full 8-group GPU step must match the oracle's one-group step).
* Workload 5 (4 groups, (65, 32, 64, 32, 64), 8.7 GB per state): the
  right-hand side at sampled nodes, and the mixed path against the FP64 path
  over the workload's 50 steps (max-relative and L2-relative error printed).
"""

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og, ops, step
from tests.gpu_util import need_gpu, maxrel, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


class _Lines:
    """numpy-style read access to a GPU tensor, fetching only what is indexed."""

    def __init__(self, t):
        self.t = t

    def __getitem__(self, idx):
        return self.t[idx].cpu().numpy()


def _sample_indices(shape, n, seed):
    rng = np.random.default_rng(seed)
    idx = [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(n)]
    e, nr, nth, nph, nTh, nPh = shape
    # boundaries and extremes: both radial ends, first/last theta and Theta nodes
    idx += [(0, 0, 0, 0, 0, 0), (e - 1, nr - 1, nth - 1, nph - 1, nTh - 1, nPh - 1),
            (0, 0, nth - 1, 1, nTh // 2, nPh // 2), (e - 1, nr - 1, 0, nph // 2, nTh // 2 - 1, 3)]
    return idx


def _check_sampled_rhs(cfg, G, Fd, coeffs, n, seed, scattering):
    k, s, e = coeffs
    g = og.make_grid(*cfg.shape, r_in=cfg.r_in, r_out=cfg.r_out)
    out = G.rhs(Fd)
    torch.cuda.synchronize()
    lines = _Lines(Fd)
    got, want = [], []
    for idx in _sample_indices(cfg.shape, n, seed):
        want.append(ops.rhs_at(lines, g, k, s, e, idx, scattering=scattering))
        got.append(out[idx].item())
    got, want = np.array(got), np.array(want)
    scale = out.abs().max().item()
    err = np.max(np.abs(got - want)) / scale
    banner(f"{cfg.name}: sampled rhs max err / max|rhs| = {err:.2e} over {len(got)} nodes")
    return err


def test_workload2_sampled_rhs_and_group_step():
    from paper_1104_5330_amd import Sp6Grid
    cfg = synth.config(2)
    dev = torch.device("cuda")
    F0 = synth.fields.shell_state(cfg, device=dev)
    coeffs = synth.fields.coefficients(cfg)
    G = Sp6Grid.from_config(cfg, scattering=False)
    G.set_coefficients(*(torch.as_tensor(a, device=dev) for a in coeffs))
    assert _check_sampled_rhs(cfg, G, F0, coeffs, 300, 0, scattering=False) <= 1e-12
    F = F0.clone()
    G.step(F, cfg.dt, 1)
    grp = 5
    sub = cfg.scaled(n_eps=1)
    g1 = og.make_grid(*sub.shape)
    k, s, e = (a[grp:grp + 1] for a in coeffs)
    want = step.rk4_step(F0[grp:grp + 1].cpu().numpy(), g1, step.Physics(k, s, e, scattering=False), cfg.dt)
    err = maxrel(F[grp:grp + 1].cpu().numpy(), want)
    banner(f"{cfg.name}: group {grp} after one step max-rel {err:.2e}")
    assert err <= 1e-12


def test_workload5_sampled_rhs_and_mixed():
    from paper_1104_5330_amd import Sp6Grid
    cfg = synth.config(5)
    dev = torch.device("cuda")
    F0 = synth.fields.shell_state(cfg, device=dev)
    coeffs = synth.fields.coefficients(cfg)
    kd = [torch.as_tensor(a, device=dev) for a in coeffs]
    G = Sp6Grid.from_config(cfg)
    G.set_coefficients(*kd)
    assert _check_sampled_rhs(cfg, G, F0, coeffs, 100, 1, scattering=True) <= 1e-12
    Gm = Sp6Grid.from_config(cfg, precision="mixed")
    Gm.set_coefficients(*kd)
    a = F0.clone()
    G.step(a, cfg.dt, cfg.steps)
    G.close()
    b = F0.clone()
    del F0
    Gm.step(b, cfg.dt, cfg.steps)
    torch.cuda.synchronize()
    assert torch.isfinite(a).all() and torch.isfinite(b).all()
    d = (a - b).abs().max().item() / a.abs().max().item()
    l2 = (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a)).item()
    banner(f"{cfg.name}: mixed vs FP64 after {cfg.steps} steps max-rel {d:.2e} L2-rel {l2:.2e}")
    assert d <= 1e-5
