"""sp6_step_noalloc (the step without device allocation, scratch in the library's
fixed per-GPU array) against sp6_step on the same inputs, through the C ABI:
FP64 and mixed handles, two calls in a row with the second on a smaller grid
(the shared array keeps the first call's contents), no device memory taken by
the handle, oversized grids refused before anything is enqueued."""

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import need_gpu, maxrel, small, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def _pair(cfg, precision, nsteps, seed):
    """(sp6_step result, sp6_step_noalloc result, device bytes before/after the
    no-alloc call on a fresh handle)."""
    from paper_1104_5330_amd import Sp6Grid
    dev = torch.device("cuda")
    F0 = torch.as_tensor(synth.fields.shell_state(cfg, seed=seed), device=dev)
    k, s, e = (torch.as_tensor(a, device=dev) for a in synth.fields.random_coeffs(cfg, seed + 1))
    Gn = Sp6Grid.from_config(cfg, precision=precision, scattering=True)
    Gn.set_coefficients(k, s, e)
    before = Gn.device_bytes()
    b = F0.clone()
    Gn.step_noalloc(b, cfg.dt, nsteps)
    torch.cuda.synchronize()
    after = Gn.device_bytes()
    Gn.close()
    Gs = Sp6Grid.from_config(cfg, precision=precision, scattering=True)
    Gs.set_coefficients(k, s, e)
    a = F0.clone()
    Gs.step(a, cfg.dt, nsteps)
    torch.cuda.synchronize()
    Gs.close()
    return a.cpu().numpy(), b.cpu().numpy(), before, after


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_step_matches_step_twice(precision):
    big = small(3, n_eps=2, n_r=17, n_theta=8, n_phi=16, n_Theta=8, n_Phi=16)
    little = small(3, n_eps=1, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8)
    for cfg, seed in ((big, 0), (little, 3)):
        banner(f"noalloc {precision} {cfg.shape}")
        a, b, before, after = _pair(cfg, precision, 3, seed)
        err = maxrel(b, a)
        banner(f"noalloc {precision} {cfg.shape}: max-rel vs sp6_step {err:.2e}, identical {np.array_equal(a, b)}")
        assert err <= 1e-12
        assert after == before  # the handle took no scratch of its own


def test_noalloc_refuses_grids_beyond_its_scratch():
    from paper_1104_5330_amd import Sp6Grid, _lib
    # 2 x 33 x 16 x 32 x 16 x 32 = 17,301,504 points: 415 MB of FP64 scratch
    cfg = small(3, n_eps=2)
    G = Sp6Grid.from_config(cfg, scattering=True)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device="cuda")
    G.set_coefficients(z, z, z)
    F = torch.ones(cfg.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.Sp6Error) as ei:
        G.step_noalloc(F, cfg.dt, 1)
    assert ei.value.status == _lib.SP6_ERR_SHAPE
    torch.cuda.synchronize()
    assert float(F.min()) == 1.0 and float(F.max()) == 1.0  # nothing ran
    G.close()
