"""The split step of App. B on the GPU (RK4 on the angular and collision terms,
backward-Euler radial solve) against the oracle: shapes whose 16-column groups
are contiguous (n_Phi >= 16) and gathered (n_Phi < 16), ragged n_eps and n_r,
n_r up to the largest padding, inflow held or not, with the radial filter, the
matrix cache across time steps, the mixed path, and one energy group of the
full-size workload in the launch configuration of the benchmark."""

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og, ops, step
from tests.gpu_util import need_gpu, maxrel, to_dev, to_host, oracle_grid, small, banner, stable_dt

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def setup(cfg, seed=0, **kw):
    from paper_1104_5330_amd import Sp6Grid
    G = Sp6Grid.from_config(cfg, **kw)
    F = synth.fields.random_state(cfg, seed)
    k, s, e = synth.fields.random_coeffs(cfg, seed + 1)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    return G, F, (k, s, e)


SHAPES = {
    "tiny": dict(n_eps=1, n_r=5, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4),
    "ragged": dict(n_eps=3, n_r=7, n_theta=2, n_phi=4, n_Theta=4, n_Phi=8),
    "contiguous": dict(n_eps=2, n_r=17, n_theta=4, n_phi=8, n_Theta=8, n_Phi=16),
    "wide": dict(n_eps=1, n_r=9, n_theta=4, n_phi=8, n_Theta=16, n_Phi=32),
    "long_r": dict(n_eps=1, n_r=65, n_theta=2, n_phi=4, n_Theta=8, n_Phi=16),
    # the 32 x 64 position sphere: the state is held in the paired in-plane order
    # between the steps of a call, and the radial solve runs on it
    "sphere64": dict(n_eps=1, n_r=5, n_theta=32, n_phi=64, n_Theta=8, n_Phi=16),
}


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("bc", [True, False])
def test_split_step(name, bc):
    cfg = small(3, **SHAPES[name])
    banner(f"implicit {name} bc={bc} {cfg.shape}")
    G, F, (k, s, e) = setup(cfg, seed=1, bc=bc)
    g = oracle_grid(cfg)
    p = step.Physics(k, s, e, bc=bc, scattering=True, radial_implicit=True)
    # the angular terms' stability bound (the split step lifts only the radial one)
    dt = stable_dt(cfg)
    want = step.run(F, g, p, dt, 3)
    Fd = to_dev(F)
    G.step_radial_implicit(Fd, dt, 3)
    err = maxrel(to_host(Fd), want)
    banner(f"  max-rel {err:.2e}")
    assert err <= TOL


def test_inflow_nodes_held():
    cfg = small(3, **SHAPES["contiguous"])
    G, F, (k, s, e) = setup(cfg, seed=2)
    gi, go = synth.fields.inflow_planes(cfg, 3)
    G.set_inflow(to_dev(gi), to_dev(go))
    g = oracle_grid(cfg)
    F = ops.project_inflow(F, g, gi, go)
    p = step.Physics(k, s, e, radial_implicit=True)
    want = step.run(F, g, p, cfg.dt, 2)
    Fd = to_dev(F)
    G.step_radial_implicit(Fd, cfg.dt, 2)
    got = to_host(Fd)
    assert maxrel(got, want) <= TOL
    cT = np.cos(g.Theta)
    assert np.array_equal(got[:, 0][:, :, :, cT > 0], gi[:, :, :, cT > 0])
    assert np.array_equal(got[:, -1][:, :, :, cT < 0], go[:, :, :, cT < 0])


def test_with_radial_filter():
    cfg = small(3, **SHAPES["contiguous"])
    G, F, (k, s, e) = setup(cfg, seed=4, filter=2)
    g = oracle_grid(cfg)
    p = step.Physics(k, s, e, filt=True, filt_r=True, radial_implicit=True)
    want = step.run(F, g, p, cfg.dt, 2)
    Fd = to_dev(F)
    G.step_radial_implicit(Fd, cfg.dt, 2)
    assert maxrel(to_host(Fd), want) <= TOL


def test_matrix_cache_follows_dt():
    # the backward-Euler matrices depend on dt: alternate two steps sizes, and
    # interleave explicit steps, on one handle
    cfg = small(3, **SHAPES["ragged"])
    G, F, (k, s, e) = setup(cfg, seed=5)
    g = oracle_grid(cfg)
    p_imp = step.Physics(k, s, e, radial_implicit=True)
    p_exp = step.Physics(k, s, e)
    y = F
    Fd = to_dev(F)
    for dt, implicit in [(cfg.dt, True), (2 * cfg.dt, True), (cfg.dt, False), (cfg.dt, True)]:
        if implicit:
            y = step.run(y, g, p_imp, dt, 1)
            G.step_radial_implicit(Fd, dt, 1)
        else:
            y = step.run(y, g, p_exp, dt, 1)
            G.step(Fd, dt, 1)
        assert maxrel(to_host(Fd), y) <= TOL


def test_mixed_path():
    cfg = small(3, **SHAPES["wide"])
    G, F, (k, s, e) = setup(cfg, seed=6, precision="mixed")
    g = oracle_grid(cfg)
    want = step.run(F, g, step.Physics(k, s, e, radial_implicit=True), cfg.dt, 2)
    Fd = to_dev(F)
    G.step_radial_implicit(Fd, cfg.dt, 2)
    err = maxrel(to_host(Fd), want)
    banner(f"implicit mixed: max-rel {err:.2e}")
    assert err <= 1e-5


def test_argument_checks():
    from paper_1104_5330_amd import Sp6Grid
    from paper_1104_5330_amd._lib import Sp6Error
    cfg = small(3, **SHAPES["tiny"])
    G, F, _ = setup(cfg)
    Fd = to_dev(F)
    with pytest.raises(Sp6Error):
        G.step_radial_implicit(Fd, -1.0, 1)
    with pytest.raises(Sp6Error):
        G.step_radial_implicit(Fd, float("nan"), 1)
    G.step_radial_implicit(Fd, cfg.dt, 0)
    assert np.array_equal(to_host(Fd), F)
    G2 = Sp6Grid.from_config(cfg)
    with pytest.raises(Sp6Error):  # no coefficients
        G2.step_radial_implicit(Fd, cfg.dt, 1)


def test_workload2_group_split_step():
    # full size: one split step of the 8-group state (launch configuration of the
    # benchmark) and the oracle's step of one group
    from paper_1104_5330_amd import Sp6Grid
    cfg = synth.config(2)
    dev = torch.device("cuda")
    F0 = synth.fields.shell_state(cfg, device=dev)
    coeffs = synth.fields.coefficients(cfg)
    G = Sp6Grid.from_config(cfg, scattering=False)
    G.set_coefficients(*(torch.as_tensor(a, device=dev) for a in coeffs))
    F = F0.clone()
    G.step_radial_implicit(F, cfg.dt, 1)
    grp = 6
    g1 = og.make_grid(*cfg.scaled(n_eps=1).shape)
    k, s, e = (a[grp:grp + 1] for a in coeffs)
    p = step.Physics(k, s, e, scattering=False, radial_implicit=True)
    want = step.rk4_step(F0[grp:grp + 1].cpu().numpy(), g1, p, cfg.dt)
    err = maxrel(F[grp:grp + 1].cpu().numpy(), want)
    banner(f"{cfg.name}: implicit group {grp} after one step max-rel {err:.2e}")
    assert err <= TOL
