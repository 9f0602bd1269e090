"""Streams and HIP graphs.  After a grid's first call has allocated its scratch
buffers, the stepping entry points enqueue kernels only (no allocation, no
memset, no host synchronisation), so they run on any stream and can be captured
into a graph.  Each case: steps on a side stream equal those on the default
stream bit for bit; a captured graph of two steps, replayed three times with the
program's own eager steps and synchronisations in between, equals the eager
result bit for bit on every replay; the FP64 RK4 case also ends against the
oracle."""

import numpy as np
import pytest
import torch

import synth
from oracle import step
from tests.gpu_util import need_gpu, maxrel, to_dev, to_host, oracle_grid, small, banner, stable_dt

pytestmark = pytest.mark.gpu

TOL = 1e-12
SHAPE = dict(n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=8, n_Phi=16)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def setup(precision="fp64", filt=2):
    from paper_1104_5330_amd import Sp6Grid
    cfg = small(3, **SHAPE)
    G = Sp6Grid.from_config(cfg, precision=precision, scattering=True, filter=filt)
    F = synth.fields.random_state(cfg, 11)
    k, s, e = synth.fields.random_coeffs(cfg, 12)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    return cfg, G, F, (k, s, e)


def stepper(G, form, dt, H=None):
    if form == "ab2":
        return lambda F, n: G.step_ab2(F, H, dt, n, start=False)
    if form == "implicit":
        return lambda F, n: G.step_radial_implicit(F, dt, n)
    return lambda F, n: G.step(F, dt, n)


def test_side_stream_equals_default_stream():
    cfg, G, F, _ = setup()
    a, b = to_dev(F), to_dev(F)
    G.step(a, cfg.dt, 2)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        G.step(b, cfg.dt, 2)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    banner("side stream")
    assert torch.equal(a, b)


@pytest.mark.parametrize("form,precision", [("rk4", "fp64"), ("rk4", "mixed"), ("ab2", "fp64"),
                                            ("implicit", "fp64")])
def test_graph_replays_equal_eager(form, precision):
    cfg, G, F, (k, s, e) = setup(precision)
    dt = cfg.dt
    Fe, Fg = to_dev(F), to_dev(F)
    He = Hg = None
    if form == "ab2":
        He, Hg = G.empty(), G.empty()
        G.step_ab2(Fe, He, dt, 1, start=True)
        G.step_ab2(Fg, Hg, dt, 1, start=True)
    else:
        # the first call allocates the scratch buffers (and builds the radial matrices)
        stepper(G, form, dt)(Fe, 1)
        stepper(G, form, dt)(Fg, 1)
    eager = stepper(G, form, dt, He)
    captured = stepper(G, form, dt, Hg)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    # capture records the launches without running them: Fg keeps its value
    with torch.cuda.graph(graph):
        captured(Fg, 2)
    torch.cuda.synchronize()
    assert torch.equal(Fe, Fg)
    for rep in range(3):
        graph.replay()
        eager(Fe, 2)
        torch.cuda.synchronize()
        banner(f"graph {form} {precision}: replay {rep}")
        assert torch.equal(Fe, Fg), f"replay {rep} differs from the eager steps"
        if He is not None:
            assert torch.equal(He, Hg)
    if form == "rk4" and precision == "fp64":
        g = oracle_grid(cfg)
        p = step.Physics(k, s, e, bc=True, scattering=True, filt=True, filt_r=True)
        want = step.run(F, g, p, dt, 7)
        err = maxrel(to_host(Fg), want)
        banner(f"graph rk4 fp64: 7 steps vs oracle {err:.2e}")
        assert err <= TOL
    del graph


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_equal_eager_sphere64(precision):
    """The 32 x 64 position sphere, no filter: the captured two-step call holds the
    state in the paired in-plane order between its steps (FP64) and the stage
    buffers in it (both paths); every replay equals the eager call bit for bit."""
    from paper_1104_5330_amd import Sp6Grid
    cfg = small(5, n_eps=1, n_r=3, n_Theta=8, n_Phi=16)
    G = Sp6Grid.from_config(cfg, precision=precision, scattering=True)
    F = synth.fields.random_state(cfg, 13)
    k, s, e = synth.fields.random_coeffs(cfg, 14)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    dt = stable_dt(cfg)
    Fe, Fg = to_dev(F), to_dev(F)
    G.step(Fe, dt, 1)
    G.step(Fg, dt, 1)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        G.step(Fg, dt, 2)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        G.step(Fe, dt, 2)
        torch.cuda.synchronize()
        banner(f"graph sphere64 {precision}: replay {rep}")
        assert torch.equal(Fe, Fg), f"replay {rep} differs from the eager steps"
    del graph
