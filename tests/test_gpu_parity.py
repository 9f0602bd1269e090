"""GPU parity: every entry point of the HIP library against the FP64 oracle,
element by element, on seeded inputs that span several tiles and ragged tails.
Tolerance: 1e-12 normwise relative (FP64 path)."""

import numpy as np
import pytest
import torch

import synth
from oracle import ops, step, adjoint, diagnostics
from tests.gpu_util import need_gpu, maxrel, l2rel, to_dev, to_host, oracle_grid, small, banner, stable_dt

pytestmark = pytest.mark.gpu

TOL = 1e-12

# (name, config) shapes: tiny, ragged (odd n_eps * n_r with the 16-plane kernel),
# the small workload, a reduced workload-2 shape, one of each line length, a
# wide (Theta, Phi) plane whose fused theta-phi tiles are split Theta rows, the
# radial lengths of the large workloads (n_r = 33: nine 4-row k-steps; n_r = 65:
# seventeen, five 16-row tiles, the last one ragged), one (eps, r) slab set of the
# large grid's angular shape (theta lines of 64 points, 2048-point planes), and
# the 32 x 64 position sphere on small planes (fused theta-phi tiles spanning two
# Theta rows of a 128-byte line; odd n_eps * n_r, so the last workgroups are idle)
# and on 16 x 32 planes (two-plane workgroups of the plane pass),
# and the smallest and largest radial lines the descriptor accepts (n_r = 3: one
# k-step, one row tile mostly padding; n_r = 80: twenty k-steps, five full row tiles)
SHAPES = {
    "tiny": small(3, n_eps=1, n_r=5, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4),
    "ragged": small(3, n_eps=3, n_r=7, n_theta=2, n_phi=4, n_Theta=2, n_Phi=4),
    "cfg1": small(3, n_eps=1),
    "w2_reduced": small(3, n_eps=2, n_r=9),
    "mixed_lines": small(3, n_eps=2, n_r=17, n_theta=4, n_phi=64, n_Theta=8, n_Phi=16),
    "big_lines": small(3, n_eps=1, n_r=6, n_theta=32, n_phi=8, n_Theta=32, n_Phi=64),
    "wide_plane": small(3, n_eps=2, n_r=5, n_theta=4, n_phi=8, n_Theta=32, n_Phi=64),
    "r33": small(3, n_eps=3, n_r=33, n_theta=2, n_phi=4, n_Theta=4, n_Phi=8),
    "r65": small(3, n_eps=1, n_r=65, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8),
    "w5_slab": small(5, n_eps=1, n_r=3),
    "s64_small": small(5, n_eps=1, n_r=3, n_Theta=8, n_Phi=16),
    "s64_ragged": small(5, n_eps=3, n_r=5, n_Theta=8, n_Phi=16),
    "s64_mid": small(5, n_eps=1, n_r=3, n_Theta=16, n_Phi=32),
    "r3": small(3, n_eps=2, n_r=3, n_theta=2, n_phi=4, n_Theta=4, n_Phi=8),
    "r80": small(3, n_eps=1, n_r=80, n_theta=2, n_phi=4, n_Theta=4, n_Phi=8),
}
SHAPES["cfg1"] = synth.config(1).scaled(physics="scatter")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401  (fails loudly if the library is missing)


def make(cfg, **kw):
    from paper_1104_5330_amd import Sp6Grid
    return Sp6Grid.from_config(cfg, **kw)


def setup(cfg, seed=0, bc=True, scattering=True):
    G = make(cfg, bc=bc, scattering=scattering)
    F = synth.fields.random_state(cfg, seed)
    k, s, e = synth.fields.random_coeffs(cfg, seed + 1)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    return G, F, (k, s, e)


@pytest.mark.parametrize("name", list(SHAPES))
def test_terms(name):
    cfg = SHAPES[name]
    banner(f"terms {name} {cfg.shape}")
    G, F, _ = setup(cfg)
    g = oracle_grid(cfg)
    c_r, c_th, c_ph, c_Th, c_Ph = ops.liouville_coefficients(g)
    want = {1: c_r * ops.d_r(F, g), 2: c_th * ops.d_theta(F, g), 4: c_ph * ops.d_phi(F, g),
            8: c_Th * ops.d_Theta(F, g), 16: c_Ph * ops.d_Phi(F, g)}
    Fd = to_dev(F)
    errs = {bit: maxrel(to_host(G.apply_L_terms(bit, Fd)), w) for bit, w in want.items()}
    errs[31] = maxrel(to_host(G.apply_L(Fd)), ops.apply_L(F, g))
    assert max(errs.values()) <= TOL, (name, errs)


@pytest.mark.parametrize("name", list(SHAPES))
def test_rhs_and_transpose(name):
    cfg = SHAPES[name]
    banner(f"rhs/LT {name}")
    G, F, (k, s, e) = setup(cfg, seed=3)
    g = oracle_grid(cfg)
    got = to_host(G.rhs(to_dev(F)))
    assert maxrel(got, ops.rhs(F, g, k, s, e)) <= TOL
    X = synth.fields.random_state(cfg, 9)
    got = to_host(G.apply_LT(to_dev(X)))
    assert maxrel(got, ops.apply_LT(X, g)) <= TOL


@pytest.mark.parametrize("bc,scat", [(True, True), (False, False), (True, False)])
def test_rhs_switches(bc, scat):
    cfg = SHAPES["w2_reduced"]
    G, F, (k, s, e) = setup(cfg, seed=4, bc=bc, scattering=scat)
    g = oracle_grid(cfg)
    got = to_host(G.rhs(to_dev(F)))
    assert maxrel(got, ops.rhs(F, g, k, s, e, bc=bc, scattering=scat)) <= TOL


@pytest.mark.parametrize("name", ["tiny", "ragged", "cfg1", "w2_reduced", "big_lines", "wide_plane", "r33", "r65",
                                  "w5_slab", "s64_small", "s64_ragged", "s64_mid", "r3", "r80"])
def test_step(name):
    cfg = SHAPES[name]
    banner(f"step {name}")
    G, F, (k, s, e) = setup(cfg, seed=5)
    g = oracle_grid(cfg)
    dt = stable_dt(cfg)
    p = step.Physics(k, s, e, bc=True, scattering=True)
    want = step.run(F, g, p, dt, 3)
    Fd = to_dev(F)
    G.step(Fd, dt, 3)
    assert maxrel(to_host(Fd), want) <= TOL


@pytest.mark.parametrize("name", ["w5_slab", "s64_ragged", "w2_reduced"])
def test_step_calls_agree(name):
    """Three steps in one call against three one-step calls: on the 32 x 64 sphere
    the state is held in the paired in-plane order between the steps of a call
    and written back in the plain order by its last step.  Without scattering
    the arithmetic does not depend on the order: bit for bit.  With isotropic
    scattering a plane's angular mean is summed over the lanes in the order of
    their columns, which the paired order permutes: equal to rounding.  The
    16 x 32 sphere keeps the plain order throughout (bit for bit either way)."""
    cfg = SHAPES[name]
    dt = stable_dt(cfg)
    for scat in (False, True):
        G, F, _ = setup(cfg, seed=11, scattering=scat)
        a, b = to_dev(F), to_dev(F)
        G.step(a, dt, 3)
        for _ in range(3):
            G.step(b, dt, 1)
        if scat and name != "w2_reduced":
            assert maxrel(to_host(a), to_host(b)) <= 1e-14
        else:
            assert torch.equal(a, b), (name, scat)


def test_step_is_deterministic():
    cfg = SHAPES["w2_reduced"]
    G, F, _ = setup(cfg, seed=6)
    a = to_dev(F)
    b = to_dev(F)
    G.step(a, cfg.dt, 2)
    G.step(b, cfg.dt, 2)
    assert torch.equal(a, b)


@pytest.mark.parametrize("name", ["tiny", "ragged", "cfg1", "w2_reduced", "wide_plane", "r33", "r65", "s64_small",
                                  "s64_ragged", "r3", "r80"])
def test_adjoint_step(name):
    cfg = SHAPES[name]
    banner(f"adjoint {name}")
    G, F, (k, s, e) = setup(cfg, seed=7)
    g = oracle_grid(cfg)
    dt = stable_dt(cfg)
    p = step.Physics(k, s, e, bc=True, scattering=True)
    lam = synth.fields.random_state(cfg, 8)
    lam_prev, gk, ge, gs = adjoint.adjoint_step(F, lam, g, p, dt)
    lam_d = to_dev(lam)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device="cuda")
    gkd, ged, gsd = z.clone() + 1.0, z.clone(), z.clone()
    G.adjoint_step(to_dev(F), dt, lam_d, gkd, ged, gsd)
    assert maxrel(to_host(lam_d), lam_prev) <= TOL
    assert maxrel(to_host(gkd) - 1.0, gk) <= 1e-11  # accumulated onto 1.0
    assert maxrel(to_host(ged), ge) <= 1e-11
    assert maxrel(to_host(gsd), gs) <= 1e-11


def test_adjoint_dot_product_gpu():
    cfg = SHAPES["w2_reduced"]
    G, F, _ = setup(cfg, seed=10)
    lam = synth.fields.random_state(cfg, 11)
    dF = synth.fields.random_state(cfg, 12)
    dt = cfg.dt
    Fd = to_dev(F + dF)
    G.step(Fd, dt, 1)
    F0 = to_dev(F)
    G.step(F0, dt, 1)
    lin = to_host(Fd) - to_host(F0)  # the step is affine in F: exact up to rounding
    lam_d = to_dev(lam)
    G.adjoint_step(to_dev(F), dt, lam_d)
    lhs = float(np.sum(lam * lin))
    rhs = float(np.sum(to_host(lam_d) * dF))
    assert lhs == pytest.approx(rhs, rel=1e-10)


@pytest.mark.parametrize("name", ["tiny", "cfg1", "big_lines"])
def test_filter(name):
    cfg = SHAPES[name]
    G, F, _ = setup(cfg, seed=13)
    g = oracle_grid(cfg)
    Fd = to_dev(F)
    G.apply_filter(Fd)
    assert maxrel(to_host(Fd), ops.apply_filter(F, g)) <= TOL


def test_step_with_filter():
    cfg = SHAPES["cfg1"]
    G = make(cfg, filter=True)
    F = synth.fields.beam(cfg)
    k, s, e = synth.fields.random_coeffs(cfg, 2)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    g = oracle_grid(cfg)
    p = step.Physics(k, s, e, filt=True)
    want = step.run(F, g, p, cfg.dt, 2)
    Fd = to_dev(F)
    G.step(Fd, cfg.dt, 2)
    assert maxrel(to_host(Fd), want) <= TOL
    lam = synth.fields.random_state(cfg, 3)
    lp, gk, ge, gs = adjoint.adjoint_step(F, lam, g, p, cfg.dt)
    ld = to_dev(lam)
    G.adjoint_step(to_dev(F), cfg.dt, ld)
    assert maxrel(to_host(ld), lp) <= TOL


@pytest.mark.parametrize("name", ["tiny", "ragged", "cfg1", "w2_reduced"])
def test_diagnostics_and_flux(name):
    cfg = SHAPES[name]
    G, F, _ = setup(cfg, seed=14)
    g = oracle_grid(cfg)
    N, Ji, Jo = G.diagnostics(to_dev(F))
    wN, wJi, wJo = diagnostics.fluxes(F, g)
    scale = np.max(np.abs(wN)) + np.max(np.abs(wJi)) + np.max(np.abs(wJo))
    assert np.max(np.abs(N - wN)) <= 1e-13 * scale
    assert np.max(np.abs(Ji - wJi)) <= 1e-13 * scale
    assert np.max(np.abs(Jo - wJo)) <= 1e-13 * scale
    j = to_host(G.outgoing_flux(to_dev(F)))
    assert maxrel(j, diagnostics.outgoing_flux_map(F, g)) <= 1e-13


def test_inflow_projection_and_hold():
    cfg = SHAPES["w2_reduced"]
    G, F, (k, s, e) = setup(cfg, seed=15)
    gi, go = synth.fields.inflow_planes(cfg, 16)
    G.set_inflow(to_dev(gi), to_dev(go))
    g = oracle_grid(cfg)
    want = ops.project_inflow(F, g, gi, go)
    Fd = to_dev(F)
    G.project_inflow(Fd)
    assert np.array_equal(to_host(Fd), want)
    # the inflow values are held by the step
    p = step.Physics(k, s, e)
    want = step.run(want, g, p, cfg.dt, 2)
    G.step(Fd, cfg.dt, 2)
    got = to_host(Fd)
    assert maxrel(got, want) <= TOL
    cT = np.cos(g.Theta)
    assert np.array_equal(got[:, 0][:, :, :, cT > 0], gi[:, :, :, cT > 0])
    G.set_inflow(None, None)
    Fd = to_dev(F)
    G.project_inflow(Fd)
    assert np.all(to_host(Fd)[:, 0][:, :, :, cT > 0] == 0.0)


def test_config1_free_streaming_vs_oracle_and_closed_form():
    # vacuum, zero inflow, 10 steps: against the oracle (gated), and against the
    # closed form F0(x - t omega, omega) in the shell (Sect. 2.1; resolution
    # limited, reported with a loose bound)
    from oracle import closed_forms
    cfg = synth.config(1)
    G = make(cfg, scattering=False)
    z = torch.zeros(cfg.shape[:4], dtype=torch.float64, device="cuda")
    G.set_coefficients(z, z, z)
    F = synth.fields.beam(cfg)
    g = oracle_grid(cfg)
    F = ops.project_inflow(F, g)
    Fd = to_dev(F)
    G.step(Fd, cfg.dt, cfg.steps)
    want = step.run(F, g, step.Physics.vacuum(g), cfg.dt, cfg.steps)
    got = to_host(Fd)
    assert maxrel(got, want) <= TOL
    exact = closed_forms.free_streaming_shell(g, synth.fields.beam_function(cfg), cfg.steps * cfg.dt)
    mr, lr = maxrel(got, exact), l2rel(got, exact)
    banner(f"config 1 after {cfg.steps} steps vs closed form: max-rel {mr:.3e} L2-rel {lr:.3e}")
    assert lr < 0.15 and mr < 0.3


@pytest.mark.parametrize("name", ["tiny", "cfg1", "r65", "w5_slab"])
def test_nodes_and_weights_match_oracle(name):
    # the host tables behind sp6_get_nodes / sp6_get_weights against the oracle's
    # grid (CGL, half-shifted and equispaced nodes; Clenshaw-Curtis, Fejer and
    # trapezoid weights)
    cfg = SHAPES[name]
    G = make(cfg)
    g = oracle_grid(cfg)
    for got, want in zip(G.nodes(), (g.r, g.theta, g.phi, g.Theta, g.Phi)):
        np.testing.assert_allclose(got, want, rtol=0, atol=4e-16 * np.max(np.abs(want)))
    wr, wth, wph, wTh, wPh = G.weights()
    np.testing.assert_allclose(wr, g.w_r, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(wth, g.w_theta, rtol=1e-14)
    np.testing.assert_allclose(wTh, g.w_Theta, rtol=1e-14)
    np.testing.assert_allclose(wph, np.full(cfg.n_phi, 2 * np.pi / cfg.n_phi), rtol=1e-15)
    np.testing.assert_allclose(wPh, np.full(cfg.n_Phi, 2 * np.pi / cfg.n_Phi), rtol=1e-15)
