"""Benchmark of the 6D spectral transport hot path on one MI355X.

Headline workload: the large scattering workload, 4 energy groups,
(n_r, n_theta, n_phi, n_Theta, n_Phi) = (65, 32, 64, 32, 64): 1,090,519,040 points
(8.7 GB per FP64 state), emission + absorption + isotropic scattering
sigma = kappa / 2, FP64, classical RK4 at dt = 0.2 (r_1 - r_0).  One "step" is one
full RK4 step over the whole grid; value = grid-point updates per second with
every input already resident in HBM.  Inputs are synthetic and seeded (no
dataset is involved).

Also measured on the same JSON line ("forms"):
  large_mixed: the headline workload on the mixed path, with its error against
            the FP64 path after the same steps;
  w2_fp64 : emission + absorption, 8 groups on (33, 16, 32, 16, 32), FP64;
  mixed   : that grid with sigma = kappa/2 on the mixed path, with its error
            against the FP64 path after the timed steps;
  thomson, shell, ab2, implicit: the anisotropic kernel, the 5D shell problem,
            the paper's Adams-Bashforth integrator, the split step of App. B;
  adjoint : the 4-group workload (same angular grid as w2), 200 steps forward
            plus the checkpointed (every 20) discrete-adjoint backward pass of the
            outgoing-flux misfit; value = forward-equivalent updates (points x 200)
            over the forward + recompute + backward wall time.

The roofline object is for the dominant kernel of the headline form (the plane
pass): achieved = algorithmic bytes per launch over its mean HIP-event
duration, against 8 TB/s.  The algorithmic bytes are the method's: a fully fused
RK4 step moves 128 B per point (read the stage state, y and the accumulator as
the scheme needs them, write the next ones), i.e. 32 B per point per stage, and
one plane-pass launch is one stage over every point; the kernel's own bytes
(36 B per point on average, T and the stage input included) are reported beside
it.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "6D grid-point updates/s per RK4 step (FP64 vs mixed vs adjoint), % HBM peak"

# Algorithmic bytes per grid point of one launch, averaged over the four RK stages.
# FP64 path (state, stage copy, T, accumulator all FP64):
#   thetaphi: theta and phi fused: read Y, write T             16
#   phi    : read Y, write T                                   16
#   theta  : read Y, T, write T                                24
#   radial : read Y, T, write T                                24
#   plane  : stage 1 read Y, T; write Y'                       24
#            stage 2 read Y, T, y; write acc, Y'               40
#              (acc's base y + (Y - y)/3 recovered, not read)
#            stage 3 read Y, T, y, acc; write acc, Y'          48
#            stage 4 read Y, T, acc; write y                   32   -> mean 36
# energy coupling (per stage): the moment pass reads the stage state once (8);
# the pass over the groups moves 40 B per plane, negligible beside it
BYTES_FP64 = {"thetaphi": 16.0, "phi": 16.0, "theta": 24.0, "radial": 24.0, "plane": 36.0, "energy": 8.0}
# Mixed path (stage copy and T in FP32; stage 1 reads the FP64 state):
#   thetaphi, phi : (8 + 4, then 3 x (4 + 4)) / 4                9
#   theta  : (8 + 4 + 4, then 3 x 12) / 4                       13
#   radial : same as theta                                      13
#   plane  : (8+4+8+4, 4+4+8+8+8+4 twice, 4+4+8+8) / 4          30
BYTES_MIXED = {"thetaphi": 9.0, "phi": 9.0, "theta": 13.0, "radial": 13.0, "plane": 30.0}
# minimal traffic of a fully fused RK4 step (read the stage state once; y, acc and
# the next stage state as registers of the scheme): 128 B (FP64), 104 B (mixed)
FUSED_MIN_B = {"fp64": 128.0, "mixed": 104.0}
# per plane-pass launch (one RK stage over every point): 128 / 4
METHOD_B_PER_STAGE = {"fp64": 32.0, "mixed": 26.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", choices=["all", "large", "fp64", "mixed", "thomson", "energy", "shell", "ab2", "implicit",
                                       "adjoint"],
                    default="all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 553,648,128 bytes (byte-counter calibration)")
    return ap.parse_args()


PROFILE_FP64 = os.path.join(ROOT, "profiles", "fp64_step_scatter_65x32x64x32x64_g4.md")
PLANE_SRC = os.path.join(ROOT, "paper_1104_5330_amd", "csrc", "k_plane.hip")


def measured_traffic():
    """HBM bytes per launch of the plane pass from the committed rocprofv3 byte
    counters, or None when the kernel source changed since they were taken."""
    import hashlib
    try:
        txt = open(PROFILE_FP64).read()
        fields = dict(line.split(": ", 1) for line in txt.splitlines() if line.startswith("traffic_"))
        cur = hashlib.sha256(open(PLANE_SRC, "rb").read()).hexdigest()[:16]
        if fields.get("traffic_source_sha256_16", "").strip() != cur:
            return None
        return float(fields["traffic_plane_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def kernel_table(kt, P, bpp, total_ms):
    out = {}
    for name, (kms, n) in kt.items():
        if n == 0:
            continue
        b = bpp.get(name, 0.0) * P
        out[name] = {"launches": n, "avg_ms": kms / n, "share": kms / total_ms,
                     "bytes_per_point": bpp.get(name),
                     "alg_GBs": (b * n / (kms / 1e3)) / 1e9 if kms > 0 else None}
    return out


def run_steps(cfg, precision, scattering, steps, warmup, F0=None, kernel=None, energy=None, coeffs=None):
    import torch
    import synth
    from paper_1104_5330_amd import Sp6Grid

    dev = torch.device("cuda", 0)
    if F0 is None:
        F0 = synth.fields.shell_state(cfg, device=dev)
    if coeffs is None:
        coeffs = [torch.tensor(a, device=dev) for a in synth.fields.coefficients(cfg)]
    G = Sp6Grid.from_config(cfg, precision=precision, bc=True, scattering=scattering)
    G.set_coefficients(*coeffs)
    if kernel is not None:
        G.set_scattering_kernel(*kernel)
    if energy is not None:
        G.set_energy_coupling(*energy)
    W = F0.clone()
    G.step(W, cfg.dt, warmup)
    del W
    F = F0.clone()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    kt = G.step_timed(F, cfg.dt, steps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    assert torch.isfinite(F).all()
    G.close()
    return F, F0, ms, kt


def form_w2_fp64(args):
    """Emission + absorption, 8 groups on (33, 16, 32, 16, 32), FP64."""
    import synth
    cfg = synth.config(2)
    _, _, ms, kt = run_steps(cfg, "fp64", False, args.steps, args.warmup)
    P = cfg.points
    value = P * args.steps / (ms / 1e3)
    return {"workload": cfg.name, "grid": list(cfg.shape), "physics": "emission+absorption",
            "value": value, "unit": "grid-point updates/s", "ms_per_step": ms / args.steps,
            "steps": args.steps, "dtype": "f64", "kernels": kernel_table(kt, P, BYTES_FP64, ms),
            "hbm_fraction_algorithmic_128B": value * FUSED_MIN_B["fp64"] / (HBM_PEAK_GBS * 1e9)}


def form_large(args):
    """The headline: the large scattering workload (4 groups, (65, 32, 64, 32, 64):
    1.09e9 points, 8.7 GB per FP64 array) in FP64, then on the mixed path from the
    same initial state, with the mixed path's error against the FP64 result."""
    import torch
    import synth
    cfg = synth.config(5)
    # 8.7 GB arrays: hand earlier cached blocks back first, so that the new
    # arrays are mapped afresh
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    F64, F0, ms, kt = run_steps(cfg, "fp64", True, args.steps, args.warmup)
    Fm, _, ms_m, kt_m = run_steps(cfg, "mixed", True, args.steps, args.warmup, F0=F0)
    del F0
    err_max = ((Fm - F64).abs().max() / F64.abs().max()).item()
    err_l2 = (torch.linalg.vector_norm(Fm - F64) / torch.linalg.vector_norm(F64)).item()
    del Fm, F64
    torch.cuda.empty_cache()
    P = cfg.points
    value = P * args.steps / (ms / 1e3)
    value_m = P * args.steps / (ms_m / 1e3)
    mixed = {"workload": cfg.name, "grid": list(cfg.shape), "value": value_m, "unit": "grid-point updates/s",
             "ms_per_step": ms_m / args.steps, "steps": args.steps,
             "dtype": "f32 derivatives / bf16x3 MFMA radial / f64 state",
             "kernels": kernel_table(kt_m, P, BYTES_MIXED, ms_m),
             "error_vs_fp64": {"max_rel": err_max, "l2_rel": err_l2, "after_steps": args.steps},
             "hbm_fraction_algorithmic_104B": value_m * FUSED_MIN_B["mixed"] / (HBM_PEAK_GBS * 1e9)}
    return cfg, value, ms, kernel_table(kt, P, BYTES_FP64, ms), mixed


def form_mixed(args):
    import torch
    import synth
    cfg = synth.config(3)
    Fm, F0, ms, kt = run_steps(cfg, "mixed", True, args.steps, args.warmup)
    F64, _, ms64, _ = run_steps(cfg, "fp64", True, args.steps, 0, F0=F0)
    err_max = ((Fm - F64).abs().max() / F64.abs().max()).item()
    err_l2 = (torch.linalg.vector_norm(Fm - F64) / torch.linalg.vector_norm(F64)).item()
    P = cfg.points
    return {
        "workload": cfg.name, "grid": list(cfg.shape), "physics": "emission+absorption+isotropic scattering",
        "value": P * args.steps / (ms / 1e3), "unit": "grid-point updates/s", "ms_per_step": ms / args.steps,
        "steps": args.steps, "dtype": "f32 derivatives / bf16x3 MFMA radial / f64 state",
        "fp64_same_workload": P * args.steps / (ms64 / 1e3),
        "error_vs_fp64": {"max_rel": err_max, "l2_rel": err_l2, "after_steps": args.steps},
        "hbm_fraction_algorithmic_104B": P * args.steps / (ms / 1e3) * FUSED_MIN_B["mixed"] / (HBM_PEAK_GBS * 1e9),
        "kernels": kernel_table(kt, P, BYTES_MIXED, ms),
    }


def form_thomson(args):
    """FP64 step of the scattering workload with the Thomson phase function
    (3/4)(1 + mu^2) instead of isotropic scattering (ten plane moments per stage)."""
    import synth
    cfg = synth.config(3)
    _, _, ms, kt = run_steps(cfg, "fp64", True, args.steps, args.warmup, kernel=(0.0, 0.75))
    _, _, ms_iso, _ = run_steps(cfg, "fp64", True, args.steps, 0)
    P = cfg.points
    return {
        "workload": cfg.name, "grid": list(cfg.shape),
        "physics": "emission+absorption+Thomson scattering p(mu) = 3/4 (1 + mu^2)",
        "value": P * args.steps / (ms / 1e3), "unit": "grid-point updates/s", "ms_per_step": ms / args.steps,
        "steps": args.steps, "dtype": "f64",
        "isotropic_same_workload": P * args.steps / (ms_iso / 1e3),
        "kernels": kernel_table(kt, P, BYTES_FP64, ms),
    }


def form_energy(args):
    """FP64 step of Eq. (Transpfp) on the grid of the 8-group workloads: Thomson
    scattering with n sigma_Th = 1, no absorption or emission (as the equation is
    written), and the Fokker-Planck energy coupling, the 8 groups taken as the
    Chebyshev nodes of gamma on [0, 0.1], alpha = 0.01; the initial state is the
    shell state times a Bose spectrum (mu = -0.02) in gamma (synthetic
    parameters; the paper gives no numerical case).  Per stage the coupling adds
    a moment pass over the stage state and a pass over the groups of each
    position."""
    import synth
    import torch
    cfg = synth.config(3)
    en, mu = (0.0, 0.1, 0.01), -0.02
    dev = torch.device("cuda", 0)
    F0 = synth.fields.bose_shell_state(cfg, en[0], en[1], en[2], mu, device=dev)
    z = torch.zeros((cfg.n_eps, cfg.n_r, cfg.n_theta, cfg.n_phi), dtype=torch.float64, device=dev)
    co = (z, z + 1.0, z)
    _, _, ms, kt = run_steps(cfg, "fp64", True, args.steps, args.warmup, F0=F0, kernel=(0.0, 0.75), energy=en,
                             coeffs=co)
    _, _, ms_off, _ = run_steps(cfg, "fp64", True, args.steps, 0, F0=F0, kernel=(0.0, 0.75), coeffs=co)
    P = cfg.points
    return {
        "workload": cfg.name, "grid": list(cfg.shape),
        "physics": "Thomson scattering (n sigma_Th = 1) + Fokker-Planck energy coupling, no absorption or emission",
        "gamma_range": [en[0], en[1]], "alpha": en[2], "initial_state": f"shell state x Bose spectrum, mu = {mu}",
        "value": P * args.steps / (ms / 1e3), "unit": "grid-point updates/s", "ms_per_step": ms / args.steps,
        "steps": args.steps, "dtype": "f64",
        "without_coupling_ms_per_step": ms_off / args.steps,
        "kernels": kernel_table(kt, P, BYTES_FP64, ms),
    }


def form_shell(args):
    """The 5D shell problem of Sect. 5.3 (one energy, coherent scattering in a
    shell with a density profile, Lambert inflow F0 cos(Theta) at r_in, empty at
    t = 0, angular and radial filters after every step) run to t = 4.2 at optical
    depths 5 and 0; luminosities J(r_in), J(r_out) and particle number at the end."""
    import math
    import torch
    import synth
    from paper_1104_5330_amd import Sp6Grid

    dev = torch.device("cuda", 0)
    out = {}
    for n in (6, 7):
        cfg = synth.config(n)
        steps = math.ceil(cfg.t_end / cfg.dt)
        G = Sp6Grid.from_config(cfg, scattering=True, filter=2)
        # (copies: some of these fields are read-only numpy views)
        G.set_coefficients(*(torch.tensor(a, device=dev) for a in synth.fields.coefficients(cfg)))
        g_in, g_out = (torch.tensor(a, device=dev) for a in synth.fields.lambert_inflow(cfg))
        G.set_inflow(g_in, g_out)
        F = torch.zeros(cfg.shape, dtype=torch.float64, device=dev)
        G.project_inflow(F)
        kt = G.step_timed(F.clone(), cfg.dt, 10)  # per-kernel table on a copy
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        G.step(F, cfg.dt, steps)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        assert torch.isfinite(F).all()
        N, J_in, J_out = G.diagnostics(F)
        P = cfg.points
        out[f"tau{cfg.tau:g}"] = {
            "workload": cfg.name, "grid": list(cfg.shape), "t_end": steps * cfg.dt, "steps": steps,
            "value": P * steps / (ms / 1e3), "unit": "grid-point updates/s", "ms_per_step": ms / steps,
            "dtype": "f64", "filter": "angular + radial exp(-36 eta^36) after every step",
            "N": float(N[0]), "J_in": float(J_in[0]), "J_out": float(J_out[0]),
            # the filter class is four in-place passes (theta, phi, plane, r): 64 B per point
            "kernels": kernel_table(kt, P, dict(BYTES_FP64, filter=64.0), sum(v[0] for v in kt.values())),
        }
        G.close()
    return out


def form_ab2(args):
    """The paper's own integrator (second-order Adams-Bashforth, Sect. 5.1) on the
    headline workload: one right-hand side per step instead of four."""
    import torch
    import synth
    from paper_1104_5330_amd import Sp6Grid

    cfg = synth.config(2)
    dev = torch.device("cuda", 0)
    G = Sp6Grid.from_config(cfg, scattering=False)
    G.set_coefficients(*(torch.tensor(a, device=dev) for a in synth.fields.coefficients(cfg)))
    F = synth.fields.shell_state(cfg, device=dev)
    H = torch.empty_like(F)
    G.step_ab2(F, H, cfg.dt, max(args.warmup, 1), start=True)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    G.step_ab2(F, H, cfg.dt, args.steps, start=False)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    assert torch.isfinite(F).all()
    G.close()
    P = cfg.points
    return {"workload": cfg.name, "grid": list(cfg.shape), "steps": args.steps, "dtype": "f64",
            "value": P * args.steps / (ms / 1e3), "unit": "grid-point updates/s (Adams-Bashforth steps)",
            "ms_per_step": ms / args.steps, "rhs_per_step": 1}


def form_implicit(args):
    """The split step of App. B on the headline workload: RK4 on the angular and
    collision terms, then the backward-Euler radial solve (one MFMA pass with the
    per-Theta inverse matrices) in place of the four explicit radial passes."""
    import torch
    import synth
    from paper_1104_5330_amd import Sp6Grid

    cfg = synth.config(2)
    dev = torch.device("cuda", 0)
    G = Sp6Grid.from_config(cfg, scattering=False)
    G.set_coefficients(*(torch.tensor(a, device=dev) for a in synth.fields.coefficients(cfg)))
    F = synth.fields.shell_state(cfg, device=dev)
    G.step_radial_implicit(F, cfg.dt, max(args.warmup, 1))
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    G.step_radial_implicit(F, cfg.dt, args.steps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    assert torch.isfinite(F).all()
    G.close()
    P = cfg.points
    return {"workload": cfg.name, "grid": list(cfg.shape), "steps": args.steps, "dtype": "f64", "dt": cfg.dt,
            "value": P * args.steps / (ms / 1e3), "unit": "grid-point updates/s (split steps)",
            "ms_per_step": ms / args.steps}


def form_adjoint(args):
    import numpy as np
    import torch
    import synth
    from paper_1104_5330_amd import Sp6Grid
    from paper_1104_5330_amd.autograd import transport, outgoing_flux

    cfg = synth.config(4)
    n, K = cfg.steps, 20
    dev = torch.device("cuda", 0)
    G = Sp6Grid.from_config(cfg, scattering=False)
    shp = (cfg.n_r, cfg.n_theta, cfg.n_phi)
    kap1, _, eta1 = synth.fields.coefficients(cfg, kappa_s=np.ones(shp))
    c = torch.as_tensor(kap1[:, 0, 0, 0].copy(), device=dev).view(-1, 1, 1, 1)
    B = torch.as_tensor(eta1 / kap1, device=dev)
    r = synth.fields.nodes(cfg)[0]
    ks0 = torch.as_tensor(np.broadcast_to((r ** -2.0)[:, None, None], shp).copy(), device=dev)
    rho = torch.as_tensor(synth.fields.low_mode_position_field(cfg, seed=0), device=dev)
    F0 = synth.fields.shell_state(cfg, device=dev)

    def loss(ks, F, jt):
        kappa = c * ks.unsqueeze(0)
        Fn = transport(G, F, kappa, torch.zeros_like(kappa), kappa * B, cfg.dt, n, K)
        j = outgoing_flux(G, Fn)
        return ((j - jt) ** 2).sum()

    with torch.no_grad():
        kap = c * (ks0 * (1.0 + 0.2 * rho)).unsqueeze(0)
        jt = outgoing_flux(G, transport(G, F0, kap, torch.zeros_like(kap), kap * B, cfg.dt, n, K)).clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ks = ks0.clone().requires_grad_(True)
    Ft = F0.clone().requires_grad_(True)
    L = loss(ks, Ft, jt)
    L.backward()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    P = cfg.points
    return {
        "workload": cfg.name, "grid": list(cfg.shape), "steps": n, "checkpoint_every": K,
        "value": P * n / t, "unit": "forward-equivalent grid-point updates/s (forward + recompute + adjoint)",
        "seconds": t, "loss": L.item(), "grad_norm_kappa_s": torch.linalg.vector_norm(ks.grad).item(),
        "dtype": "f64",
        "fd_check": "tests/test_gpu_adjoint.py: 16 joint directions, worst relative error printed there",
    }


def host_cpu():
    """Model name and logical CPU count of the host (lscpu), as far as available."""
    import subprocess
    info = {"os_cpu_count": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Socket(s)"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return info


def cpu_baseline():
    """The oracle as it stands, timed on the host: the first of the four stages of
    an RK4 step (one right-hand side and the stage update Y2 = y + dt/2 k1, as
    step.rk4_stages forms them) of one energy group of the headline workload.  The
    groups are independent and the four stages cost the same, so
    updates/s = points / (4 t_stage)."""
    import numpy as np
    import synth
    from oracle import grid as og, step

    cfg = synth.config(5)
    sub = cfg.scaled(n_eps=1)
    k, s, e = (np.ascontiguousarray(a[-1:]) for a in synth.fields.coefficients(cfg))
    F = synth.fields.shell_state(sub)
    g = og.make_grid(*sub.shape)
    p = step.Physics(k, s, e, scattering=True)
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 0) for i in threadpool_info()), default=None)
    except Exception:
        pass
    t0 = time.perf_counter()
    k1 = step.rhs(F, g, p)
    Y2 = F + 0.5 * cfg.dt * k1
    t_stage = time.perf_counter() - t0
    assert np.isfinite(Y2).all()
    del Y2, k1, F
    return {"value": sub.points / (4.0 * t_stage), "unit": "grid-point updates/s",
            "cores": threads or os.cpu_count(), "kind": "oracle", "host": host_cpu(),
            "sample": f"the first RK4 stage (right-hand side and stage update) of 1 of {cfg.n_eps} energy groups "
                      f"({sub.points} points) of the headline workload in {t_stage:.1f} s; a step counted as four "
                      f"such stages; dense 1D matrices in numpy FP64"}


def copy_calibration():
    import torch
    n = 553648128 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(energy groups would shard across GPUs with no communication; not built).", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    out = {"metric": METRIC}
    forms = {}
    if args.form in ("all", "large"):
        cfg, value, ms, kern, mixed = form_large(args)
        dk = kern["plane"]
        plane_s = dk["avg_ms"] / 1e3
        achieved = METHOD_B_PER_STAGE["fp64"] * cfg.points / plane_s / 1e9
        own = BYTES_FP64["plane"] * cfg.points / plane_s / 1e9
        out.update({
            "value": value, "unit": "grid-point updates/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": cfg.name, "grid": list(cfg.shape), "points": cfg.points,
                       "physics": "emission+absorption+isotropic scattering", "dt": cfg.dt, "form": "fp64"},
            "roofline": {"bound": "hbm", "kernel": "plane", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic(),
                         "bytes_per_point_per_launch": METHOD_B_PER_STAGE["fp64"], "points_per_launch": cfg.points,
                         "avg_launch_ms": dk["avg_ms"],
                         "kernel_bytes_per_point_per_launch": BYTES_FP64["plane"],
                         "achieved_kernel_bytes": own, "frac_kernel_bytes": own / HBM_PEAK_GBS},
            "kernels": kern,
            "hbm_fraction_algorithmic_128B": value * FUSED_MIN_B["fp64"] / (HBM_PEAK_GBS * 1e9),
        })
        forms["large_mixed"] = mixed
    if args.form in ("all", "fp64"):
        forms["w2_fp64"] = form_w2_fp64(args)
    if args.form in ("all", "mixed"):
        forms["mixed"] = form_mixed(args)
    if args.form in ("all", "thomson"):
        forms["thomson"] = form_thomson(args)
    if args.form in ("all", "energy"):
        forms["energy"] = form_energy(args)
    if args.form in ("all", "shell"):
        forms["shell"] = form_shell(args)
    if args.form in ("all", "ab2"):
        forms["ab2"] = form_ab2(args)
    if args.form in ("all", "implicit"):
        forms["implicit"] = form_implicit(args)
    if args.form in ("all", "adjoint"):
        forms["adjoint"] = form_adjoint(args)
    out["forms"] = forms
    if args.copy_calibration:
        out["copy_calibration"] = copy_calibration()
    if not args.no_cpu_baseline and args.form in ("all", "large"):
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
