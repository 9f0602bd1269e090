"""Benchmark of the 6D spectral transport hot path on one MI355X.

Workload: emission + absorption, 8 energy groups,
(n_r, n_theta, n_phi, n_Theta, n_Phi) = (33, 16, 32, 16, 32): 69,206,016 points,
FP64, RK4 at dt = 0.2 (r_1 - r_0).  One "step" is one full RK4 step over the
whole grid; value = grid-point updates per second with every input resident in
HBM.  Synthetic seeded inputs (no dataset is involved).

Prints one JSON line with the headline metric, the roofline of the dominant
kernel (algorithmic bytes / HIP-event duration) and the CPU oracle baseline.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per grid point of one launch of each kernel class (FP64):
#   phi    : read Y, write T                          16
#   theta  : read Y, read T, write T                  24
#   radial : read Y, read T, write T                  24
#   plane  : stage 1 read Y, T; write acc, Y'         32
#            stages 2-3 read Y, T, y, acc; write acc, Y'   48
#            stage 4 read Y, T, acc; write y          32   -> mean 40 per launch
BYTES_PER_POINT = {"phi": 16.0, "theta": 24.0, "radial": 24.0, "plane": 40.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    return ap.parse_args()


def cpu_baseline(cfg, nsteps):
    """The oracle as it stands, timed on the host: nsteps RK4 steps of one energy
    group of the workload (the groups are independent)."""
    import numpy as np
    import synth
    from oracle import grid as og, step

    sub = cfg.scaled(n_eps=1)
    F = synth.fields.shell_state(sub)
    k, s, e = synth.fields.coefficients(sub)
    g = og.make_grid(*sub.shape)
    p = step.Physics(k, s, e, scattering=sub.physics == "scatter")
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 0) for i in threadpool_info()), default=None)
    except Exception:
        pass
    t0 = time.perf_counter()
    y = F
    for _ in range(nsteps):
        y = step.rk4_step(y, g, p, sub.dt)
    t = time.perf_counter() - t0
    assert np.isfinite(y).all()
    return {"value": sub.points * nsteps / t, "unit": "grid-point updates/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"{nsteps} RK4 steps of 1 of {cfg.n_eps} energy groups ({sub.points} points), "
                      f"dense 1D matrices in numpy FP64, {t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(energy groups would shard across GPUs with no communication; not built).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_1104_5330_amd import Sp6Grid

    cfg = synth.config(2)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    F0 = synth.fields.shell_state(cfg, device=dev)
    k, s, e = (torch.as_tensor(a, device=dev) for a in synth.fields.coefficients(cfg))
    G = Sp6Grid.from_config(cfg, precision="fp64", bc=True, scattering=False)
    G.set_coefficients(k, s, e)
    F = F0.clone()
    G.step(F, cfg.dt, args.warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    kt = G.step_timed(F, cfg.dt, args.steps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    assert torch.isfinite(F).all()
    P = cfg.points
    value = P * args.steps / (ms / 1e3)

    kernels = {}
    for name, (kms, n) in kt.items():
        if n == 0:
            continue
        b = BYTES_PER_POINT.get(name, 0.0) * P
        kernels[name] = {"launches": n, "avg_ms": kms / n, "share": kms / ms,
                         "alg_GBs": (b * n / (kms / 1e3)) / 1e9 if kms > 0 else None}
    dom = max(kernels, key=lambda c: kt[c][0])
    dk = kernels[dom]
    roof = {"bound": "hbm", "kernel": dom, "achieved": dk["alg_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dk["alg_GBs"] / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_point_per_launch": BYTES_PER_POINT[dom], "points_per_launch": P}

    out = {
        "metric": "6D grid-point updates/s per RK4 step (FP64 vs mixed vs adjoint), % HBM peak",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "grid": list(cfg.shape), "points": P, "physics": "emission+absorption",
                   "dt": cfg.dt, "form": "fp64"},
        "roofline": roof,
        "kernels": kernels,
        "hbm_fraction_algorithmic_128B": value * 128.0 / (HBM_PEAK_GBS * 1e9),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
