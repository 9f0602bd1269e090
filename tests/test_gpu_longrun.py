"""Long runs against the FP64 oracle at the workload's real grid.

The scattering workload (8 groups on (33, 16, 32, 16, 32), sigma = kappa / 2) has
independent energy groups (coherent scattering, Eq. sigmadif), so one group
advanced alone on the GPU is that group of the full run.  Its highest-energy
group (eps = 100: the largest opacities) is advanced 100 RK4 steps by the FP64
path, the mixed path and the oracle; the FP64 path is gated at 1e-12 and the
mixed path at its stated 1e-5, both normwise relative (max |a - b| / max |b|),
and both errors are printed with the L2-relative error.  The oracle takes about
two minutes on 16 host threads.
"""

import time

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og, step
from tests.gpu_util import need_gpu, maxrel, l2rel, to_dev, to_host, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


@pytest.mark.timeout(900)
def test_workload3_top_group_100_steps_vs_oracle():
    from paper_1104_5330_amd import Sp6Grid
    full = synth.config(3)
    grp = full.n_eps - 1
    sub = full.scaled(n_eps=1)
    k, s, e = (np.ascontiguousarray(a[grp:grp + 1]) for a in synth.fields.coefficients(full))
    F0 = synth.fields.shell_state(sub)
    n = full.steps
    res = {}
    for prec in ("fp64", "mixed"):
        G = Sp6Grid.from_config(sub, precision=prec, scattering=True)
        G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
        Fd = to_dev(F0)
        G.step(Fd, full.dt, n)
        res[prec] = to_host(Fd)
        G.close()
    banner(f"oracle: {n} RK4 steps of group {grp} (eps = {full.eps[grp]:g}) of {full.name}")
    t0 = time.perf_counter()
    g = og.make_grid(*sub.shape)
    want = step.run(F0, g, step.Physics(k, s, e, scattering=True), full.dt, n)
    banner(f"oracle done in {time.perf_counter() - t0:.0f} s")
    e64 = (maxrel(res["fp64"], want), l2rel(res["fp64"], want))
    emx = (maxrel(res["mixed"], want), l2rel(res["mixed"], want))
    banner(f"{full.name} group {grp}, {n} steps: FP64 max-rel {e64[0]:.3e} L2-rel {e64[1]:.3e}; "
           f"mixed max-rel {emx[0]:.3e} L2-rel {emx[1]:.3e}")
    assert e64[0] <= 1e-12
    assert emx[0] <= 1e-5
