"""Workload definitions: grid sizes, energy groups, physics switches, step counts.

Five workloads, all on the shell 1 <= r <= 3:

1. free streaming in vacuum, one group, (n_r, n_theta, n_phi, n_Theta, n_Phi)
   = (17, 8, 16, 8, 16), 10 steps;
2. emission + absorption, 8 groups, (33, 16, 32, 16, 32), 100 steps;
3. workload 2 plus isotropic scattering sigma = kappa / 2 (mixed precision);
4. adjoint of the outgoing-flux misfit, 4 groups, (33, 16, 32, 16, 32),
   200 steps, checkpoints every 20;
5. large: (65, 32, 64, 32, 64), 4 groups, scattering, 50 steps;
6, 7. the 5D shell of Sect. 5.3: one energy (coherent scattering only),
   (33, 16, 32, 16, 32), scattering opacity from the density profile, Lambert
   inflow F0 cos(Theta) at r_in, an empty shell at t = 0, up to t = 4.2;
   scattering optical depth 5 (6) and 0 (7).

The time step is 0.2 times the first radial spacing of the
Chebyshev-Gauss-Lobatto grid (the paper's radial stability limit scales as
(R2 - R1) / N_r^2, Sect. 5.4).
"""

from dataclasses import dataclass, replace
import math


@dataclass(frozen=True)
class Config:
    name: str
    n_eps: int
    n_r: int
    n_theta: int
    n_phi: int
    n_Theta: int
    n_Phi: int
    steps: int
    physics: str  # "vacuum" | "emit_abs" | "scatter" | "shell"
    r_in: float = 1.0
    r_out: float = 3.0
    T0: float = 10.0
    kappa0: float = 1.0
    tau: float = 0.0        # "shell": radial scattering optical depth of the shell
    F0: float = 1.0         # "shell": Lambert inflow amplitude
    t_end: float = 0.0      # "shell": physical end time (steps = ceil(t_end / dt))

    @property
    def shape(self):
        return (self.n_eps, self.n_r, self.n_theta, self.n_phi, self.n_Theta, self.n_Phi)

    @property
    def points(self):
        return math.prod(self.shape)

    @property
    def dt(self):
        """0.2 (r_1 - r_0) on the Chebyshev-Gauss-Lobatto grid."""
        dr = 0.5 * (self.r_out - self.r_in) * (1.0 - math.cos(math.pi / (self.n_r - 1)))
        return 0.2 * dr

    @property
    def eps(self):
        """Energy groups, logarithmic in [1, 100] with both ends included
        (a single group sits at eps = 1)."""
        if self.n_eps == 1:
            return [1.0]
        return [100.0 ** (k / (self.n_eps - 1)) for k in range(self.n_eps)]

    def scaled(self, **kw):
        return replace(self, **kw)


WORKLOADS = {
    1: Config("vacuum_17x8x16x8x16", 1, 17, 8, 16, 8, 16, 10, "vacuum"),
    2: Config("emit_abs_33x16x32x16x32_g8", 8, 33, 16, 32, 16, 32, 100, "emit_abs"),
    3: Config("scatter_33x16x32x16x32_g8", 8, 33, 16, 32, 16, 32, 100, "scatter"),
    4: Config("adjoint_33x16x32x16x32_g4", 4, 33, 16, 32, 16, 32, 200, "emit_abs"),
    5: Config("scatter_65x32x64x32x64_g4", 4, 65, 32, 64, 32, 64, 50, "scatter"),
    6: Config("shell5d_tau5_33x16x32x16x32", 1, 33, 16, 32, 16, 32, 4362, "shell", tau=5.0, t_end=4.2),
    7: Config("shell5d_tau0_33x16x32x16x32", 1, 33, 16, 32, 16, 32, 4362, "shell", tau=0.0, t_end=4.2),
}


def config(n):
    return WORKLOADS[n]
