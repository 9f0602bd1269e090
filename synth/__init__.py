"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package only generates data: grid sizes, node positions at which fields
are sampled, initial distributions, coefficient fields and inflow planes.  It
contains none of the transport scheme's arithmetic (no derivatives, no
quadratures, no time stepping), so it can feed both the oracle and the GPU
path without either depending on the other.
"""

from .configs import WORKLOADS, Config, config  # noqa: F401
from . import fields  # noqa: F401
