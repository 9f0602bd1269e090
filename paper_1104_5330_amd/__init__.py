"""MI355X-native hot path of the 6D spectral transport scheme of Bonazzola,
Vasset & Peres (2011): Liouville operator in doubly spherical coordinates,
linear collision term, inflow conditions and RK4, with its discrete adjoint.

The arithmetic lives in the HIP library libsp6d.so (C ABI in include/sp6d.h);
this package only marshals torch tensors into it.
"""

from ._lib import Sp6Error, SP6_FP64, SP6_MIXED  # noqa: F401
from .grid import Sp6Grid  # noqa: F401

__all__ = ["Sp6Grid", "Sp6Error", "SP6_FP64", "SP6_MIXED"]
