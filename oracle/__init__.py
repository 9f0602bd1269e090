"""Plain FP64 CPU oracle for the 6D spectral transport hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU path.

What it computes (Bonazzola, Vasset & Peres 2011, "Solving the transport
equation by the use of 6D spectral methods in spherical coordinates"):

* the transport equation dF/dt + L_sph F = CT (Sect. 2, Eqs. Tra1/Transpfpsph),
  with c = 1;
* the Liouville operator in doubly spherical coordinates (Sect. 4.1,
  Eq. Liouvsph), discretised by collocation: Chebyshev-Gauss-Lobatto in r and
  Fourier in the four angles, theta and Theta on double-Fourier-sphere (DFS)
  lines;
* the linear, coherent, isotropic collision term (Sect. 2.2 Eq. Transp with
  Sect. 3.1 Eqs. sigmadif and sigman at B = 0): emission, absorption and
  isotropic scattering;
* inflow boundary conditions from the characteristic analysis of Sect. 4.2
  (Eq. Sphedif);
* classical RK4 in time, its discrete adjoint, an optional exponential
  filter and the particle-number / flux diagnostics of App. A (Eqs. Npho,
  Flux, Cons);
* optionally, the Fokker-Planck energy coupling of Sect. 3.2 (Eq. Transpfp)
  on a Chebyshev energy axis (energy.py).

Every 1D transform is an explicit dense matrix applied along one axis, with no
FFT, no blocking and no fusion, so that each function can be checked against
the paper by eye.  Readings of the paper where it is silent or garbled are
listed in each function's docstring.
"""

from .grid import Grid, make_grid  # noqa: F401
from . import ops, step, adjoint, diagnostics, closed_forms, conservative, energy  # noqa: F401
