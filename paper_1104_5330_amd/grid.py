"""Python handle over the C ABI: argument marshalling only.

Every computation runs in the HIP library; this module checks that tensors are
FP64, contiguous and on the GPU, passes their device pointers, and runs each call
on torch's current HIP stream.
"""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Sp6Desc, check


def _ptr(t, name, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape) and t.numel() != int(np.prod(shape)):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Sp6Grid:
    """A grid handle (sp6_create) bound to one GPU.

    Shapes: states [n_eps, n_r, n_theta, n_phi, n_Theta, n_Phi]; coefficient fields
    [n_eps, n_r, n_theta, n_phi]; inflow planes [n_eps, n_theta, n_phi, n_Theta, n_Phi].
    filter: 0/False off, 1/True angular line filters, 2 angular and radial.
    """

    def __init__(self, n_eps, n_r, n_theta, n_phi, n_Theta, n_Phi, r_in=1.0, r_out=3.0,
                 precision="fp64", bc=True, scattering=True, filter=False, device=None):
        self.lib = _lib.load()
        self.desc = Sp6Desc(n_eps, n_r, n_theta, n_phi, n_Theta, n_Phi, float(r_in), float(r_out),
                            {"fp64": _lib.SP6_FP64, "mixed": _lib.SP6_MIXED}[precision], int(bool(bc)),
                            int(bool(scattering)), int(filter))
        self.shape = (n_eps, n_r, n_theta, n_phi, n_Theta, n_Phi)
        self.coef_shape = (n_eps, n_r, n_theta, n_phi)
        self.plane_shape = (n_eps, n_theta, n_phi, n_Theta, n_Phi)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.precision = precision
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self.lib.sp6_create(ctypes.byref(self.desc), self._stream(), ctypes.byref(self._h)))

    @classmethod
    def from_config(cls, cfg, **kw):
        return cls(cfg.n_eps, cfg.n_r, cfg.n_theta, cfg.n_phi, cfg.n_Theta, cfg.n_Phi, cfg.r_in, cfg.r_out, **kw)

    # -- plumbing ------------------------------------------------------------------
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _call(self, fn, *args):
        check(self.lib.sp6_set_stream(self._h, self._stream()))
        check(fn(self._h, *args))

    def close(self):
        if self._h:
            self.lib.sp6_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def empty(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    @property
    def points(self):
        return int(np.prod(self.shape))

    # -- tables --------------------------------------------------------------------
    def nodes(self):
        n = self.shape[1:]
        arrs = [np.zeros(k) for k in n]
        ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]
        check(self.lib.sp6_get_nodes(self._h, *ptrs))
        return tuple(arrs)

    def weights(self):
        n = self.shape[1:]
        arrs = [np.zeros(k) for k in n]
        ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]
        check(self.lib.sp6_get_weights(self._h, *ptrs))
        return tuple(arrs)

    def device_bytes(self):
        b = ctypes.c_size_t()
        check(self.lib.sp6_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    # -- setup -----------------------------------------------------------------------
    def set_coefficients(self, kappa, sigma, eta):
        s = self.coef_shape
        self._call(self.lib.sp6_set_coefficients, _ptr(kappa, "kappa", s), _ptr(sigma, "sigma", s),
                   _ptr(eta, "eta", s))

    def set_scattering_kernel(self, c1=0.0, c2=0.0):
        """Phase function p(mu) = (1 - c2/3) + c1 mu + c2 mu^2 of the scattering term
        (isotropic by default; Thomson is c1 = 0, c2 = 3/4)."""
        self._call(self.lib.sp6_set_scattering_kernel, ctypes.c_double(c1), ctypes.c_double(c2))

    def set_energy_coupling(self, gamma_min=0.0, gamma_max=1.0, alpha=0.0, enable=True):
        """Fokker-Planck energy coupling (Eq. Transpfp): the groups become the
        Chebyshev nodes of gamma on [gamma_min, gamma_max]; enable=False turns it off."""
        self._call(self.lib.sp6_set_energy_coupling, ctypes.c_int32(1 if enable else 0), ctypes.c_double(gamma_min),
                   ctypes.c_double(gamma_max), ctypes.c_double(alpha))

    def set_inflow(self, g_in=None, g_out=None):
        s = self.plane_shape
        self._call(self.lib.sp6_set_inflow, _ptr(g_in, "g_in", s), _ptr(g_out, "g_out", s))

    def project_inflow(self, F):
        self._call(self.lib.sp6_project_inflow, _ptr(F, "F", self.shape))
        return F

    # -- operators ------------------------------------------------------------------
    def apply_L(self, F, out=None):
        out = self.empty() if out is None else out
        self._call(self.lib.sp6_apply_L, _ptr(F, "F", self.shape), _ptr(out, "out", self.shape))
        return out

    def apply_L_terms(self, mask, F, out=None):
        out = self.empty() if out is None else out
        self._call(self.lib.sp6_apply_L_terms, ctypes.c_uint32(mask), _ptr(F, "F", self.shape),
                   _ptr(out, "out", self.shape))
        return out

    def apply_LT(self, G, out=None):
        out = self.empty() if out is None else out
        self._call(self.lib.sp6_apply_LT, _ptr(G, "G", self.shape), _ptr(out, "out", self.shape))
        return out

    def rhs(self, F, out=None):
        out = self.empty() if out is None else out
        self._call(self.lib.sp6_rhs, _ptr(F, "F", self.shape), _ptr(out, "out", self.shape))
        return out

    def step(self, F, dt, nsteps=1):
        self._call(self.lib.sp6_step, _ptr(F, "F", self.shape), ctypes.c_double(dt), ctypes.c_int32(nsteps))
        return F

    def step_noalloc(self, F, dt, nsteps=1):
        """step() with its scratch in the library's fixed per-GPU array (no device
        allocation; grids of up to SP6_NOALLOC_SCRATCH_BYTES / 24 points FP64, / 16
        mixed; concurrent calls on one GPU race)."""
        self._call(self.lib.sp6_step_noalloc, _ptr(F, "F", self.shape), ctypes.c_double(dt), ctypes.c_int32(nsteps))
        return F

    def step_radial_implicit(self, F, dt, nsteps=1):
        """Split steps in place on F: RK4 on the angular and collision terms, then
        a backward-Euler radial step (no radial step limit)."""
        self._call(self.lib.sp6_step_radial_implicit, _ptr(F, "F", self.shape), ctypes.c_double(dt),
                   ctypes.c_int32(nsteps))
        return F

    KERNEL_CLASSES = ("phi", "theta", "radial", "plane", "filter", "thetaphi", "energy")

    def step_timed(self, F, dt, nsteps=1):
        """step() with per-kernel HIP-event timing; returns {class: (ms_total, launches)}."""
        ms = (ctypes.c_double * len(self.KERNEL_CLASSES))()
        n = (ctypes.c_int64 * len(self.KERNEL_CLASSES))()
        self._call(self.lib.sp6_step_timed, _ptr(F, "F", self.shape), ctypes.c_double(dt), ctypes.c_int32(nsteps),
                   ms, n)
        return {c: (ms[i], n[i]) for i, c in enumerate(self.KERNEL_CLASSES)}

    def step_ab2(self, F, H, dt, nsteps=1, start=True):
        """Adams-Bashforth steps in place on F; H carries the history between calls
        (start=True: forward-Euler first step, H initialised)."""
        self._call(self.lib.sp6_step_ab2, _ptr(F, "F", self.shape), _ptr(H, "H", self.shape), ctypes.c_double(dt),
                   ctypes.c_int32(nsteps), ctypes.c_int32(1 if start else 0))
        return F

    def step_stages(self, F, dt, Ystages):
        """One RK4 step in place on F that also writes its stage inputs Y2, Y3, Y4
        into Ystages (shape (3,) + state shape)."""
        self._call(self.lib.sp6_step_stages, _ptr(F, "F", self.shape), ctypes.c_double(dt),
                   _ptr(Ystages, "Ystages", (3,) + self.shape))
        return F

    def adjoint_step_stages(self, F_n, Ystages, dt, lam, grad_kappa=None, grad_eta=None, grad_sigma=None):
        """adjoint_step reading the step's stage inputs from step_stages."""
        s = self.coef_shape
        self._call(self.lib.sp6_adjoint_step_stages, _ptr(F_n, "F_n", self.shape),
                   _ptr(Ystages, "Ystages", (3,) + self.shape), ctypes.c_double(dt), _ptr(lam, "lam", self.shape),
                   _ptr(grad_kappa, "grad_kappa", s), _ptr(grad_eta, "grad_eta", s), _ptr(grad_sigma, "grad_sigma", s))
        return lam

    def adjoint_step(self, F_n, dt, lam, grad_kappa=None, grad_eta=None, grad_sigma=None):
        s = self.coef_shape
        self._call(self.lib.sp6_adjoint_step, _ptr(F_n, "F_n", self.shape), ctypes.c_double(dt),
                   _ptr(lam, "lam", self.shape), _ptr(grad_kappa, "grad_kappa", s),
                   _ptr(grad_eta, "grad_eta", s), _ptr(grad_sigma, "grad_sigma", s))
        return lam

    def apply_filter(self, F):
        self._call(self.lib.sp6_apply_filter, _ptr(F, "F", self.shape))
        return F

    def diagnostics(self, F):
        n = self.shape[0]
        N, Ji, Jo = np.zeros(n), np.zeros(n), np.zeros(n)
        dp = ctypes.POINTER(ctypes.c_double)
        self._call(self.lib.sp6_diagnostics, _ptr(F, "F", self.shape), N.ctypes.data_as(dp),
                   Ji.ctypes.data_as(dp), Jo.ctypes.data_as(dp))
        return N, Ji, Jo

    def outgoing_flux(self, F, out=None):
        s = (self.shape[0], self.shape[2], self.shape[3])
        out = torch.empty(s, dtype=torch.float64, device=self.device) if out is None else out
        self._call(self.lib.sp6_outgoing_flux, _ptr(F, "F", self.shape), _ptr(out, "j", s))
        return out

    def outgoing_flux_T(self, jbar, out=None):
        s = (self.shape[0], self.shape[2], self.shape[3])
        out = self.empty() if out is None else out
        self._call(self.lib.sp6_outgoing_flux_T, _ptr(jbar, "jbar", s), _ptr(out, "out", self.shape))
        return out
