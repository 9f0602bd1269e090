"""ctypes declarations of the C ABI in include/sp6d.h (libsp6d.so, built in-tree).

Loading fails loudly when the library has not been built: there is no fallback.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsp6d.so")

SP6_OK, SP6_ERR_ARG, SP6_ERR_SHAPE, SP6_ERR_ALLOC, SP6_ERR_HIP, SP6_ERR_STATE = range(6)
SP6_FP64, SP6_MIXED = 0, 1
SP6_NOALLOC_SCRATCH_BYTES = 256 << 20
STATUS_NAMES = {0: "SP6_OK", 1: "SP6_ERR_ARG", 2: "SP6_ERR_SHAPE", 3: "SP6_ERR_ALLOC", 4: "SP6_ERR_HIP",
                5: "SP6_ERR_STATE"}

# the exported entry points, in header order
SYMBOLS = [
    "sp6_validate_desc", "sp6_create", "sp6_destroy", "sp6_set_stream", "sp6_last_error",
    "sp6_get_nodes", "sp6_get_weights", "sp6_set_coefficients", "sp6_set_scattering_kernel", "sp6_set_energy_coupling",
    "sp6_set_inflow",
    "sp6_project_inflow", "sp6_apply_L", "sp6_apply_L_terms", "sp6_apply_LT", "sp6_rhs",
    "sp6_step", "sp6_step_stages", "sp6_adjoint_step_stages", "sp6_step_radial_implicit", "sp6_step_ab2", "sp6_step_timed", "sp6_adjoint_step", "sp6_apply_filter", "sp6_diagnostics",
    "sp6_outgoing_flux", "sp6_outgoing_flux_T", "sp6_step_noalloc", "sp6_device_bytes",
]


class Sp6Desc(ctypes.Structure):
    _fields_ = [
        ("n_eps", ctypes.c_int32), ("n_r", ctypes.c_int32), ("n_theta", ctypes.c_int32),
        ("n_phi", ctypes.c_int32), ("n_Theta", ctypes.c_int32), ("n_Phi", ctypes.c_int32),
        ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
        ("precision", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("scattering", ctypes.c_int32), ("filter", ctypes.c_int32),
    ]


class Sp6Error(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load libsp6d.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with paper_1104_5330_amd/build.py "
                      "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I32, U32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_uint32
    dp = ctypes.POINTER(ctypes.c_double)
    S = ctypes.c_int
    sig = {
        "sp6_validate_desc": (S, [ctypes.POINTER(Sp6Desc)]),
        "sp6_create": (S, [ctypes.POINTER(Sp6Desc), P, ctypes.POINTER(P)]),
        "sp6_destroy": (None, [P]),
        "sp6_set_stream": (S, [P, P]),
        "sp6_last_error": (ctypes.c_char_p, []),
        "sp6_get_nodes": (S, [P, dp, dp, dp, dp, dp]),
        "sp6_get_weights": (S, [P, dp, dp, dp, dp, dp]),
        "sp6_set_coefficients": (S, [P, P, P, P]),
        "sp6_set_scattering_kernel": (S, [P, D, D]),
        "sp6_set_energy_coupling": (S, [P, I32, D, D, D]),
        "sp6_set_inflow": (S, [P, P, P]),
        "sp6_project_inflow": (S, [P, P]),
        "sp6_apply_L": (S, [P, P, P]),
        "sp6_apply_L_terms": (S, [P, U32, P, P]),
        "sp6_apply_LT": (S, [P, P, P]),
        "sp6_rhs": (S, [P, P, P]),
        "sp6_step": (S, [P, P, D, I32]),
        "sp6_step_stages": (S, [P, P, D, P]),
        "sp6_adjoint_step_stages": (S, [P, P, P, D, P, P, P, P]),
        "sp6_step_radial_implicit": (S, [P, P, D, I32]),
        "sp6_step_ab2": (S, [P, P, P, D, I32, I32]),
        "sp6_step_timed": (S, [P, P, D, I32, dp, ctypes.POINTER(ctypes.c_int64)]),
        "sp6_adjoint_step": (S, [P, P, D, P, P, P, P]),
        "sp6_apply_filter": (S, [P, P]),
        "sp6_diagnostics": (S, [P, P, dp, dp, dp]),
        "sp6_outgoing_flux": (S, [P, P, P]),
        "sp6_outgoing_flux_T": (S, [P, P, P]),
        "sp6_step_noalloc": (S, [P, P, D, I32]),
        "sp6_device_bytes": (S, [P, ctypes.POINTER(ctypes.c_size_t)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != SP6_OK:
        msg = load().sp6_last_error()
        raise Sp6Error(status, msg.decode() if msg else "")
