"""Host validation of device buffers through the raw C ABI (no Python checks in
between): a state buffer whose extent runs past the end of its device
allocation, or a buffer far smaller than a state, is rejected with SP6_ERR_ARG
before anything is enqueued; an exactly sized allocation is accepted."""

import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_util import need_gpu, small, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1104_5330_amd  # noqa: F401


def test_buffer_extent_checked_against_its_allocation():
    from paper_1104_5330_amd import Sp6Grid, _lib
    # 1,048,576 points: a state is 8 MiB, a whole number of 2 MiB pages, so a
    # hipMalloc of exactly one state has no slack after it
    cfg = small(3, n_eps=1, n_r=64, n_theta=16, n_phi=32, n_Theta=4, n_Phi=8)
    G = Sp6Grid.from_config(cfg)
    B = cfg.points * 8
    assert B == 8 << 20
    hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime already loaded by torch and the library
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    hip.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), B) == 0
    try:
        assert hip.hipMemset(p, 0, B) == 0
        out = torch.empty(cfg.shape, dtype=torch.float64, device="cuda")
        o = ctypes.c_void_p(out.data_ptr())
        lib = G.lib
        assert lib.sp6_set_stream(G._h, G._stream()) == 0
        st = lib.sp6_apply_L(G._h, ctypes.c_void_p(p.value + 16), o)
        msg = lib.sp6_last_error().decode()
        banner(f"offset state: status {st}, '{msg}'")
        assert st == _lib.SP6_ERR_ARG and "too small" in msg
        tiny = torch.zeros(1000, dtype=torch.float64, device="cuda")
        st = lib.sp6_apply_L(G._h, ctypes.c_void_p(tiny.data_ptr()), o)
        assert st == _lib.SP6_ERR_ARG
        st = lib.sp6_step(G._h, ctypes.c_void_p(p.value + 16), ctypes.c_double(cfg.dt), ctypes.c_int32(1))
        assert st in (_lib.SP6_ERR_ARG, _lib.SP6_ERR_STATE)
        st = lib.sp6_apply_L(G._h, p, o)
        assert st == _lib.SP6_OK, lib.sp6_last_error().decode()
        torch.cuda.synchronize()
        assert float(out.abs().max()) == 0.0  # L of the zero state
    finally:
        torch.cuda.synchronize()
        hip.hipFree(p)
    G.close()
