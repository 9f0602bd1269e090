"""Host validation through the raw C ABI (no Python checks in between): a state
buffer whose extent runs past the end of its device allocation, or a buffer far
smaller than a state, is rejected with SP6_ERR_ARG before anything is enqueued,
and an exactly sized allocation is accepted; the degenerate stepping calls (zero
steps, a negative count, a time step that is not finite and positive, no
coefficients yet) return their documented status and leave the state untouched."""

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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_degenerate_step_calls(precision):
    import synth
    from paper_1104_5330_amd import Sp6Grid, _lib
    from tests.gpu_util import to_dev
    cfg = small(3, n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8)
    G = Sp6Grid.from_config(cfg, precision=precision)
    lib, h = G.lib, G._h
    assert lib.sp6_set_stream(h, G._stream()) == 0
    F = to_dev(synth.fields.random_state(cfg, 3))
    F0 = F.clone()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    dt = ctypes.c_double(cfg.dt)
    # coefficients not set yet: the step is refused
    assert lib.sp6_step(h, vp(F), dt, ctypes.c_int32(1)) == _lib.SP6_ERR_STATE
    k, s, e = synth.fields.random_coeffs(cfg, 4)
    G.set_coefficients(to_dev(k), to_dev(s), to_dev(e))
    calls = {
        "step": lambda n, t: lib.sp6_step(h, vp(F), ctypes.c_double(t), ctypes.c_int32(n)),
        "step_noalloc": lambda n, t: lib.sp6_step_noalloc(h, vp(F), ctypes.c_double(t), ctypes.c_int32(n)),
        "step_radial_implicit": lambda n, t: lib.sp6_step_radial_implicit(h, vp(F), ctypes.c_double(t),
                                                                          ctypes.c_int32(n)),
    }
    if precision == "fp64":
        H = to_dev(synth.fields.random_state(cfg, 5))
        H0 = H.clone()
        calls["step_ab2"] = lambda n, t: lib.sp6_step_ab2(h, vp(F), vp(H), ctypes.c_double(t), ctypes.c_int32(n),
                                                          ctypes.c_int32(0))
    for name, call in calls.items():
        assert call(0, cfg.dt) == _lib.SP6_OK, (name, lib.sp6_last_error().decode())
        assert call(-1, cfg.dt) == _lib.SP6_ERR_ARG, name
        for bad in (0.0, -cfg.dt, float("nan"), float("inf")):
            assert call(1, bad) == _lib.SP6_ERR_ARG, (name, bad)
            assert "dt" in lib.sp6_last_error().decode()
    torch.cuda.synchronize()
    banner(f"degenerate step calls ({precision}): {sorted(calls)} left the state untouched")
    assert torch.equal(F, F0)
    if precision == "fp64":
        assert torch.equal(H, H0)
    G.close()
