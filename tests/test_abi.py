"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/sp6d.h, and validates descriptors."""

import ctypes
import os
import re

import pytest

from paper_1104_5330_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "sp6d.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(sp6_[A-Za-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = header_symbols()
    assert len(declared) >= 19
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_lib.SYMBOLS) == declared


def desc(**kw):
    base = dict(n_eps=2, n_r=9, n_theta=4, n_phi=8, n_Theta=4, n_Phi=8, r_in=1.0, r_out=3.0,
                precision=0, bc=1, scattering=1, filter=0)
    base.update(kw)
    return _lib.Sp6Desc(**base)


def test_validate_accepts_workload_shapes(lib):
    for shp in [(1, 17, 8, 16, 8, 16), (8, 33, 16, 32, 16, 32), (4, 65, 32, 64, 32, 64), (1, 3, 2, 4, 2, 4)]:
        d = desc(n_eps=shp[0], n_r=shp[1], n_theta=shp[2], n_phi=shp[3], n_Theta=shp[4], n_Phi=shp[5])
        assert lib.sp6_validate_desc(ctypes.byref(d)) == 0, lib.sp6_last_error()


@pytest.mark.parametrize("kw,code", [
    (dict(n_eps=0), _lib.SP6_ERR_SHAPE),
    (dict(n_r=2), _lib.SP6_ERR_SHAPE),
    (dict(n_r=81), _lib.SP6_ERR_SHAPE),
    (dict(n_theta=3), _lib.SP6_ERR_SHAPE),
    (dict(n_theta=64), _lib.SP6_ERR_SHAPE),
    (dict(n_phi=6), _lib.SP6_ERR_SHAPE),
    (dict(n_phi=2), _lib.SP6_ERR_SHAPE),
    (dict(n_Phi=16), _lib.SP6_ERR_SHAPE),
    (dict(n_Theta=1, n_Phi=2), _lib.SP6_ERR_SHAPE),
    (dict(r_in=0.0), _lib.SP6_ERR_ARG),
    (dict(r_out=1.0), _lib.SP6_ERR_ARG),
    (dict(r_in=float("nan")), _lib.SP6_ERR_ARG),
    (dict(precision=2), _lib.SP6_ERR_ARG),
    (dict(bc=2), _lib.SP6_ERR_ARG),
    (dict(scattering=-1), _lib.SP6_ERR_ARG),
    (dict(filter=7), _lib.SP6_ERR_ARG),
])
def test_validate_rejects(lib, kw, code):
    d = desc(**kw)
    assert lib.sp6_validate_desc(ctypes.byref(d)) == code
    assert lib.sp6_last_error().decode()


def test_validate_null_and_max_size(lib):
    assert lib.sp6_validate_desc(None) == _lib.SP6_ERR_ARG
    big = desc(n_eps=100000, n_r=80, n_theta=32, n_phi=64, n_Theta=32, n_Phi=64)
    assert lib.sp6_validate_desc(ctypes.byref(big)) == _lib.SP6_ERR_SHAPE
    assert "maximum" in lib.sp6_last_error().decode()
    # under the point limit but with more planes than 32-bit kernel counters take
    many = desc(n_eps=1_900_000, n_r=80, n_theta=4, n_phi=8, n_Theta=2, n_Phi=4)
    assert lib.sp6_validate_desc(ctypes.byref(many)) == _lib.SP6_ERR_SHAPE
    assert "planes" in lib.sp6_last_error().decode()


def test_null_handle_calls_fail_cleanly(lib):
    # every entry point rejects a NULL handle before touching the GPU
    assert lib.sp6_set_stream(None, None) == _lib.SP6_ERR_ARG
    assert lib.sp6_apply_L(None, None, None) == _lib.SP6_ERR_ARG
    assert lib.sp6_rhs(None, None, None) == _lib.SP6_ERR_ARG
    assert lib.sp6_step(None, None, 1.0, 1) == _lib.SP6_ERR_ARG
    assert lib.sp6_adjoint_step(None, None, 1.0, None, None, None, None) == _lib.SP6_ERR_ARG
    assert lib.sp6_diagnostics(None, None, None, None, None) == _lib.SP6_ERR_ARG
    out = ctypes.c_void_p()
    assert lib.sp6_create(None, None, ctypes.byref(out)) == _lib.SP6_ERR_ARG
    assert lib.sp6_create(ctypes.byref(desc(n_r=2)), None, ctypes.byref(out)) == _lib.SP6_ERR_SHAPE
    assert not out.value
    lib.sp6_destroy(None)  # NULL-safe


def test_product_path_does_not_import_oracle():
    # the binding and the library sources never reference the oracle
    pkg = os.path.join(ROOT, "paper_1104_5330_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                with open(os.path.join(dirpath, f)) as fh:
                    txt = fh.read()
                assert "oracle" not in txt.lower() or f == "build.py", f


def test_range_check_host_build(tmp_path, root):
    # the bounds arithmetic of the host validation (csrc/range_check.h), built on
    # its own with the host compiler: edges, wrap-around, zero sizes
    src = tmp_path / "t.cpp"
    src.write_text(r'''
#include "range_check.h"
#include <cstdio>
#include <cstdint>
int main() {
  const uintptr_t B = 0x7f0000000000ull;
  struct { uintptr_t base; size_t size; uintptr_t p; size_t bytes; bool want; } c[] = {
    {B, 4096, B, 4096, true}, {B, 4096, B, 4097, false}, {B, 4096, B + 16, 4080, true},
    {B, 4096, B + 16, 4081, false}, {B, 4096, B - 16, 16, false}, {B, 4096, B + 4096, 0, true},
    {B, 4096, B + 4112, 0, false}, {B, 4096, B + 8, SIZE_MAX, false}, {B, 0, B, 0, true},
    {B, 4096, UINTPTR_MAX - 8, 16, false}, {0, SIZE_MAX, 16, SIZE_MAX - 16, true},
  };
  int bad = 0;
  for (auto& k : c) bad += sp6_range_inside(k.base, k.size, k.p, k.bytes) != k.want;
  std::printf("%d\n", bad);
  return bad;
}
''')
    import shutil
    import subprocess
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    inc = os.path.join(root, "paper_1104_5330_amd", "csrc")
    exe = tmp_path / "t"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-I", inc, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout


def test_paired_order_host_build(tmp_path, root):
    # the paired in-plane order of the FP64 stage buffers (csrc/paired_order.h),
    # built on its own with the host compiler: a permutation inside each row with
    # its inverse, and every fused theta-phi tile of eight columns (four at Phi,
    # four at Phi + pi) one contiguous run in the order
    src = tmp_path / "p.cpp"
    src.write_text(r'''
#include "paired_order.h"
#include <cstdio>
int main() {
  int bad = 0;
  for (int G = 4; G <= 8; G *= 2)
    for (int nPh = 16; nPh <= 64; nPh *= 2) {
      const int hP = nPh / 2;
      int seen[64] = {0};
      for (int phi = 0; phi < nPh; ++phi) {
        const int p = paired_pos(phi, hP, G);
        bad += p < 0 || p >= nPh;
        if (p >= 0 && p < nPh) seen[p]++;
        bad += paired_phi(p, hP, G) != phi;
        bad += p / nPh != 0;
      }
      for (int p = 0; p < nPh; ++p) bad += seen[p] != 1;
      // tile t of a row: columns G t .. G t + G - 1 and their partners at + hP,
      // stored side by side from position 2 G t
      for (int t = 0; t < hP / G; ++t)
        for (int col = 0; col < 2 * G; ++col) {
          const int phi = G * t + (col % G) + (col >= G ? hP : 0);
          bad += paired_pos(phi, hP, G) != 2 * G * t + col;
        }
    }
  static_assert(paired_pos(37, 32) == 12 + 1, "Phi = 37 of 64: group 1 of the second half");
  static_assert(paired_pos(37, 32, 8) == 8 + 5, "FP32 groups of eight: Phi = 37 is 5 into the first group's partner");
  std::printf("%d\n", bad);
  return bad;
}
''')
    import shutil
    import subprocess
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    inc = os.path.join(root, "paper_1104_5330_amd", "csrc")
    exe = tmp_path / "p"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-I", inc, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout + r.stderr
