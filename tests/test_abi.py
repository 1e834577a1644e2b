"""C ABI checks that need no GPU: every function declared in include/*.h is
exported by the built library, the ctypes mirrors of the public structs have
the C layout, and argument validation rejects bad input before touching the
device."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slar.h")
LIB = os.path.join(ROOT, "paper_2606_29027_amd", "libslar.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w ]*\*?\s+\*?(slar_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


@needs_lib
def test_every_declared_symbol_is_exported():
    lib = C.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@needs_lib
def test_binding_covers_header():
    from paper_2606_29027_amd import lib as L
    assert set(declared_functions()) <= set(L.EXPORTS)


@needs_lib
def test_status_strings_and_invalid_arguments_without_gpu():
    from paper_2606_29027_amd import lib as L
    lib = L.load()
    assert L.status_str(0) == "ok" and "rank" in L.status_str(3)
    g = L.Grid()
    g.dx, g.dv = 2, 1                           # dx != dv: rejected before any HIP call
    h = C.c_void_p()
    assert lib.slar_workspace_create(C.byref(g), 40, C.byref(h)) == L.SLAR_E_INVAL
    g.dx, g.dv = 1, 1
    g.n[0], g.n[1] = 2, 64                      # too few cells
    g.hi[0], g.hi[1] = 1.0, 1.0
    assert lib.slar_workspace_create(C.byref(g), 40, C.byref(h)) == L.SLAR_E_INVAL
    assert lib.slar_cnn_create(0, None, 1, 1, C.byref(h)) == L.SLAR_E_INVAL
    assert lib.slar_truncate(None, None, 1e-6, 10, None, None, None) == L.SLAR_E_INVAL
    assert lib.slar_nested_cross(None, None, None, L.F64, 1e-6, 10, 0, None, None, None, None, None,
                                 None) == L.SLAR_E_INVAL


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "slar.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("slar_grid %zu\n", sizeof(slar_grid));
  P(slar_grid, n) P(slar_grid, lo) P(slar_grid, hi)
  printf("slar_ht %zu\n", sizeof(slar_ht));
  P(slar_ht, rank) P(slar_ht, dtype) P(slar_ht, leaf) P(slar_ht, B12) P(slar_ht, root)
  printf("slar_frames %zu\n", sizeof(slar_frames));
  P(slar_frames, X) P(slar_frames, P)
  printf("slar_adv %zu\n", sizeof(slar_adv));
  P(slar_adv, tau) P(slar_adv, cv) P(slar_adv, E) P(slar_adv, cE)
  printf("slar_lowrank %zu\n", sizeof(slar_lowrank));
  P(slar_lowrank, U) P(slar_lowrank, V)
  printf("slar_cross_info %zu\n", sizeof(slar_cross_info));
  P(slar_cross_info, samples)
  printf("slar_nested_info %zu\n", sizeof(slar_nested_info));
  P(slar_nested_info, rank) P(slar_nested_info, samples)
  printf("slar_macro_system %zu\n", sizeof(slar_macro_system));
  P(slar_macro_system, U) P(slar_macro_system, c) P(slar_macro_system, nstage)
  P(slar_macro_system, R) P(slar_macro_system, d) P(slar_macro_system, beta)
  return 0;
}
"""


@needs_lib
def test_workspace_bytes_and_caller_memory_checks_without_gpu():
    """slar_workspace_bytes is host arithmetic: it grows with the grid, and
    slar_workspace_create_in rejects a null, misaligned or too small buffer
    before any device call (a host buffer stands in; it is never written)."""
    import slar_inputs as SI
    from paper_2606_29027_amd import lib as L
    lib = L.load()
    small = L.make_grid(SI.config("landau2d", n=16))
    big = L.make_grid(SI.config("stronglandau2d"))
    b16, b128 = L.slar_workspace_bytes(small, 40), L.slar_workspace_bytes(big, 60)
    assert 0 < b16 < b128 and b16 % 256 == 0 and b128 % 256 == 0
    n = C.c_size_t(0)
    assert lib.slar_workspace_bytes(C.byref(small), 65, C.byref(n)) == L.SLAR_E_INVAL
    h = C.c_void_p()
    buf = (C.c_uint8 * 4096)()
    addr = (C.addressof(buf) + 255) & ~255
    assert lib.slar_workspace_create_in(C.byref(small), 40, None, b16, C.byref(h)) == L.SLAR_E_INVAL
    assert lib.slar_workspace_create_in(C.byref(small), 40, C.c_void_p(addr), 2048, C.byref(h)) == L.SLAR_E_NOMEM
    assert lib.slar_workspace_create_in(C.byref(small), 40, C.c_void_p(addr + 8), b16, C.byref(h)) == L.SLAR_E_INVAL
    assert not h.value


def test_ctypes_struct_layout_matches_header(tmp_path):
    gcc = shutil.which("gcc")
    inc = "/opt/rocm/include"
    if gcc is None or not os.path.isdir(inc):
        pytest.skip("no C compiler or HIP headers")
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    r = subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", inc,
                        str(src), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("header does not compile as C here: " + r.stderr[-300:])
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if l)
    from paper_2606_29027_amd import lib as L
    mirror = {"slar_grid": L.Grid, "slar_ht": L.HT, "slar_frames": L.Frames, "slar_adv": L.Adv,
              "slar_lowrank": L.LowRank, "slar_cross_info": L.CrossInfo,
              "slar_macro_system": L.MacroSystem, "slar_nested_info": L.NestedInfo}
    for key, val in out.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(mirror[t], f).offset == int(val), key
        else:
            assert C.sizeof(mirror[key]) == int(val), key


@needs_lib
def test_host_time_integrator_weights_match_oracle():
    """The library's DIRK-3 tableau and variable-step BDF weights (host
    code, no GPU) equal the oracle's, including unequal steps; times that do
    not decrease are rejected."""
    import numpy as np
    from oracle import timeint as TI
    from paper_2606_29027_amd import lib as L
    A, c = L.slar_dirk3_tableau()
    Ao, _, co = TI.dirk3()
    # gamma: bisection here, a companion-matrix eigenvalue in the oracle; both
    # agree to ~1e-15, and b1, b2 scale that by at most ~4
    assert np.allclose(A, Ao, rtol=0, atol=1e-14) and np.allclose(c, co, rtol=0, atol=1e-14)
    rng = np.random.default_rng(3)
    for k in (1, 2, 3):
        for _ in range(5):
            t = np.cumsum(np.concatenate([[0.0], rng.uniform(0.05, 0.4, k)]))[::-1] + 1.7
            cw, beta = L.slar_bdf_weights(list(t))
            cwo, betao = TI.bdf(t)
            assert np.allclose(cw, cwo, rtol=1e-13, atol=0) and abs(beta - betao) < 1e-15
    with pytest.raises(L.SlarError):
        L.slar_bdf_weights([1.0, 1.0, 0.5])
    with pytest.raises(L.SlarError):
        L.slar_bdf_weights([1.0, 0.9, 0.8, 0.7, 0.6])
