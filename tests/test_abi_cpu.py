"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/mm.h, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2103_12819_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libmm.so not built (run __graft_entry__.build())")
    return N.load()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "mm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:mm_status|void|const char \*)\s*\*?\s*(mm_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_python_mirror():
    assert declared_symbols() == sorted(N.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name


STRUCTS = ("mm_grid", "mm_materials", "mm_bias", "mm_source", "mm_hard_source", "mm_surface_current",
           "mm_pml", "mm_options", "mm_probe_desc")


def test_ctypes_mirror_matches_the_c_compiler(tmp_path):
    """Size and every field offset of each struct, as gcc lays out the
    header, against the ctypes mirror; and MM_MAX_HARD."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mm.h"', 'int main(void) {']
    for st in STRUCTS:
        lines.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for name, _ in getattr(N, st)._fields_:
            lines.append(f'  printf("{st} {name} %zu\\n", offsetof({st}, {name}));')
    lines.append('  printf("MM_MAX_HARD %d\\n", MM_MAX_HARD);')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split() if len(line.split()) == 3 else (line.split()[0], "", line.split()[1])
            got[(a, b)] = int(v)
    for st in STRUCTS:
        cls = getattr(N, st)
        assert got[(st, "size")] == C.sizeof(cls), st
        for name, _ in cls._fields_:
            assert got[(st, name)] == getattr(cls, name).offset, (st, name)
    assert got[("MM_MAX_HARD", "")] == N.MM_MAX_HARD


def test_struct_layouts_match_the_header():
    # sizes on x86-64 (LP64): int32 x6 + padding + doubles / pointers
    assert C.sizeof(N.mm_grid) == 48
    assert C.sizeof(N.mm_materials) == 7 * 8
    assert C.sizeof(N.mm_bias) == 24
    assert C.sizeof(N.mm_source) == 40
    assert C.sizeof(N.mm_options) == 80
    assert C.sizeof(N.mm_pml) == 40
    assert C.sizeof(N.mm_hard_source) == 40
    assert C.sizeof(N.mm_surface_current) == 48
    assert C.sizeof(N.mm_probe_desc) == 20


def _init(lib, n=(8, 4, 4), d=(1e-6,) * 3, dt=None, tol=1e-10, max_iter=10, prec=0, Ms=None,
          eps=None, bc=(0, 0, 0), scheme=0, pml=None, fused=0):
    ctx = C.c_void_p()
    g = N.mm_grid(n[0], n[1], n[2], (C.c_int32 * 3)(*bc), d[0], d[1], d[2])
    keep = [] if Ms is None else [Ms]
    mat = N.mm_materials()
    if Ms is not None:
        mat.Ms = Ms.ctypes.data_as(C.POINTER(C.c_double))
    if eps is not None:
        keep.append(eps)
        mat.eps_r = eps.ctypes.data_as(C.POINTER(C.c_double))
    opt = N.mm_options()
    opt.prec, opt.tol, opt.max_iter, opt.scheme, opt.fused = prec, tol, max_iter, scheme, fused
    if pml is not None:
        cells, R0, order = pml
        keep.append(N.mm_pml((C.c_int32 * 6)(*cells), R0, order))
        opt.pml = C.pointer(keep[-1])
    if dt is None:
        dt = W.cfl_dt(0.9, *d)
    st = lib.mm_init(C.byref(ctx), C.byref(g), dt, C.byref(mat), None, None, C.byref(opt))
    return st, ctx


@pytest.mark.parametrize("kw", [
    dict(dt=W.cfl_dt(1.01, 1e-6, 1e-6, 1e-6)),          # above the CFL limit
    dict(dt=-1.0),
    dict(tol=0.0),
    dict(max_iter=0),
    dict(prec=7),
    dict(scheme=3),
    dict(fused=2),
    dict(pml=((2, 2, 0, 0, 0, 0), 1e-6, 3), bc=(1, 0, 0)),     # layer on a periodic axis
    dict(pml=((4, 4, 0, 0, 0, 0), 1e-6, 3)),                  # layers fill the axis (8 cells)
    dict(pml=((2, 0, 0, 0, 0, 0), 1.5, 3)),                   # R0 >= 1
    dict(pml=((2, 0, 0, 0, 0, 0), 1e-6, 0.5)),                # order < 1
    dict(pml=((-1, 0, 0, 0, 0, 0), 1e-6, 3)),
    dict(n=(0, 4, 4)),
    dict(d=(1e-6, 0.0, 1e-6), dt=1e-16),
    dict(bc=(0, 2, 0)),
    dict(Ms=-np.ones(128)),
    dict(eps=np.zeros(128)),
    dict(eps=np.full(128, np.nan)),
])
def test_bad_arguments_are_rejected_before_any_device_work(kw):
    lib = _lib()
    st, ctx = _init(lib, **kw)
    assert st == N.MM_EINVAL
    assert not ctx.value


def test_null_pointers_are_rejected():
    lib = _lib()
    assert lib.mm_init(None, None, 1.0, None, None, None, None) == N.MM_EINVAL
    assert lib.mm_step(None, 1) == N.MM_EINVAL
    assert lib.mm_add_hard_source(None, None) == N.MM_EINVAL
    assert lib.mm_add_surface_current(None, None) == N.MM_EINVAL
    assert lib.mm_sync(None) == N.MM_EINVAL
    lib.mm_destroy(None)
