"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects invalid arguments before launching."""
import ctypes as C
import os
import re

import pytest

from paper_2001_04886_amd import sstep as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "sstep.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sstep_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_binding_exports():
    assert header_functions() == sorted(S.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    lib = S.load()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    for st in (0, 1, -1, -2, -3, -4, -5):
        assert len(S.status_string(st)) > 3
    assert S.status_string(99) == "unknown status"


def test_workspace_sizing_and_argument_checks():
    A = S.Stencil(3, 256, 256, 256, (1.0,) * 7)
    nb = S.workspace_bytes(A, S.METHOD_GMRES, 8, 40)
    N = 256 ** 3
    assert nb >= 321 * N * 8            # the basis: m*s+1 FP64 columns
    assert nb < 321 * N * 8 * 1.01
    nb32 = S.workspace_bytes(A, S.METHOD_GMRES, 8, 40, S.MIXED)
    assert 321 * N * 4 <= nb32 < nb
    assert S.workspace_bytes(A, S.METHOD_OMIN, 8, 8) >= (2 * 64 + 9) * N * 8
    assert S.workspace_bytes(A, S.METHOD_GMRES, 0, 40) == 0
    assert S.workspace_bytes(A, S.METHOD_GMRES, 17, 40) == 0
    assert S.workspace_bytes(A, S.METHOD_GMRES, 8, 300) == 0   # m*s > 2048
    assert S.workspace_bytes(A, S.METHOD_OMIN, 8, 65) == 0
    assert S.workspace_bytes(A, S.METHOD_OMIN, 8, 8, S.MIXED) == 0
    bad = S.Stencil(4, 8, 8, 8, (1.0,) * 7)
    assert S.workspace_bytes(bad, S.METHOD_GMRES, 4, 4) == 0


def test_solvers_reject_bad_arguments_without_launching():
    lib = S.load()
    A = S.Stencil(2, 8, 8, 1, (4.0, -1, -1, -1, -1, 0, 0)).c_struct()
    info = S.InfoC()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.sstep_gmres_solve(C.byref(A), fake, fake, 0, 4, 1e-8, None, C.byref(info)) == -1
    assert info.status == -1
    assert lib.sstep_gmres_solve(C.byref(A), fake, fake, 4, 4, -1.0, None, None) == -1
    assert lib.sstep_gmres_solve(C.byref(A), None, fake, 4, 4, 1e-8, None, None) == -1
    assert lib.sstep_omin_solve(C.byref(A), fake, fake, 4, 0, 1e-8, None, None) == -1
    o = S.OptionsC()
    lib.sstep_default_options(C.byref(o))
    o.precision = 1
    assert lib.sstep_omin_solve(C.byref(A), fake, fake, 4, 4, 1e-8, C.byref(o), None) == -1
    o.precision = 0
    o.basis = 7
    assert lib.sstep_gmres_solve(C.byref(A), fake, fake, 4, 4, 1e-8, C.byref(o), None) == -1
    Bad = S.Stencil(2, 0, 8, 1, (4.0, -1, -1, -1, -1, 0, 0)).c_struct()
    assert lib.sstep_gmres_solve(C.byref(Bad), fake, fake, 4, 4, 1e-8, None, None) == -1
    assert lib.sstep_stencil_apply(C.byref(A), fake, fake, None) == -1   # x == y
    assert lib.sstep_kernel_gram(fake, 10, 3, fake, 10, 17, 10, fake, None) == -1
