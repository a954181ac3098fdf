"""The C-ABI library loads and exports every entry point include/cdcs.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1611_01828_amd import cdcs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "cdcs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cdcs_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["cdcs_setup", "cdcs_iterate", "cdcs_solve", "cdcs_get_solution",
                 "cdcs_get_certificate", "cdcs_setup_batch", "cdcs_destroy"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = cdcs.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(cdcs.EXPORTS)
    assert lib.cdcs_abi_version() == 6 == cdcs.ABI_VERSION


def test_default_settings_match_the_paper():
    s = cdcs.default_settings()
    assert s.eps_tol == 1e-4 and s.max_iter == 2000 and s.check_every == 1
    assert s.eig_fp32 == 0 and s.autotune == 0 and s.alpha == 1.0 and s.eig_warm == 0
    assert s.method == cdcs.SELF_DUAL and s.rho == 1.0 and s.jacobi_max == 0


def test_struct_layouts():
    # cdcs_problem: 2 ints, (int64 + 3 ptrs), (int64 + 4 ptrs), ptr, int, 3 ptrs
    assert ctypes.sizeof(cdcs.Problem) == 8 + 32 + 40 + 8 + 8 + 24
    assert ctypes.sizeof(cdcs.Settings) == 64
    assert ctypes.sizeof(cdcs.Info) == 8 + 9 * 8
