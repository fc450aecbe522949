"""Host-side checks of the C-ABI library: it was built, it loads, and it exports exactly the
entry points include/a2a.h declares, with the binding covering each one.  No GPU calls."""
import ctypes
import os
import re

import pytest

from paper_1405_4524_amd import a2a

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "a2a.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*\*?\s*(a2a_[a-z0-9_]+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(a2a.LIB_PATH):
        pytest.fail("liba2a.so is not built: run python -m paper_1405_4524_amd.build")
    return a2a.lib()


def test_header_declares_the_documented_entry_points():
    names = declared()
    for must in ("a2a_init", "a2a_load_gauge", "a2a_load_clover", "a2a_dslash_clover", "a2a_solve_propagators",
                 "a2a_contract_pion_2pt", "a2a_contract_pipi_2pt", "a2a_engine_submit", "a2a_engine_step"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def test_binding_covers_header():
    assert sorted(a2a.EXPORTS) == declared()


def test_struct_layouts_match_header():
    assert ctypes.sizeof(a2a.Geom) == 5 * 4
    # 4 ints, 2 doubles, then the solver kind and a reserved int
    assert ctypes.sizeof(a2a.SolveInfo) == 4 * 4 + 2 * 8 + 2 * 4
    assert a2a.SolveInfo.solver.offset == 32
    assert a2a.SolveInfo.true_rel_residual.offset == 16


def test_library_is_gfx950_code(lib):
    data = open(a2a.LIB_PATH, "rb").read()
    assert b"gfx950" in data
