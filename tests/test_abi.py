"""The C-ABI library loads and exports every entry point include/pdcs.h
declares, and its default settings are the readings the oracle uses (CPU only:
no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdcs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdcs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("pdcs_problem_create", "pdcs_solve", "pdcs_project", "pdcs_spmv", "pdcs_kkt"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2505_00311_amd import pdcs
    lib = pdcs.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(pdcs.SYMBOLS)


def test_default_settings_match_the_oracle_readings(orc):
    from paper_2505_00311_amd import pdcs
    g = pdcs.settings_default()
    o = orc.default_settings()
    for name, _ in orc.Settings._fields_:
        assert getattr(g, name) == getattr(o, name), name


def test_status_strings_and_null_arguments():
    from paper_2505_00311_amd import pdcs
    lib = pdcs.load()
    assert lib.pdcs_status_string(0) == b"ok"
    assert lib.pdcs_settings_default(None) == -1
    out = ctypes.c_void_p()
    assert lib.pdcs_problem_create(None, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert b"NULL" in lib.pdcs_last_error()


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(ROOT, "paper_2505_00311_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "pdcs_oracle" not in src and "orc_" not in src, f
