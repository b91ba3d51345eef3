"""The C-ABI library builds, loads and exports every entry point the header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2210_03523_amd as dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dgtau.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(dg.LIB_PATH)
    names = _declared()
    assert "dg_residual" in names and "dg_tau_estimate" in names and "dg_rk3_step" in names
    for name in names:
        assert hasattr(L, name), name


def test_binding_covers_the_header():
    names = set(_declared()) - {"dg_last_error"}
    assert names == set(dg.SIGNATURES)


def test_last_error_is_empty_string_initially():
    if not os.path.exists(dg.LIB_PATH):
        pytest.skip("library not built")
    assert dg.lib().dg_last_error() == b""


def _arities():
    """Parameter count of every declared entry point, read from the header."""
    src = open(os.path.join(ROOT, "include", "dgtau.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(dg_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", src):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_arities_match_the_header():
    ar = _arities()
    for name, args in dg.SIGNATURES.items():
        assert ar[name] == len(args), (name, ar[name], len(args))
