"""The C-ABI library loads and exports every entry point declared in include/lp.h
(no device calls, runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ["lp_create", "lp_destroy", "lp_neighbors", "lp_gfd", "lp_gfd3", "lp_step", "lp_run", "lp_conservation"]:
        assert n in names


def test_library_exports_all_declared_symbols():
    from paper_2206_11998_amd import lp
    if not os.path.exists(lp.LIB_PATH):
        from paper_2206_11998_amd import build
        build.build()
    L = lp.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(lp.EXPORTS) <= set(_declared())


def test_status_strings():
    from paper_2206_11998_amd import lp
    L = lp.lib()
    assert L.lp_status_str(lp.OK) == b"ok"
    assert b"capacity" in L.lp_status_str(lp.E_CAPACITY)
