"""The C-ABI library loads and exports every symbol include/amfmm.h declares
(no compute calls, so this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amfmm.h")
LIB = os.path.join(ROOT, "paper_1706_06989_amd", "libamfmm_hip.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(amfmm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ("amfmm_build_tree", "amfmm_compute_moments", "amfmm_solve_gravity",
                 "amfmm_create", "amfmm_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libamfmm_hip.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1706_06989_amd import amfmm
    assert sorted(amfmm.EXPORTED) == declared()
    L = amfmm.lib()
    assert L.amfmm_status_string(-3) == b"out of device memory"
