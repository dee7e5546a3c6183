"""The C-ABI library loads and exports every function include/rm.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1909_07321_amd", "librm.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rm_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_parsed():
    names = declared_functions()
    for must in ["rm_create", "rm_form_R", "rm_asymptotic", "rm_solve_K", "rm_collision_strengths", "rm_submit",
                 "rm_poll"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librm.so not built")
def test_binding_lists_every_symbol():
    from paper_1909_07321_amd import rm
    assert sorted(rm.EXPORTS) == declared_functions()


def test_oracle_not_linked_into_library():
    # the product library must not depend on the oracle
    if not os.path.exists(LIB):
        pytest.skip("librm.so not built")
    data = open(LIB, "rb").read()
    assert b"rmo_" not in data and b"librmo" not in data
