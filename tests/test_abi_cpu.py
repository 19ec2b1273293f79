"""CPU checks of the boundary: the C-ABI library loads (no GPU call) and exports every
function include/mrhs.h declares; the binding declares the same names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrhs.h")
LIB = os.path.join(ROOT, "paper_1601_03184_amd", "libmrhs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["mrhs_op_create", "dirac_apply_mrhs", "sap_smooth_mrhs", "block_orthonormalize", "coarse_op_build",
              "mrhs_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_binding_exposes_the_same_names():
    from paper_1601_03184_amd import mrhs
    for n in declared_functions():
        assert callable(getattr(mrhs, n)), n
