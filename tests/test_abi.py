"""CPU checks of the boundary: libbkry.so loads (no GPU needed for that) and
exports every function that include/bkry.h declares; the Python binding names
the same entry points.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bkry.h")
LIB = os.path.join(ROOT, "paper_2104_02494_amd", "libbkry.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(bkry_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_entry_points():
    names = declared()
    for need in ["bkry_cg_solve", "bkry_gmres_solve", "bkry_spmm", "bkry_bdot", "bkry_tsqr", "bkry_sddmm",
                 "bkry_csr_transpose", "bkry_create", "bkry_destroy", "bkry_last_error"]:
        assert need in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbkry.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(L, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbkry.so not built")
def test_binding_matches_header():
    import paper_2104_02494_amd as P
    assert sorted(P.EXPORTS) == declared()
    for name in declared():
        if name not in ("bkry_create", "bkry_destroy", "bkry_set_stream", "bkry_last_error", "bkry_spmm_f32",
                        "bkry_bdot_f32"):
            assert hasattr(P, name), name


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2104_02494_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "bkry_oracle" not in txt, f
