"""The C-ABI library loads on the host and exports every entry point that
include/bh.h declares (no compute calls: those need the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bh.h")
LIB = os.path.join(ROOT, "paper_0909_0541_amd", "libbh.so")


def declared():
    src = open(HEADER).read()
    return re.findall(r"^(?:bh_status|void|const char \*)\s*(bh_\w+)\(", src, re.M)


def test_header_declares_the_boundary():
    names = declared()
    for n in ["bh_create", "bh_destroy", "bh_build_tree", "bh_make_groups", "bh_compute_forces",
              "bh_build_batch", "bh_compute_forces_batch", "bh_direct_sampled", "bh_get_stats"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libbh.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_0909_0541_amd import bh
    src = open(bh.__file__).read()
    missing = [n for n in declared() if f'"{n}"' not in src]
    assert not missing, missing


def test_null_context_is_rejected_without_a_gpu():
    lib = ctypes.CDLL(LIB)
    lib.bh_build_tree.restype = ctypes.c_int
    lib.bh_build_tree.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.bh_build_tree(None, 0, None, None) == -1
    lib.bh_last_error.restype = ctypes.c_char_p
    lib.bh_last_error.argtypes = [ctypes.c_void_p]
    assert lib.bh_last_error(None) == b"null context"


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_0909_0541_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and "bh_oracle" not in text, f
