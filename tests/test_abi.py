"""The C-ABI library loads and exports every entry point include/rbffd.h
declares; argument checks that need no GPU compute."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")
LIB = os.path.join(ROOT, "paper_1509_02615_amd", "librbffd.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char \*|float \*)\s*(rbffd_\w+)\s*\(", text, re.M)))


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("rbffd_knn", "rbffd_weights", "rbffd_model_create", "rbffd_rhs", "rbffd_step", "rbffd_ghost"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_1509_02615_amd.build)"
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_mirrors_the_abi():
    from paper_1509_02615_amd import rbffd as R
    assert sorted(R.EXPORTS) == declared()
    for n in ("rbffd_knn", "rbffd_weights", "rbffd_model_create", "rbffd_rhs", "rbffd_step", "rbffd_ghost"):
        assert callable(getattr(R, n))


def test_null_context_is_rejected_without_a_device():
    lib = ctypes.CDLL(LIB)
    lib.rbffd_knn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.rbffd_knn(None, None, None) == -1
    lib.rbffd_last_error.restype = ctypes.c_char_p
    assert lib.rbffd_last_error(None) == b"null context"
