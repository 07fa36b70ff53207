"""The C-ABI library loads on the host and exports every entry point the header declares (CPU)."""

import ctypes
import os
import re

from paper_2210_11797_amd import ABI_FUNCTIONS, LIB_PATH

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hyb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hyb_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB_PATH), "libhyb.so not built (run paper_2210_11797_amd/build.py)"
    lib = ctypes.CDLL(LIB_PATH)
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, missing


def test_null_arguments_are_rejected_without_a_device():
    """Argument validation happens before any HIP call."""
    lib = ctypes.CDLL(LIB_PATH)
    lib.hyb_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.hyb_create(None, None, None, ctypes.byref(out)) == -1
    assert lib.hyb_create(None, None, None, None) == -1
    lib.hyb_last_error.restype = ctypes.c_char_p
    assert lib.hyb_last_error(None) == b"null context"
    for name in ("hyb_condense", "hyb_trace_apply", "hyb_precondition", "hyb_solve", "hyb_recover"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
    assert lib.hyb_trace_apply(None, None, None) == -1
    assert lib.hyb_condense(None, None, None, None) == -1
