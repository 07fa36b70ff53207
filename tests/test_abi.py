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


def _struct_fields(src, name):
    """Field names, in order, of `typedef struct { ... } name;` in the header."""
    blocks = dict((n, b) for b, n in re.findall(r"typedef struct \{([^{}]*)\}\s*(\w+);", src))
    assert name in blocks, name
    body = re.sub(r"/\*.*?\*/", "", blocks[name], flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = re.sub(r"^(const\s+)?[A-Za-z_0-9]+\s*", "", decl)  # the type
        for part in decl.split(","):
            names.append(part.strip().lstrip("*").strip())
    return names


def test_structs_match_the_binding():
    from paper_2210_11797_amd import _native as N

    src = open(os.path.join(ROOT, "include", "hyb.h")).read()
    for cname, ctype in (("hyb_level", N._Level), ("hyb_mesh", N._Mesh), ("hyb_params", N._Params),
                         ("hyb_info", N._Info)):
        assert _struct_fields(src, cname) == [f[0] for f in ctype._fields_], cname


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
