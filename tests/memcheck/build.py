"""Build the library's own sources for the CPU stand-in of the HIP runtime, with AddressSanitizer.

Test harness only.  The sources are taken unchanged from paper_2210_11797_amd/csrc except for textual
substitutions that g++ needs (the dynamic LDS array becomes the stand-in's per-launch buffer; the
header include gets an absolute path; clang's vector types used as matrix-core operands become the
stand-in's structs); the result is a separate shared object in a
scratch directory, never the product library.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2210_11797_amd", "csrc")
sys.path.insert(0, ROOT)
from paper_2210_11797_amd.build import SOURCES  # noqa: E402

CXX = os.environ.get("CXX_MEMCHECK", "g++")
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-fsanitize=address", "-fno-omit-frame-pointer", "-w"]


def asan_runtime() -> str:
    return subprocess.run([CXX, "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()


def _prepare(outdir: str) -> list[str]:
    hdr = os.path.join(ROOT, "include", "hyb.h")
    out = []
    for name in ["hyb_internal.h", *SOURCES]:
        text = open(os.path.join(CSRC, name)).read()
        text = text.replace('"../../include/hyb.h"', f'"{hdr}"')
        text = text.replace("extern __shared__ unsigned char smem_raw[];",
                            "unsigned char *smem_raw = emu::dyn_smem();")
        text = text.replace("typedef float f32x4 __attribute__((ext_vector_type(4)));", "typedef emu_f32x4 f32x4;")
        text = text.replace("typedef short bf16x4 __attribute__((ext_vector_type(4)));", "typedef emu_bf16x4 bf16x4;")
        text = text.replace("typedef float p1_f2 __attribute__((ext_vector_type(2)));", "typedef emu_f32x2 p1_f2;")
        text = text.replace("typedef float nn_f32x4 __attribute__((ext_vector_type(4)));", "typedef emu_f32x4 nn_f32x4;")
        text = text.replace("typedef short nn_bf16x4 __attribute__((ext_vector_type(4)));",
                            "typedef emu_bf16x4 nn_bf16x4;")
        text = text.replace("typedef __bf16 nn_bf16x8 __attribute__((ext_vector_type(8)));",
                            "typedef emu_s16x8 nn_bf16x8;")
        text = text.replace("typedef unsigned int nn_u32x4 __attribute__((ext_vector_type(4)));",
                            "typedef emu_u32x4 nn_u32x4;")
        text = text.replace("typedef short nn_s16x8 __attribute__((ext_vector_type(8)));", "typedef emu_s16x8 nn_s16x8;")
        dst = os.path.join(outdir, name if name.endswith(".h") else name.replace(".hip", ".cpp"))
        with open(dst, "w") as f:
            f.write(text)
        if dst.endswith(".cpp"):
            out.append(dst)
    return out


def build(outdir: str) -> str:
    os.makedirs(outdir, exist_ok=True)
    srcs = _prepare(outdir) + [os.path.join(HERE, "emu_rt.cpp")]
    inc = ["-I" + os.path.join(HERE, "include"), "-I" + outdir]

    def compile_one(src):
        obj = os.path.join(outdir, os.path.basename(src).replace(".cpp", ".o"))
        res = subprocess.run([CXX, *FLAGS, *inc, "-c", src, "-o", obj], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"{CXX} failed on {src}:\n{res.stderr[-4000:]}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = os.path.join(outdir, "libhyb_memcheck.so")
    subprocess.run([CXX, "-shared", "-fsanitize=address", "-o", lib, *objs], check=True)
    return lib


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "_build")))
