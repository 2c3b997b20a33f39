"""Compile the plain-C example against include/cpht.h and libcpht.so with the
host C compiler (no HIP compiler, no torch): proof that the boundary is a C
ABI.  Used by the build entry point and by tests/test_c_abi.py."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "cuckoo_then_iceberg.c")
BIN = os.path.join(HERE, "cuckoo_then_iceberg")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out: str = BIN) -> str:
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no host C compiler")
    libdir = os.path.join(ROOT, "paper_2406_09255_amd")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", out,
           "-L", libdir, "-lcpht", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{libdir}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


if __name__ == "__main__":
    print(build())
