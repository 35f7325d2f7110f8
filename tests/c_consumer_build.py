"""Build tests/_bin/c_consumer from tests/c_consumer.c: a plain C program
linked against libsa.so (the HIP library must be built first) and the HIP
runtime.  The run-time search path points at the library in the tree."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c_consumer.c")
BIN = os.path.join(HERE, "_bin", "c_consumer")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler")
    os.makedirs(os.path.dirname(BIN), exist_ok=True)
    cmd = [cc, "-O2", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", BIN,
           "-L", os.path.join(ROOT, "paper_1907_04435_amd"), "-lsa", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1907_04435_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C consumer build failed:\n" + r.stdout + r.stderr)
    return BIN


if __name__ == "__main__":
    print(build())
