"""Build the CPU oracle library (test infrastructure) with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRCS = ["solar.c", "shadow.c"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", "-Wall",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SRCS] + ["-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
