"""Build the CPU oracle shared library (plain C, gcc, OpenMP, no contraction).

Test infrastructure only: the GPU library never links or loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ka_oracle.c")
LIB = os.path.join(HERE, "libka_oracle.so")


def build(force: bool = True) -> str:
    """Compile oracle/ka_oracle.c into oracle/libka_oracle.so and return its path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
