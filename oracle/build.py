"""Build step for the CPU oracle (test infrastructure; see oracle/__init__.py)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "lhaf_oracle.c"), os.path.join(HERE, "lhaf_body.h")]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB):
        return LIB
    cmd = [
        "gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
        "-Wall", "-Wextra", "-o", LIB + ".tmp", SOURCES[0], "-lm",
    ]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
