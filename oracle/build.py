"""Build the CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain gcc, -O2 with OpenMP, no fast-math and no flush-to-zero, so that the
oracle's integer and FP64 arithmetic follow their plain C definitions.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "oracle.c")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-fno-fast-math", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
