"""Compile the C oracle into oracle/liboracle_wd.so (test infrastructure)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wdref.c")
LIB = os.path.join(HERE, "liboracle_wd.so")


def build(verbose=False, out=None, native=False):
    """The in-tree build is portable (x86-64-v2: it is built once and may run
    on another host); native=True builds for the host at hand (-march=native)
    into `out`, for timing the oracle where it runs."""
    lib = out or LIB
    arch = "-march=native" if native else "-march=x86-64-v2"
    cmd = ["gcc", "-O3", arch, "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", lib + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
