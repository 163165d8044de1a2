"""Build the oracle shared library (plain C++ on MPFR, host only).

Usage: python oracle/build.py   -> oracle/libmps_oracle.so
MPFR/GMP headers and libraries are taken from MPFR_PREFIX (default /opt/conda).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mps_oracle.cpp")
OUT = os.path.join(HERE, "libmps_oracle.so")


def build(verbose: bool = False) -> str:
    prefix = os.environ.get("MPFR_PREFIX", "/opt/conda")
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
           "-I" + os.path.join(prefix, "include"), SRC, "-o", OUT + ".tmp",
           "-L" + os.path.join(prefix, "lib"), "-Wl,-rpath," + os.path.join(prefix, "lib"),
           "-lmpfr", "-lgmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
