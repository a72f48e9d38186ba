"""Build the CPU oracle library (plain C++17, FP64, no GPU code).

TEST INFRASTRUCTURE ONLY.  ``-ffp-contract=off`` keeps every product and sum
rounded on its own, in the order the source writes it.  ``liboracle.so`` is the
serial build the tests load; ``liboracle_omp.so`` is the same source built
with OpenMP, which only the benchmark's CPU-baseline leg loads (its
target-ordered evaluation runs on all host cores; every other function is
serial and identical).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
SRC = os.path.join(HERE, "oracle.cpp")
HDR = os.path.join(HERE, "oracle.h")


def _compile(out, extra, verbose):
    cmd = ["g++", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c++17",
           "-Wall", "-Wextra", *extra, SRC, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    _compile(LIB_OMP, ["-fopenmp"], verbose)
    return _compile(LIB, ["-Wno-unknown-pragmas"], verbose)


def _stale(lib):
    return not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(SRC), os.path.getmtime(HDR))


def ensure_built() -> str:
    if _stale(LIB):
        _compile(LIB, ["-Wno-unknown-pragmas"], False)
    return LIB


def ensure_built_omp() -> str:
    if _stale(LIB_OMP):
        _compile(LIB_OMP, ["-fopenmp"], False)
    return LIB_OMP


if __name__ == "__main__":
    print(build(verbose=True))
