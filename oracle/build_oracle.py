"""Build the CPU oracle (test infrastructure): oracle/liboracle.so (FP64) and
oracle/liboracle_ld.so (the same source in x87 extended precision, the
reference for the rounding error of FP64 evaluations).

The oracle is plain C compiled with gcc; it is the reference the HIP library
is checked against and is never linked into that library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_LD = os.path.join(HERE, "liboracle_ld.so")


def _build(out, extra, verbose):
    src = os.path.join(HERE, "bssn_oracle.c")
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=gnu11", "-Wall", "-Wno-unused-variable"] + extra + ["-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    _build(LIB, [], verbose)
    _build(LIB_LD, ["-DORACLE_REAL=long double"], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
