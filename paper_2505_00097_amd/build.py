"""Build the HIP library libbhah.so (gfx950) in-tree.

Each source is compiled with hipcc for gfx950; the right-hand-side unit also
gets -fno-signed-zeros -ffinite-math-only so that structurally zero
reference-metric terms fold away (no reassociation is enabled).
"""
import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbhah.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast"]
SOURCES = {
    "rhs_fused.hip": DEVICE + ["-fno-signed-zeros", "-ffinite-math-only"],
    "rhs_pair.hip": DEVICE + ["-fno-signed-zeros", "-ffinite-math-only"],
    "hamiltonian.hip": DEVICE + ["-fno-signed-zeros", "-ffinite-math-only"],
    "misc.hip": DEVICE,
    "probe.hip": DEVICE,
    "grid.cpp": [],
    "capi.cpp": [],
    "engine.cpp": [],
    "batch.cpp": [],
    "server.cpp": [],
}


def _compile(name, extra, verbose):
    src = os.path.join(CSRC, name)
    obj = os.path.join(OBJ, name + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {name}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        futs = [ex.submit(_compile, n, e, verbose) for n, e in SOURCES.items()]
        objs = [f.result() for f in futs]
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
