"""FP64 operations per interior point of one right-hand-side evaluation.

Compiles the right-hand-side kernel source to optimised device LLVM IR with
the library's own flags and counts, in each k_rhs_fused<C, AX, KO, H, STG> kernel
(AX: the variant for grids with two phi planes, whose identically vanishing
phi derivatives the compiler removes; KO: Kreiss-Oliger dissipation on; H:
ghost layers, 3 for 4th-order and 5 for 8th-order differences; STG: phase 1
through the LDS stage, the same arithmetic on the same values), the double
precision fadd / fsub / fmul / fdiv instructions (an fma or fmuladd call
counts 2) of the basic blocks that store nothing to global memory (plain or
buffer stores), less those whose results only feed such stores (the stage
combination the compiler computes ahead of its store): that is
the per-point arithmetic of Eqs. 7-15 after common-subexpression elimination,
without the RK stage combination that follows it. The result is the FLOP
figure the benchmark divides by the measured launch time.

    python paper_2505_00097_amd/count_flops.py
"""
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

COORD_NAMES = {0: "SinhSpherical", 1: "SinhCylindrical", 2: "Spherical"}


def device_ir(src):
    import build
    flags = [f for f in build.SOURCES[os.path.basename(src)]]
    out = os.path.join(tempfile.mkdtemp(prefix="bhah_ir_"), "k.ll")
    cmd = [build.HIPCC, "--offload-arch=gfx950", "--cuda-device-only", "-S", "-emit-llvm"] + flags + [src, "-o", out]
    subprocess.run(cmd, check=True, stderr=subprocess.DEVNULL)
    with open(out) as f:
        return f.read()


def count(ir, kernel_prefix="_ZN4bhah11k_rhs_fusedILi", dissipation=False, nghosts=3, staged=False):
    """{(coord, two_phi_planes): FP64 operations per point} of the kernels
    with `nghosts` ghost layers, without (or, with dissipation=True, with)
    Kreiss-Oliger dissipation; staged=True counts the forms whose phase 1
    reads stencils from the LDS stage (every variant at 4th order, the
    two-phi-plane ones at 8th)"""
    res = {}
    pat = r"(\d)ELb(\d)ELb(\d)ELi(\d)ELb(\d)E\S*)\("
    for m in re.finditer(r"define [^@]*@(" + re.escape(kernel_prefix) + pat, ir):
        if bool(int(m.group(4))) != dissipation or int(m.group(5)) != nghosts or bool(int(m.group(6))) != staged:
            continue
        name, c = m.group(1), (int(m.group(2)), bool(int(m.group(3))))
        body = ir[m.start():ir.index("\n}\n", m.start())]
        blocks = re.split(r"\n(?=[\w.]+:)", body)
        stores = [bool(re.search(r"store double [^,]+, ptr addrspace\(1\)", b)) or "buffer.store" in b for b in blocks]
        # FP64 operations of the blocks that store nothing, by result name and weight
        ops, uses = {}, {}
        for bi, blk in enumerate(blocks):
            for line in blk.split("\n"):
                d = re.match(r"\s*(%[\w.]+) = (?:(?:fadd|fsub|fmul|fdiv)(?: [a-z ]+)? double|"
                             r".*call [a-z ]*double @llvm\.(?:fma|fmuladd)\.f64)", line)
                if d and not stores[bi]:
                    ops[d.group(1)] = 2 if "llvm.fma" in line else 1
                for u in re.findall(r"%[\w.]+", line.split("=", 1)[1] if " = " in line else line):
                    uses.setdefault(u, []).append((bi, d.group(1) if d else None))
        # an operation whose every use is a store block's, or another such
        # operation's, is the stage combination computed ahead of its store
        dead = set()
        changed = True
        while changed:
            changed = False
            for v in ops:
                if v in dead:
                    continue
                us = uses.get(v, [])
                if us and all(stores[bi] or (r is not None and r in dead) for bi, r in us):
                    dead.add(v)
                    changed = True
        res[c] = sum(w for v, w in ops.items() if v not in dead)
    return res


def main():
    ir = device_ir(os.path.join(HERE, "csrc", "rhs_fused.hip"))
    for ng in (3, 5):
        for ko in (False, True):
            staged = count(ir, dissipation=ko, nghosts=ng, staged=True)
            for (c, ax), n in sorted(count(ir, dissipation=ko, nghosts=ng).items()):
                st = f" (staged form: {staged[(c, ax)]})" if (c, ax) in staged else ""
                print(f"order {2 * (ng - 1)}: {COORD_NAMES[c]}{' (two phi planes)' if ax else ''}"
                      f"{' + dissipation' if ko else ''}: {n} FP64 operations per point{st}")


if __name__ == "__main__":
    main()
