"""Shared helpers of the GPU parity tests (comparison metric, transfers).

The reference of every floating-point comparison is the extended-precision
build of the oracle (x87 long double). Beside it the FP64 oracle gives the
rounding error that a plain FP64 evaluation of the same discrete operator
makes on the same input. The GPU passes a case when, for every
gridfunction, its own error against the extended-precision result is at
most twice the FP64 oracle's error plus the stated tolerance (1e-12 per
right-hand side, 1e-9 after an evolution), both relative to the largest
magnitude of the gridfunction's tensor. On well-conditioned inputs the FP64
oracle's error is far below the tolerance, so this is the stated tolerance;
at ill-conditioned points (fine sinh cells near the axis and the origin,
where second differences amplify input rounding by 1/h^2) the bar is that
the GPU is no worse than the plain FP64 evaluation.
"""
import numpy as np

# gridfunctions grouped by tensor: a component is measured against the size
# of its whole tensor (components mix under a change of basis, and a
# component that vanishes by symmetry holds only round-off of that size)
GROUPS = [range(0, 6), [6], range(7, 10), [10], range(11, 17), range(17, 20), [20], range(21, 24)]


def gf_errors(gpu, cpu, interior, groups=GROUPS):
    """Per-gridfunction error: max |gpu - cpu| over interior points divided by
    the largest interior magnitude of the gridfunction's tensor (absolute
    max |gpu| where that tensor is identically zero in the oracle)."""
    out = np.zeros(gpu.shape[0])
    for grp in groups:
        m = max(np.max(np.abs(cpu[g][interior])) for g in grp)
        for g in grp:
            d = np.max(np.abs(gpu[g][interior] - cpu[g][interior]))
            out[g] = d / m if m > 0 else np.max(np.abs(gpu[g][interior]))
    return out


def _rel_errors(a, ref, pts, groups):
    """max |a - ref| over pts per gridfunction, relative to the largest |ref|
    of its tensor group (absolute where the group is zero), in float64"""
    out = np.zeros(len(ref))
    for grp in groups:
        m = max(float(np.max(np.abs(ref[g][pts]))) for g in grp)
        for g in grp:
            d = float(np.max(np.abs(a[g][pts].astype(np.longdouble) - ref[g][pts])))
            out[g] = d / m if m > 0 else d
    return out


def pointwise(a, ref, pts):
    """p50 / p99 / max of |a - ref| / |ref| over the points where |ref| exceeds
    1e-8 of its gridfunction's largest magnitude, all gridfunctions together"""
    rel = []
    for g in range(len(ref)):
        r = ref[g][pts]
        m = float(np.max(np.abs(r))) if r.size else 0.0
        if m == 0.0:
            continue
        sel = np.abs(r) > 1e-8 * m
        rel.append((np.abs(a[g][pts][sel].astype(np.longdouble) - r[sel]) / np.abs(r[sel])).astype(np.float64))
    v = np.concatenate(rel) if rel else np.zeros(1)
    return float(np.percentile(v, 50)), float(np.percentile(v, 99)), float(np.max(v))


def check_parity(label, gpu, fp64, ld, pts, tol, groups=GROUPS, names=None):
    """Assert that gpu is within 2 x (FP64 oracle's error) + tol of the
    extended-precision oracle for every gridfunction (errors relative to the
    tensor's largest magnitude over pts). Prints one PARITY line: the case,
    the worst GPU error, the worst FP64-oracle error (the rounding floor of
    a plain FP64 evaluation on this input), the worst ratio to the allowed
    bound, and the pointwise relative-error distribution of the GPU.
    With ld None (long full-size evolutions, where the extended-precision
    twin would cost minutes) the reference is the FP64 oracle itself and
    the bound is tol alone, with no allowance."""
    if ld is None:
        ld, e_cpu = fp64, np.zeros(len(fp64))
        label += " (against the FP64 oracle)"
    else:
        e_cpu = _rel_errors(fp64, ld, pts, groups)
    e_gpu = _rel_errors(gpu, ld, pts, groups)
    allowed = 2.0 * e_cpu + tol
    p50, p99, pmax = pointwise(gpu, ld, pts)
    worst = int(np.argmax(e_gpu / allowed))
    nm = names[worst] if names is not None else str(worst)
    print(f"PARITY {label} | gpu {np.max(e_gpu):.2e} | fp64 {np.max(e_cpu):.2e} | tol {tol:.0e} | "
          f"worst {nm} {e_gpu[worst]:.2e} <= {allowed[worst]:.2e} | pointwise p50 {p50:.1e} p99 {p99:.1e} "
          f"max {pmax:.1e}", flush=True)
    bad = [(names[g] if names is not None else g, e_gpu[g], allowed[g]) for g in range(len(e_gpu))
           if not e_gpu[g] <= allowed[g]]
    assert not bad, (label, bad)
    return e_gpu, e_cpu


def fmt(names, err):
    return ", ".join(f"{n}={e:.2e}" for n, e in zip(names, err))


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_cpu(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def ld(a):
    """a as the extended-precision oracle's array type"""
    return np.ascontiguousarray(a, dtype=np.longdouble)
