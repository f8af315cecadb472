"""Shared helpers of the GPU parity tests (comparison metric, transfers).

The reference of every floating-point comparison is the extended-precision
build of the oracle (x87 long double). Beside it the FP64 oracle gives the
rounding error that a plain FP64 evaluation of the same discrete operator
makes on the same input. The GPU passes a case when, for every
gridfunction g, its own error against the extended-precision result is at
most twice the FP64 oracle's error plus the stated tolerance (1e-12 per
right-hand side, 1e-9 after an evolution) times the gridfunction's own
largest magnitude:
    max|gpu_g - ld_g| <= 2 max|fp64_g - ld_g| + tol * max|ld_g|.
Two cases take another scale for the tolerance term: a component that
vanishes by symmetry (its largest magnitude below 1e-6 of its tensor's)
holds only round-off of the tensor's size and is measured against the
tensor; a tensor that is identically zero in the reference must come out
within twice the FP64 oracle's error plus 1e-30. On well-conditioned
inputs the FP64 oracle's error is far below the tolerance, so this is the
stated tolerance; at ill-conditioned points (fine sinh cells near the axis
and the origin, where second differences amplify input rounding by 1/h^2)
the bar is that the GPU is no worse than the plain FP64 evaluation.
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


def _scales(ref, pts, groups):
    """the scale of each gridfunction's tolerance term: its own largest
    magnitude over pts, its tensor's where it vanishes by symmetry (below
    1e-6 of the tensor's), 0 where the whole tensor is zero"""
    out = np.zeros(len(ref))
    for grp in groups:
        own = {g: float(np.max(np.abs(ref[g][pts]))) for g in grp}
        m = max(own.values())
        for g in grp:
            out[g] = own[g] if own[g] >= 1e-6 * m else m
    return out


def _abs_errors(a, ref, pts):
    """max |a - ref| over pts per gridfunction, in float64"""
    return np.array([float(np.max(np.abs(a[g][pts].astype(np.longdouble) - ref[g][pts]))) for g in range(len(ref))])


def pointwise(a, ref, pts, groups=GROUPS):
    """p50 / p99 / max of |a - ref| / |ref| over the points where |ref| exceeds
    1e-8 of its gridfunction's largest magnitude, all gridfunctions together;
    components that vanish by symmetry (largest magnitude below 1e-6 of their
    tensor's, round-off only) are left out"""
    rel = []
    for grp in groups:
        own = {g: float(np.max(np.abs(ref[g][pts]))) if ref[g][pts].size else 0.0 for g in grp}
        top = max(own.values())
        for g in grp:
            m = own[g]
            if m == 0.0 or m < 1e-6 * top:
                continue
            r = ref[g][pts]
            sel = np.abs(r) > 1e-8 * m
            rel.append((np.abs(a[g][pts][sel].astype(np.longdouble) - r[sel]) / np.abs(r[sel])).astype(np.float64))
    v = np.concatenate(rel) if rel else np.zeros(1)
    return float(np.percentile(v, 50)), float(np.percentile(v, 99)), float(np.max(v))


def check_parity(label, gpu, fp64, ld, pts, tol, groups=GROUPS, names=None):
    """Assert that gpu is within 2 x (FP64 oracle's error) + tol x scale of
    the extended-precision oracle for every gridfunction (the rule and the
    scales in the module docstring). Prints one PARITY line: the case,
    the worst GPU error, the worst FP64-oracle error (the rounding floor of
    a plain FP64 evaluation on this input), the worst ratio to the allowed
    bound, and the pointwise relative-error distribution of the GPU.
    With ld None (long full-size evolutions, where the extended-precision
    twin would cost minutes) the reference is the FP64 oracle itself and
    the bound is tol alone, with no allowance."""
    scale = _scales(ld if ld is not None else fp64, pts, groups)
    if ld is None:
        ld, d_cpu = fp64, np.zeros(len(fp64))
        label += " (against the FP64 oracle)"
    else:
        d_cpu = _abs_errors(fp64, ld, pts)
    d_gpu = _abs_errors(gpu, ld, pts)
    allowed = 2.0 * d_cpu + np.where(scale > 0, tol * scale, 1e-30)
    # relative errors for the report (absolute where the tensor is zero)
    rel = np.where(scale > 0, scale, 1.0)
    e_gpu, e_cpu = d_gpu / rel, d_cpu / rel
    p50, p99, pmax = pointwise(gpu, ld, pts, groups)
    worst = int(np.argmax(d_gpu / allowed))
    nm = names[worst] if names is not None else str(worst)
    print(f"PARITY {label} | gpu {np.max(e_gpu):.2e} | fp64 {np.max(e_cpu):.2e} | tol {tol:.0e} | "
          f"worst {nm} {e_gpu[worst]:.2e} <= {allowed[worst] / rel[worst]:.2e} | pointwise p50 {p50:.1e} "
          f"p99 {p99:.1e} max {pmax:.1e}", flush=True)
    bad = [(names[g] if names is not None else g, e_gpu[g], allowed[g] / rel[g]) for g in range(len(e_gpu))
           if not d_gpu[g] <= allowed[g]]
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
