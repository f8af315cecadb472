"""Shared helpers of the GPU parity tests (comparison metric, transfers)."""
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


def fmt(names, err):
    return ", ".join(f"{n}={e:.2e}" for n, e in zip(names, err))


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_cpu(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()

def ulp_perturbed(y, seed):
    """y with every entry moved by -1, 0 or +1 unit in the last place."""
    rng = np.random.default_rng(seed)
    return y * (1.0 + 2.220446049250313e-16 * rng.choice([-1.0, 0.0, 1.0], size=y.shape))


def rounding_floor(fn, y, err_fn, trials=2):
    """The oracle's own response to one-ulp perturbations of its input,
    measured with the same error metric: the rounding floor of the discrete
    operator on this input (any two FP64 evaluations that round differently
    can disagree by about this much)."""
    base = fn(y)
    worst = None
    for t in range(trials):
        e = err_fn(fn(ulp_perturbed(y, 1000 + t)), base)
        worst = e if worst is None else np.maximum(worst, e)
    return worst
