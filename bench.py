#!/usr/bin/env python3
"""Benchmark of the FP64 BSSN evolution on one MI355X.

One step = one classical RK4 step of the whole hot path on the workload grid:
4 right-hand-side evaluations (BSSN + gauge, Eqs. 7-15 of arXiv:2505.00097)
with the fused stage update, and the ghost fill after every stage. The
head-on workload also evaluates the Hamiltonian constraint every 50 steps.
Prints one JSON line: whole-run throughput in interior grid-point RK4
updates per second, the roofline of the right-hand-side evaluation (timed
with HIP events on the stream it runs on), and the CPU oracle's rate on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 grid-point RHS+RK4 updates/s (plain vs batched/served); p50/p99 step latency"
UNIT = "grid-point updates/s"
PEAK_FP64_VECTOR = 78.6e12  # MI355X FP64 vector FLOP/s (no MFMA: stencil code)
PEAK_HBM = 8.0e12           # bytes/s

# FP64 operations per interior point for one right-hand-side evaluation: the
# fadd/fsub/fmul/fdiv count of the optimised, fully unrolled fused kernel
# (contracted to FMAs only later, so an FMA counts 2); per
# coordinate family.
F_ALG = {0: 5892, 1: 5414, 2: 5697}
# algorithmic HBM bytes per interior point per right-hand-side evaluation:
# read 24 state gridfunctions, write 24 results (FP64)
BYTES_ALG = 24 * 8 * 2


def percentile(v, p):
    v = sorted(v)
    if not v:
        return None
    k = (len(v) - 1) * p / 100.0
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def cpu_baseline(w, budget_s):
    """The oracle as it stands, timed on the host cores on whole RK4 steps of
    the same workload until about budget_s seconds have passed."""
    from oracle import oracle as orc
    og = orc.Grid(w["coord"], w["N"], ampl=w["ampl"], sinhw=w["sinhw"], cfl=w["cfl"])
    y = og.brill_lindquist(w["masses"], w["positions"])
    dt = og.dt()
    n_int = og.N[0] * og.N[1] * og.N[2]
    steps = 0
    t0 = time.perf_counter()
    while True:
        og.rk4_step(y, dt, eta=w["eta"])
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 1000:
            break
    return {"value": n_int * steps / el, "unit": UNIT, "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{steps} RK4 steps of the {w['name']} workload ({n_int} interior points), "
                      f"{el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="headon_sinhcylindrical_128x2x256")
    ap.add_argument("--rhs-reps", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2505_00097_amd import capi
    from paper_2505_00097_amd import workloads as wl

    w = dict(wl.WORKLOADS[args.workload])
    w["name"] = args.workload
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"])
        n_int = g.info.n_interior
        y = g.state()
        ws = g.workspace()
        H = g._empty(1)
        capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y, stream=stream)
        dt = g.dt
        h_every = w.get("h_every", 0)
        for _ in range(args.warmup):
            capi.rk4_step(g.h, y, ws, dt, eta=w["eta"], stream=stream)
        torch.cuda.synchronize()

        # ---- timed region: exactly `steps` RK4 steps ----------------------
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for s in range(args.steps):
            capi.rk4_step(g.h, y, ws, dt, eta=w["eta"], stream=stream)
            if h_every and (s + 1) % h_every == 0:
                capi.hamiltonian_constraint(g.h, y, H, stream=stream)
            ev[s + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
        elapsed = t1 - t0
        finite = bool(torch.isfinite(y).all().item())

        # ---- the dominant kernel: one right-hand-side evaluation ----------
        rhs = g.state()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for _ in range(5):
            capi.bssn_rhs(g.h, y, rhs, None, eta=w["eta"], stream=stream)
        e0.record(stream)
        for _ in range(args.rhs_reps):
            capi.bssn_rhs(g.h, y, rhs, None, eta=w["eta"], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        rhs_s = e0.elapsed_time(e1) / 1e3 / args.rhs_reps

    flops = F_ALG[w["coord"]] * n_int
    achieved = flops / rhs_s
    out = {
        "metric": METRIC,
        "value": n_int * args.steps / elapsed,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Brill-Lindquist punctures, seeded)",
        "config": {"workload": args.workload, "grid": {0: "SinhSpherical", 1: "SinhCylindrical",
                                                       2: "Spherical"}[w["coord"]] +
                   " {}x{}x{}".format(*w["N"]), "interior_points": n_int,
                   "hamiltonian_every": h_every, "dt": dt, "parallelism": "single GPU"},
        "latency": {"p50_step_ms": percentile(step_ms, 50), "p99_step_ms": percentile(step_ms, 99)},
        "finite": finite,
        "roofline": {"kernel": "k_rhs_fused", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VECTOR, "traffic": None,
                     "flops_per_point": F_ALG[w["coord"]], "points": n_int, "launch_s": rhs_s,
                     "hbm_alg_GBps": BYTES_ALG * n_int / rhs_s / 1e9},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
