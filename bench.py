#!/usr/bin/env python3
"""Benchmark of the FP64 BSSN evolution on one MI355X.

One step = one classical RK4 step of the whole hot path on the workload grid:
4 right-hand-side evaluations (BSSN + gauge, Eqs. 7-15 of arXiv:2505.00097)
with the fused stage update, and the ghost fill after every stage. The
head-on workload also evaluates the Hamiltonian constraint every 50 steps.
Prints one JSON line: whole-run throughput in interior grid-point RK4
updates per second, the roofline of the right-hand-side kernel (timed with
HIP events on the stream it runs on), the CPU oracle's rate on a bounded
sample of the same workload, and, beside them, the ensemble forms:
64 uneven head-on jobs advanced together against the same jobs one at a
time, and Poisson-arriving jobs served with continuous batching.
"""
import argparse
import hashlib
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

# FP64 operations per interior point for one right-hand-side evaluation, per
# (coordinate family, two phi planes): the fadd/fsub/fmul/fdiv count (an FMA
# counts 2) of the optimised per-point code, as
# paper_2505_00097_amd/count_flops.py prints it (a CPU test keeps the two in
# step). On grids with two phi planes the kernel variant drops the phi
# derivatives that vanish identically there, and its own count applies.
F_ALG = {(0, False): 5858, (0, True): 5037, (1, False): 5380, (1, True): 4553, (2, False): 5663,
         (2, True): 4842}
# the same for the 8th-order kernels (five ghost layers), with Kreiss-Oliger
# dissipation as the production head-on numerics run them
F_ALG8_KO = {(0, False): 11510, (0, True): 8220, (1, False): 11032, (1, True): 7736, (2, False): 11315,
             (2, True): 8025}


def two_planes(coord, N):
    """True where the grid has exactly two phi planes (phi = i1 on
    SinhCylindrical grids, i2 otherwise)."""
    return (N[1] if coord == 1 else N[2]) == 2


def f_alg(coord, N):
    """FP64 operations per point of the kernel variant that runs on this grid."""
    return F_ALG[(coord, two_planes(coord, N))]
# algorithmic HBM bytes per interior point per right-hand-side evaluation:
# read 24 state gridfunctions, write 24 results (FP64)
BYTES_ALG = 24 * 8 * 2
# measured HBM traffic of the right-hand-side kernel (rocprofv3 counters,
# calibrated by a copy of known size); valid only for the kernel source it
# was taken from
COUNTERS = os.path.join(ROOT, "profiles", "k_rhs_fused_headon_counters.txt")
COUNTERS_3D = os.path.join(ROOT, "profiles", "k_rhs_fused_vacuum3d_counters.txt")
COUNTERS_8 = os.path.join(ROOT, "profiles", "k_rhs_fused_headon_8th_order_counters.txt")
COUNTERS_3D_8 = os.path.join(ROOT, "profiles", "k_rhs_fused_vacuum3d_8th_order_counters.txt")
KERNEL_SOURCES = ["paper_2505_00097_amd/csrc/rhs_fused.hip", "paper_2505_00097_amd/csrc/rhs_stencil.h",
                  "paper_2505_00097_amd/csrc/rhs_common.h", "paper_2505_00097_amd/csrc/bhah_internal.h"]


_T0 = time.perf_counter()


def stamp():
    """seconds since the benchmark started, for the progress lines"""
    return "%6.1fs" % (time.perf_counter() - _T0)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counters_path(workload, nghosts=3):
    """the committed counter summary of a workload's right-hand-side kernel
    (at 8th order: the variant with the production dissipation)"""
    return {("headon_sinhcylindrical_128x2x256", 3): COUNTERS,
            ("vacuum3d_sinhspherical_256x128x64", 3): COUNTERS_3D,
            ("headon_sinhcylindrical_128x2x256", 5): COUNTERS_8,
            ("vacuum3d_sinhspherical_256x128x64", 5): COUNTERS_3D_8}.get((workload, nghosts))


def measured_traffic(workload, tile=None, nghosts=3):
    """HBM bytes per launch from the committed counter summary, or None if it
    is absent, for another workload or tile shape, or older than the kernel
    source."""
    path = counters_path(workload, nghosts)
    if not path or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash() or vals.get("workload") != workload:
        return None
    key = "hbm_bytes_per_launch"
    if tile is not None:  # the measurement at this tile shape, if one was taken
        key += "_tile_" + "_".join(str(int(t)) for t in tile)
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def roofline(kernel, flops_per_point, points, launch_s, traffic, probe=None):
    """Roofline entry of a right-hand-side kernel: algorithmic FP64
    operations and HBM bytes per launch over the measured launch time, the
    binding roof the one with the larger ideal time (FP64 vector ALU at
    78.6 TFLOP/s or HBM at 8 TB/s), and the measured HBM bytes per launch
    (traffic; None when no counters from the current sources exist)."""
    flops = flops_per_point * points
    alg_bytes = BYTES_ALG * points
    t_alu, t_mem = flops / PEAK_FP64_VECTOR, alg_bytes / PEAK_HBM
    if t_alu >= t_mem:
        bound, achieved, peak, unit = "alu", flops / launch_s / 1e12, PEAK_FP64_VECTOR / 1e12, "TFLOP/s"
    else:
        bound, achieved, peak, unit = "hbm", alg_bytes / launch_s / 1e9, PEAK_HBM / 1e9, "GB/s"
    out = {"kernel": kernel, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
           "frac": achieved / peak, "traffic": traffic, "flops_per_point": flops_per_point, "points": points,
           "launch_s": launch_s, "ideal_alu_s": t_alu, "ideal_hbm_s": t_mem,
           "hbm_alg_GBps": alg_bytes / launch_s / 1e9,
           "hbm_measured_GBps": traffic / launch_s / 1e9 if traffic else None,
           "traffic_over_algorithmic": traffic / alg_bytes if traffic else None}
    if probe:
        # ceilings measured on this device (FMA chains, streaming triad)
        out.update({"device_fp64_tflops": probe[0], "frac_of_device_fp64": flops / launch_s / 1e12 / probe[0],
                    "device_triad_GBps": probe[1]})
    return out


def kernel_name(coord, N, ko=False, nghosts=3, waves=1, tile=None):
    """The right-hand-side kernel the library launches for this grid, tile
    and mode: with row tiles (lx = 6) the one-wave kernel reads phase-1
    stencils from an LDS stage (last template argument) at 4th order, and
    at 8th order on two-phi-plane grids."""
    ax = two_planes(coord, N)
    b = lambda v: "true" if v else "false"
    if waves == 2:
        return "k_rhs_pair<%d,%s,%s,%d>" % (coord, b(ax), b(ko), nghosts)
    staged = tile is not None and tile[0] == 6 and (nghosts == 3 or ax)
    return "k_rhs_fused<%d,%s,%s,%d,%s>" % (coord, b(ax), b(ko), nghosts, b(staged))


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
    cores = orc.num_threads()
    # one more step on a single thread (same build, -O2 -fopenmp)
    orc.set_num_threads(1)
    t1 = time.perf_counter()
    og.rk4_step(y, dt, eta=w["eta"])
    el1 = time.perf_counter() - t1
    orc.set_num_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n_int * steps / el, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": f"{steps} RK4 steps of the {w['name']} workload ({n_int} interior points), "
                      f"{el:.1f} s",
            "single_thread_value": n_int / el1, "single_thread_sample": f"1 RK4 step, {el1:.1f} s",
            "cpu_model": model}


def events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def time_rhs(capi, g, y, eta, reps, stream, diss=(0.0, 0.0)):
    """Average duration of one right-hand-side launch (HIP events on the
    launch stream)."""
    import torch
    rhs = g.state()
    for _ in range(5):
        capi.bssn_rhs(g.h, y, rhs, None, eta=eta, diss=diss, stream=stream)
    e0, e1 = events(2)
    e0.record(stream)
    for _ in range(reps):
        capi.bssn_rhs(g.h, y, rhs, None, eta=eta, diss=diss, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    del rhs
    return e0.elapsed_time(e1) / 1e3 / reps


def make_grids(capi, jobs, bc_kind=0, nghosts=3):
    cache, grids = {}, []
    for j in jobs:
        key = (j["coord"], tuple(j["N"]), tuple(j["ampl"]), tuple(j["sinhw"]), j["cfl"])
        if key not in cache:
            cache[key] = capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], bc_kind, nghosts)
        grids.append(cache[key])
    return grids


def run_ssprk3(capi, wl, stream, steps, diss=(0.0, 0.0), bc_kind=0, nghosts=3, rhs_reps=0):
    """The head-on workload advanced with SSPRK3, the integrator of the
    paper's production head-on run (three right-hand sides per step), with
    optional Kreiss-Oliger dissipation (the run's strengths: 0.99, 0.3), the
    Sommerfeld outer boundary and 8th-order differences (nghosts = 5); with
    rhs_reps > 0 also the right-hand-side kernel alone (extrapolation grid of
    the same shape, same dissipation)."""
    import torch
    w = wl.WORKLOADS["headon_sinhcylindrical_128x2x256"]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"], bc_kind=bc_kind, nghosts=nghosts)
    y, ws = g.state(), g.workspace()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y, stream=stream)
    capi.grid_tune(g.h, y, g.state(), eta=w["eta"], diss=diss, stream=stream)
    for _ in range(10):
        capi.ssprk3_step(g.h, y, ws, g.dt, eta=w["eta"], diss=diss, stream=stream)
    ev = events(steps + 1)
    ev[0].record(stream)
    for s in range(steps):
        capi.ssprk3_step(g.h, y, ws, g.dt, eta=w["eta"], diss=diss, stream=stream)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    total_s = ev[0].elapsed_time(ev[-1]) / 1e3
    n = g.info.n_interior
    out = {"workload": "headon_sinhcylindrical_128x2x256 with SSPRK3"
                       + (", Kreiss-Oliger %g/%g" % diss if diss[0] or diss[1] else "")
                       + (", Sommerfeld outer boundary" if bc_kind else "")
                       + (", 8th-order differences" if nghosts == 5 else ""), "steps": steps,
           "value": n * steps / total_s, "unit": UNIT, "ms_per_step": 1e3 * total_s / steps,
           "p50_step_ms": percentile(step_ms, 50), "p99_step_ms": percentile(step_ms, 99),
           "finite": bool(torch.isfinite(y).all().item()), "tile": list(capi.grid_get_tile(g.h))}
    if rhs_reps > 0:
        ge = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"], nghosts=nghosts)
        capi.grid_set_tile(ge.h, *capi.grid_get_tile(g.h))
        ye = ge.state()
        capi.set_initial_data_brill_lindquist(ge.h, w["masses"], w["positions"], ye, stream=stream)
        rhs_s = time_rhs(capi, ge, ye, w["eta"], rhs_reps, stream, diss=diss)
        flops = (F_ALG8_KO if nghosts == 5 and (diss[0] or diss[1]) else {})
        f = flops.get((w["coord"], two_planes(w["coord"], w["N"])))
        out["rhs_launch_s"] = rhs_s
        if f is not None:
            out["rhs_flops_per_point"] = f
            out["rhs_TFLOPs"] = f * n / rhs_s / 1e12
            out["rhs_frac_fp64_peak"] = f * n / rhs_s / PEAK_FP64_VECTOR
            if nghosts == 5:
                tile = list(capi.grid_get_tile(ge.h))
                out["roofline"] = roofline(kernel_name(w["coord"], w["N"], ko=True, nghosts=5, tile=tile), f, n, rhs_s,
                                           measured_traffic("headon_sinhcylindrical_128x2x256", tile, nghosts=5))
        del ye
    return out


def run_batched(capi, wl, stream, steps, seq_steps, graph_steps, integrator=0, diss=(0.0, 0.0), bc_kind=0,
                nghosts=3, tune_launch=False):
    """64 uneven head-on jobs: one batch advancing all of them `steps` steps
    (RK4 or SSPRK3, optional dissipation and radiation boundary), against the
    same jobs advanced one at a time with the same numerics. With
    tune_launch the batch first times graph steps x blocks per CU on copies
    of the states and keeps the fastest (reported beside the default)."""
    import torch
    jobs = wl.batched_jobs()
    grids = make_grids(capi, jobs, bc_kind, nghosts)
    ys, wss = [], []
    for j, g in zip(jobs, grids):
        y = g.state()
        capi.set_initial_data_brill_lindquist(g.h, j["masses"], j["positions"], y, stream=stream)
        ys.append(y)
        wss.append(g.workspace())
    dts = [g.dt for g in grids]
    pts = sum(g.info.n_interior for g in grids)
    b = capi.batch_create([g.h for g in grids], eta=2.0, diss=diss)
    capi.batch_set_integrator(b, integrator)
    capi.batch_set_graph_steps(b, graph_steps)
    if tune_launch:
        capi.batch_set_launch_tuning(b, True)
    capi.batch_step(b, ys, wss, dts, nsteps=graph_steps, stream=stream)  # tunes tiles (and launch), captures graphs
    torch.cuda.synchronize()
    info = capi.batch_get_info(b)
    # timed in chunks of 50 steps (the engine splits each into its graphs)
    chunk = 50
    n_launch = (steps + chunk - 1) // chunk
    ev = events(n_launch + 1)
    t0 = time.perf_counter()
    ev[0].record(stream)
    done = 0
    for k in range(n_launch):
        n = min(chunk, steps - done)
        capi.batch_step(b, ys, wss, dts, nsteps=n, stream=stream)
        done += n
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    per_step = [ev[k].elapsed_time(ev[k + 1]) / min(chunk, steps - k * chunk) for k in range(n_launch)]
    finite = all(bool(torch.isfinite(y).all().item()) for y in ys)
    capi.batch_destroy(b)
    # the same jobs one after another, plain single-grid steps
    solo = capi.ssprk3_step if integrator == capi.SSPRK3 else capi.rk4_step
    e0, e1 = events(2)
    t1 = time.perf_counter()
    e0.record(stream)
    for g, y, ws in zip(grids, ys, wss):
        for _ in range(seq_steps):
            solo(g.h, y, ws, g.dt, eta=2.0, diss=diss, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t1
    batched = pts * steps / el
    seq = pts * seq_steps / el_seq
    return {"workload": "64 head-on BL jobs, SinhCylindrical N_rho~U{48..192} x 2 x 2N_rho, seed 250500097",
            "integrator": "ssprk3" if integrator == capi.SSPRK3 else "rk4", "dissipation": list(diss),
            "boundary": "radiation" if bc_kind == capi.BC_RADIATION else "extrapolation",
            "fd_order": 2 * (nghosts - 1),
            "interior_points": pts, "steps": steps, "value": batched, "unit": UNIT,
            "ms_per_step_all_jobs": el * 1e3 / steps,
            "p50_step_ms": percentile(per_step, 50), "p99_step_ms": percentile(per_step, 99),
            "sequential_value": seq, "sequential_sample": f"each job {seq_steps} steps alone, {el_seq:.2f} s",
            "speedup_vs_sequential": batched / seq, "graph_steps": info.graph_steps,
            "blocks_per_cu": info.blocks_per_cu,
            "launch_tuning": ({"graph_steps": info.graph_steps, "blocks_per_cu": info.blocks_per_cu,
                               "us_per_step": info.launch_us_per_step,
                               "default_us_per_step (10 graph steps, 4 blocks per CU)": info.launch_default_us_per_step,
                               "candidates": info.launch_candidates, "seconds": info.launch_tune_seconds,
                               "from_cache": bool(info.launch_from_cache)} if tune_launch else None),
            "tile_classes_tuned": info.n_classes_tuned, "tune_seconds": info.tune_seconds,
            "tiles": info.n_tiles, "rhs_blocks": info.rhs_blocks, "finite": finite}


def serve(capi, stream, jobs, descs, max_jobs, steps_per_tick, target_points, label, at_once=False):
    """Run jobs through a server: each submitted at its arrival time (all at
    once with at_once), ticks until every job is done. Returns the server's
    statistics and the wall time from the first arrival to the end."""
    srv = capi.server_create(200e9, max_jobs=max_jobs, steps_per_tick=steps_per_tick, keep_results=False,
                             eta=2.0, stream=stream, target_points=target_points)
    arrival = [0.0 if at_once else j["arrival"] for j in jobs]
    t0 = time.perf_counter()
    i = 0
    last_print = t0
    while True:
        now = time.perf_counter() - t0
        while i < len(jobs) and arrival[i] <= now:
            capi.server_submit(srv, descs[i])
            i += 1
        running, queued = capi.server_tick(srv)
        if running == 0 and queued == 0:
            if i >= len(jobs):
                break
            time.sleep(max(0.0, arrival[i] - (time.perf_counter() - t0)))
        if time.perf_counter() - last_print > 20.0:
            last_print = time.perf_counter()
            print(f"# {stamp()} {label}: {i}/{len(jobs)} arrived, {running} running, {queued} queued", file=sys.stderr,
                  flush=True)
    wall = time.perf_counter() - t0 - arrival[0]
    st = capi.server_get_stats(srv)
    capi.server_destroy(srv)
    return st, wall


def served_summary(st, wall):
    return {"value": st.point_steps / wall, "unit": UNIT, "wall_seconds": wall,
            "busy_value": st.point_steps / st.busy_seconds if st.busy_seconds > 0 else None,
            "busy_seconds": st.busy_seconds, "point_steps": st.point_steps, "jobs_done": st.done,
            "p50_step_ms": st.step_ms_p50, "p99_step_ms": st.step_ms_p99,
            "p50_job_s": st.job_s_p50, "p99_job_s": st.job_s_p99,
            "peak_running": st.peak_running, "peak_held_GB": st.peak_held_bytes / 1e9}


def run_served(capi, wl, stream, n_jobs, steps_per_tick, target_points, n_saturated):
    """Head-on jobs through the continuous-batching server, against the same
    jobs through the same server one at a time (max_jobs = 1, first come
    first served), both measured: the Poisson arrival trace (4 jobs/s), and
    a saturated load (the first n_saturated jobs of the trace, all arriving
    at once) where capacity rather than arrivals bounds throughput."""
    jobs = wl.served_jobs(n=n_jobs)
    descs = [capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"], j["positions"],
                           j["steps"]) for j in jobs]
    st, wall = serve(capi, stream, jobs, descs, 256, steps_per_tick, target_points, "served")
    out = {"workload": f"{n_jobs} Poisson-arriving head-on jobs (4/s), N_rho in {{64,96,128,192}}, "
                       "steps U{200..2000}, seed 250500098, 200 GB budget",
           "target_points": target_points, "steps_per_tick": steps_per_tick}
    out.update(served_summary(st, wall))
    print(f"# {stamp()} served: {out['value']:.3e} pt-steps/s", file=sys.stderr, flush=True)
    st, wall = serve(capi, stream, jobs, descs, 1, steps_per_tick, 0, "served one at a time")
    out["sequential_fcfs"] = served_summary(st, wall)
    out["sequential_fcfs"]["how"] = "the same arrivals through the same server with max_jobs = 1 (measured)"
    sat = jobs[:n_saturated]
    st, wall = serve(capi, stream, sat, descs[:n_saturated], 256, steps_per_tick, target_points, "saturated",
                     at_once=True)
    out["saturated"] = {"workload": f"the first {n_saturated} jobs of the trace, all arriving at t = 0"}
    out["saturated"].update(served_summary(st, wall))
    st, wall = serve(capi, stream, sat, descs[:n_saturated], 1, steps_per_tick, 0, "saturated one at a time",
                     at_once=True)
    out["saturated"]["sequential_fcfs"] = served_summary(st, wall)
    out["saturated"]["speedup_vs_sequential"] = out["saturated"]["value"] / out["saturated"]["sequential_fcfs"]["value"]
    print(f"# {stamp()} saturated: {out['saturated']['value']:.3e} vs one at a time "
          f"{out['saturated']['sequential_fcfs']['value']:.3e} pt-steps/s", file=sys.stderr, flush=True)
    return out


def run_rhs_study(capi, wl, stream, reps, steps):
    """Right-hand-side kernel and RK4 step on the 3-D vacuum grid."""
    import torch
    w = wl.WORKLOADS["vacuum3d_sinhspherical_256x128x64"]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"])
    y, ws = g.state(), g.workspace()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y, stream=stream)
    for _ in range(2):
        capi.rk4_step(g.h, y, ws, g.dt, eta=w["eta"], stream=stream)
    capi.grid_tune(g.h, y, g.state(), eta=w["eta"], stream=stream)
    e0, e1 = events(2)
    e0.record(stream)
    for _ in range(steps):
        capi.rk4_step(g.h, y, ws, g.dt, eta=w["eta"], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    step_s = e0.elapsed_time(e1) / 1e3 / steps
    rhs_s = time_rhs(capi, g, y, w["eta"], reps, stream)
    n = g.info.n_interior
    tile = list(capi.grid_get_tile(g.h))
    del y, ws
    torch.cuda.empty_cache()
    # the general kernel variant at 8th order with the production dissipation
    g8 = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"], nghosts=5)
    y8 = g8.state()
    capi.set_initial_data_brill_lindquist(g8.h, w["masses"], w["positions"], y8, stream=stream)
    diss = (0.99, 0.3)
    capi.grid_tune(g8.h, y8, g8.state(), eta=w["eta"], diss=diss, stream=stream)
    rhs8_s = time_rhs(capi, g8, y8, w["eta"], reps, stream, diss=diss)
    f8 = F_ALG8_KO[(w["coord"], two_planes(w["coord"], w["N"]))]
    tile8 = list(capi.grid_get_tile(g8.h))
    name = "vacuum3d_sinhspherical_256x128x64"
    eighth = {"rhs_launch_s": rhs8_s, "flops_per_point": f8, "rhs_TFLOPs": f8 * n / rhs8_s / 1e12,
              "rhs_frac_fp64_peak": f8 * n / rhs8_s / PEAK_FP64_VECTOR, "tile": tile8,
              "roofline": roofline(kernel_name(w["coord"], w["N"], ko=True, nghosts=5, tile=tile8), f8, n, rhs8_s,
                                   measured_traffic(name, tile8, nghosts=5))}
    del y8
    return {"workload": name, "interior_points": n,
            "rhs_launch_s": rhs_s, "rhs_TFLOPs": f_alg(w["coord"], w["N"]) * n / rhs_s / 1e12,
            "rhs_frac_fp64_peak": f_alg(w["coord"], w["N"]) * n / rhs_s / PEAK_FP64_VECTOR,
            "rhs_alg_GBps": BYTES_ALG * n / rhs_s / 1e9,
            "rk4_step_ms": step_s * 1e3, "value": n / step_s, "unit": UNIT,
            "tile": tile, "rhs_8th_order_with_dissipation": eighth,
            "roofline": roofline(kernel_name(w["coord"], w["N"], tile=tile), f_alg(w["coord"], w["N"]), n, rhs_s,
                                 measured_traffic(name, tile))}


def run_tiny(capi, wl, stream, steps, warmup):
    """The tiny workload (SinhSpherical 32x16x2, one puncture at the origin):
    single RK4 steps after warm-up, each timed with events (the
    latency-bound end of the range), and the flat-spacetime run, whose
    right-hand side must vanish exactly."""
    import torch
    w = wl.WORKLOADS["tiny_sinhspherical_32x16x2"]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"])
    y, ws = g.state(), g.workspace()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y, stream=stream)
    for _ in range(warmup):
        capi.rk4_step(g.h, y, ws, g.dt, eta=w["eta"], stream=stream)
    # tile shape and waves per tile: on this grid's 16 tiles two waves per
    # tile (each on its own SIMD) shorten the right-hand side
    capi.grid_tune(g.h, y, g.state(), eta=w["eta"], stream=stream)
    ev = events(steps + 1)
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(steps):
        capi.rk4_step(g.h, y, ws, g.dt, eta=w["eta"], stream=stream)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    flat = g.state()
    capi.set_initial_data_brill_lindquist(g.h, [], [], flat, lapse_kind=1, stream=stream)
    r = g.state()
    r.fill_(1.0)
    capi.bssn_rhs(g.h, flat, r, None, eta=w["eta"], stream=stream)
    ng = g.info.n_total
    interior = r.view(24, ng[2], ng[1], ng[0])[:, 3:-3, 3:-3, 3:-3]
    flat_zero = bool((interior == 0.0).all().item())
    n = g.info.n_interior
    return {"workload": "tiny_sinhspherical_32x16x2", "interior_points": n, "steps": steps,
            "tile": list(capi.grid_get_tile(g.h)), "waves_per_tile": capi.grid_get_waves_per_tile(g.h),
            "value": n * steps / wall, "unit": UNIT, "median_step_ms": percentile(ms, 50),
            "p50_step_ms": percentile(ms, 50), "p99_step_ms": percentile(ms, 99),
            "flat_spacetime_rhs_exactly_zero": flat_zero}


def run_paper_grid(capi, wl, stream, name, N, r_max, steps, graph_steps, paper):
    """One of the paper's own benchmark grids (plain Spherical, two
    punctures on z), advanced `steps` RK4 steps as a one-job batch (captured
    graphs); the paper's wall time on its hardware is quoted beside it."""
    import torch
    g = capi.Grid(wl.SPHERICAL, N, (r_max,) * 3, (0.2,) * 3, 0.5)
    y, ws = g.state(), g.workspace()
    capi.set_initial_data_brill_lindquist(g.h, [0.5, 0.5], [(0.0, 0.0, 0.5), (0.0, 0.0, -0.5)], y, stream=stream)
    b = capi.batch_create([g.h], eta=2.0)
    capi.batch_set_graph_steps(b, graph_steps)
    capi.batch_step(b, [y], [ws], [g.dt], nsteps=min(steps, graph_steps), stream=stream)  # tune + capture
    torch.cuda.synchronize()
    capi.set_initial_data_brill_lindquist(g.h, [0.5, 0.5], [(0.0, 0.0, 0.5), (0.0, 0.0, -0.5)], y, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    capi.batch_step(b, [y], [ws], [g.dt], nsteps=steps, stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    finite = bool(torch.isfinite(y).all().item())
    capi.batch_destroy(b)
    n = g.info.n_interior
    del y, ws
    return {"workload": name, "grid": "Spherical {}x{}x{}, r_max {}".format(*N, r_max), "interior_points": n,
            "steps": steps, "wall_seconds": el, "value": n * steps / el, "unit": UNIT, "finite": finite,
            "paper": paper}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="headon_sinhcylindrical_128x2x256")
    ap.add_argument("--rhs-reps", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--batched-seq-steps", type=int, default=50)
    ap.add_argument("--graph-steps", type=int, default=10)
    ap.add_argument("--served-jobs", type=int, default=256)
    ap.add_argument("--served-target-points", type=int, default=262144,
                    help="admit while running jobs hold fewer interior points (0: no limit)")
    ap.add_argument("--served-saturated-jobs", type=int, default=128,
                    help="jobs of the trace submitted at once for the saturated served leg")
    ap.add_argument("--study-steps", type=int, default=20)
    ap.add_argument("--latency-steps", type=int, default=100,
                    help="single RK4 steps timed one by one for the p50/p99 step latency")
    ap.add_argument("--tiny-steps", type=int, default=200, help="timed steps of the tiny workload (0: skip)")
    ap.add_argument("--no-paper-grids", action="store_true")
    ap.add_argument("--ssprk3-steps", type=int, default=500)
    ap.add_argument("--no-probe-peaks", action="store_true",
                    help="skip measuring the device's FP64 FMA and HBM triad ceilings")
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
        capi.grid_tune(g.h, y, g.state(), eta=w["eta"], stream=stream)  # tile shape for this grid
        tile = capi.grid_get_tile(g.h)
        torch.cuda.synchronize()

        # ---- timed region: exactly `steps` RK4 steps ----------------------
        # bhah_evolve between Hamiltonian evaluations: the stencils never
        # read the phi ghost planes, which are filled after each call's last
        # step (every ghost is valid whenever H is evaluated)
        chunk = h_every if h_every else args.steps
        bounds = list(range(0, args.steps, chunk)) + [args.steps]
        ev = events(len(bounds))
        t0 = time.perf_counter()
        ev[0].record(stream)
        for c in range(len(bounds) - 1):
            capi.evolve(g.h, y, ws, dt, bounds[c + 1] - bounds[c], eta=w["eta"], stream=stream)
            if h_every and bounds[c + 1] % h_every == 0:
                capi.hamiltonian_constraint(g.h, y, H, stream=stream)
            ev[c + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        chunk_ms = [(ev[c].elapsed_time(ev[c + 1]) / (bounds[c + 1] - bounds[c])) for c in range(len(bounds) - 1)]
        elapsed = t1 - t0
        finite = bool(torch.isfinite(y).all().item())
        print(f"# {stamp()} plain: {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
        # single-step latency: bhah_rk4_step calls, one event per step
        lat_ev = events(args.latency_steps + 1)
        lat_ev[0].record(stream)
        for s in range(args.latency_steps):
            capi.rk4_step(g.h, y, ws, dt, eta=w["eta"], stream=stream)
            lat_ev[s + 1].record(stream)
        torch.cuda.synchronize()
        step_ms = [lat_ev[i].elapsed_time(lat_ev[i + 1]) for i in range(args.latency_steps)]

        # ---- the dominant kernel: one right-hand-side evaluation ----------
        rhs_s = time_rhs(capi, g, y, w["eta"], args.rhs_reps, stream)
        del y, ws, H
        probe = None if args.no_probe_peaks else capi.probe_peaks(stream)

        extras = {}
        if args.tiny_steps > 0:
            extras["tiny"] = run_tiny(capi, wl, stream, args.tiny_steps, 20)
            print(f"# {stamp()} tiny: {extras['tiny']['value']:.3e} pt-steps/s, step p50/p99 "
                  f"{extras['tiny']['p50_step_ms']:.3f}/{extras['tiny']['p99_step_ms']:.3f} ms", file=sys.stderr,
                  flush=True)
        if args.ssprk3_steps > 0:
            # SSPRK3 without dissipation is unstable on this grid at CFL 0.5
            # (non-finite near step 480, in the oracle as well): both legs
            # carry the production dissipation and differ in the boundary
            extras["ssprk3"] = run_ssprk3(capi, wl, stream, args.ssprk3_steps, diss=(0.99, 0.3))
            extras["production_numerics"] = run_ssprk3(capi, wl, stream, args.ssprk3_steps, diss=(0.99, 0.3),
                                                        bc_kind=capi.BC_RADIATION)
            # the production head-on numerics in full (Sec. 4.1): 8th-order
            # differences, ninth-order dissipation, eighth-order radiation
            extras["production_numerics_8th_order"] = run_ssprk3(
                capi, wl, stream, args.ssprk3_steps, diss=(0.99, 0.3), bc_kind=capi.BC_RADIATION, nghosts=5,
                rhs_reps=args.rhs_reps)
            torch.cuda.empty_cache()
            print(f"# {stamp()} ssprk3 + dissipation: {extras['ssprk3']['value']:.3e} pt-steps/s, with the radiation "
                  f"boundary {extras['production_numerics']['value']:.3e}, at 8th order "
                  f"{extras['production_numerics_8th_order']['value']:.3e}", file=sys.stderr, flush=True)
        if args.batched_steps > 0:
            extras["batched"] = run_batched(capi, wl, stream, args.batched_steps, args.batched_seq_steps,
                                            args.graph_steps, tune_launch=True)
            torch.cuda.empty_cache()
            print(f"# {stamp()} batched: {extras['batched']['value']:.3e} pt-steps/s", file=sys.stderr, flush=True)
            extras["batched_production_numerics"] = run_batched(
                capi, wl, stream, args.batched_steps, args.batched_seq_steps, args.graph_steps,
                integrator=capi.SSPRK3, diss=(0.99, 0.3), bc_kind=capi.BC_RADIATION)
            torch.cuda.empty_cache()
            print(f"# {stamp()} batched, SSPRK3 + dissipation + radiation: "
                  f"{extras['batched_production_numerics']['value']:.3e} pt-steps/s", file=sys.stderr, flush=True)
            extras["batched_production_numerics_8th_order"] = run_batched(
                capi, wl, stream, args.batched_steps, args.batched_seq_steps, args.graph_steps,
                integrator=capi.SSPRK3, diss=(0.99, 0.3), bc_kind=capi.BC_RADIATION, nghosts=5)
            torch.cuda.empty_cache()
            print(f"# {stamp()} batched, production numerics at 8th order: "
                  f"{extras['batched_production_numerics_8th_order']['value']:.3e} pt-steps/s", file=sys.stderr,
                  flush=True)
        if args.study_steps > 0:
            extras["rhs_study_3d"] = run_rhs_study(capi, wl, stream, args.rhs_reps // 5 + 1, args.study_steps)
            torch.cuda.empty_cache()
            print(f"# {stamp()} 3-D study done", file=sys.stderr, flush=True)
        if not args.no_paper_grids:
            extras["paper_desktop_grid"] = run_paper_grid(
                capi, wl, stream, "the paper's single-node benchmark grid", (72, 12, 24), 7.5, 8428, 50,
                "37.2 s with NRPy/OpenMP on a 16-core Ryzen 9 3950X (62.0 s superB SMP)")
            torch.cuda.empty_cache()
            extras["paper_strong_scaling_grid"] = run_paper_grid(
                capi, wl, stream, "the paper's strong-scaling grid", (1008, 168, 336), 7.5, 124, 4,
                "about 33 s with superB on 64 nodes (7168 cores); about 1462 s with NRPy/OpenMP on one node")
            torch.cuda.empty_cache()
            print(f"# {stamp()} paper grids done", file=sys.stderr, flush=True)
        if args.served_jobs > 0:
            extras["served"] = run_served(capi, wl, stream, args.served_jobs, args.graph_steps,
                                          args.served_target_points,
                                          min(args.served_saturated_jobs, args.served_jobs))

    # the committed counters are those of the one-wave kernel
    waves = capi.grid_get_waves_per_tile(g.h)
    traffic = measured_traffic(args.workload, tile) if waves == 1 else None
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
                   "hamiltonian_every": h_every, "dt": dt, "parallelism": "single GPU",
                   "tile": list(capi.grid_get_tile(g.h)), "waves_per_tile": waves},
        "latency": {"p50_step_ms": percentile(step_ms, 50), "p99_step_ms": percentile(step_ms, 99),
                    "how": f"{args.latency_steps} single bhah_rk4_step calls after the timed region, one "
                           "event pair per step",
                    "timed_chunks_ms_per_step": chunk_ms},
        "finite": finite,
        "roofline": roofline(kernel_name(w["coord"], w["N"], waves=waves, tile=capi.grid_get_tile(g.h)),
                             f_alg(w["coord"], w["N"]), n_int, rhs_s,
                             traffic,
                             probe),
        "extras": extras,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        print(f"# {stamp()} cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
