"""Profiling driver: right-hand-side launches on one workload grid.

Runs `--reps` launches of the fused right-hand-side kernel on the workload's
Brill-Lindquist state (after a few RK4 steps so every field is nonzero), at
a given tile shape or the one the tuner picks, then
one plain device-to-device copy of exactly `--copy-mib` MiB, whose counters
calibrate the HBM traffic counters (FETCH_SIZE / WRITE_SIZE) of a profile.
Meant to run under rocprofv3.
"""
import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="vacuum3d_sinhspherical_256x128x64")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--nghosts", type=int, default=3, help="3: 4th-order differences, 5: 8th order")
    ap.add_argument("--dissipation", action="store_true", help="Kreiss-Oliger 0.99 / 0.3 (the production run)")
    ap.add_argument("--tile", type=int, nargs=3, metavar=("LX", "LY", "BAND"),
                    help="tile shape to profile (default: the tuner's pick)")
    args = ap.parse_args()
    diss = (0.99, 0.3) if args.dissipation else (0.0, 0.0)
    import torch
    from paper_2505_00097_amd import capi
    from paper_2505_00097_amd import workloads as wl
    w = wl.WORKLOADS[args.workload]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"], nghosts=args.nghosts)
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y)
    ws = g.workspace()
    for _ in range(2):
        capi.rk4_step(g.h, y, ws, g.dt, eta=w["eta"], diss=diss)
    rhs = g.state()
    # the tile shape the benchmark runs: given, or tuned on the warm device
    if args.tile:
        capi.grid_set_tile(g.h, *args.tile)
    else:
        capi.grid_tune(g.h, y, rhs, eta=w["eta"], diss=diss)
    for _ in range(args.reps):
        capi.bssn_rhs(g.h, y, rhs, None, eta=w["eta"], diss=diss)
    n = args.copy_mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile_rhs: {args.reps} launches on {args.workload} "
          f"({g.info.n_interior} interior points), tile {' '.join(map(str, capi.grid_get_tile(g.h)))}; "
          f"copied {args.copy_mib} MiB", flush=True)


if __name__ == "__main__":
    main()
