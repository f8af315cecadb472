"""Parity of the 8th-order path (N_G = 5 ghost layers, Sec. 3; the
differencing of the production head-on run of Sec. 4.1) with the CPU oracle,
through the C ABI. Same bars as the 4th-order parity: per right-hand side
within max(1e-12, the oracle's rounding floor) of each tensor's largest
interior magnitude; after evolution within max(1e-9, the evolution's
rounding floor); ghost maps bit-exact.
"""
import numpy as np
import pytest

from gpu_helpers import check_parity, fmt, gf_errors, ld, to_cpu, to_gpu
from oracle import oracle as orc
from paper_2505_00097_amd import workloads as wl

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
EVOL_TOL = 1e-9
NG = 5
DISS = (0.99, 0.3)

GRIDS = {
    "tiny": (wl.SINH_SPHERICAL, (32, 16, 2), (10.0,) * 3, (0.2,) * 3),
    "sph_ragged": (wl.SINH_SPHERICAL, (100, 12, 6), (10.0,) * 3, (0.2,) * 3),
    "cyl_ragged": (wl.SINH_CYLINDRICAL, (70, 2, 140), (20.0,) * 3, (0.2,) * 3),
    "cyl_3d": (wl.SINH_CYLINDRICAL, (20, 8, 30), (4.0, 4.0, 6.0), (0.3, 0.3, 0.4)),
    "spherical": (wl.SPHERICAL, (72, 12, 24), (7.5,) * 3, (0.2,) * 3),
}
HEADON = ([0.5, 0.5], [(0, 0, 0.5), (0, 0, -0.5)])


def _case(*a):
    print("CASE 8th-order", *a, flush=True)


def _pair(name, bc_kind=0, diss=(0.0, 0.0)):
    import torch  # noqa: F401
    from paper_2505_00097_amd import capi
    coord, N, ampl, w = GRIDS[name]
    return (capi.Grid(coord, N, ampl, w, bc_kind=bc_kind, nghosts=NG),
            orc.Grid(coord, N, ampl=ampl, sinhw=w, ng=NG, bc_kind=bc_kind, diss=diss))


@pytest.mark.parametrize("name", list(GRIDS))
def test_maps_and_dt_match_oracle(name):
    _case("maps", name)
    g, og = _pair(name)
    assert g.n == og.n
    assert g.dt == pytest.approx(og.dt(), rel=1e-14)
    kind, src, par = g.bc_maps()
    rc, okind, osrc, opar = og.bc_maps()
    assert rc == 0
    assert np.array_equal(kind, okind) and np.array_equal(src, osrc) and np.array_equal(par, opar)


@pytest.mark.parametrize("name", ["tiny", "cyl_ragged", "sph_ragged"])
def test_ghost_fill_and_initial_data_match_oracle(name):
    _case("bcs+id", name)
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    y0 = wl.smooth_random_state(og.n, seed=13)
    I = (slice(None),) + og.interior()
    start = np.full_like(y0, np.nan)
    start[I] = y0[I]
    ref = og.apply_bcs(start.copy())
    yg = to_gpu(start)
    capi.apply_bcs(g.h, yg)
    out = to_cpu(yg)
    assert np.all(np.isfinite(out))
    # five extrapolated layers: integer weights up to (10+15+6)^4 at a corner
    scale = np.max(np.abs(ref), axis=(1, 2, 3))
    err = np.max(np.abs(out - ref), axis=(1, 2, 3)) / scale
    assert np.all(err < 1e-9), err
    m, pos = HEADON
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y)
    ido = og.brill_lindquist(m, np.array(pos))
    assert np.max(np.abs(to_cpu(y)[I] - ido[I])) <= 4 * 2.3e-16 * np.max(np.abs(ido[I]))


def _check_rhs(g, og, y, diss=(0.0, 0.0), pts=None, label=""):
    from paper_2505_00097_amd import capi
    ref = og.rhs(y, eta=2.0)
    refl = og.twin().rhs(ld(y), eta=2.0)
    r = g.state()
    r.zero_()
    capi.bssn_rhs(g.h, to_gpu(y), r, eta=2.0, diss=diss)
    out = to_cpu(r)
    pts = og.interior() if pts is None else pts
    check_parity(f"8th order rhs{'+ko' if diss[0] else ''} {label}", out, ref, refl, pts, RHS_TOL,
                 names=orc.GF_NAMES)
    return out


@pytest.mark.parametrize("name", list(GRIDS))
def test_rhs_matches_oracle(name):
    """every coordinate family, general and two-plane variants, with and
    without Kreiss-Oliger dissipation (ninth order)"""
    g, og = _pair(name)
    _, ogd = _pair(name, diss=DISS)
    bl = og.brill_lindquist([0.6, 0.4], np.array([(0.1, 0.0, 0.5), (0.0, 0.1, -0.6)]))
    rnd = og.apply_bcs(wl.smooth_random_state(og.n, seed=7))
    for label, y in (("bl", bl), ("smooth_random", rnd)):
        _case("rhs", name, label)
        _check_rhs(g, og, y, label=f"{name} {label}")
        _case("rhs_diss", name, label)
        out = _check_rhs(g, ogd, y, diss=DISS, label=f"{name} {label}")
        if label == "smooth_random":  # the dissipation is really on
            plain = og.rhs(y, eta=2.0)
            I = (slice(None),) + og.interior()
            assert np.max(np.abs(out - plain)[I]) > 1e3 * RHS_TOL * np.max(np.abs(plain))


def test_flat_space_rhs_is_exactly_zero():
    _case("flat")
    g, og = _pair("cyl_3d")
    y = og.brill_lindquist([], np.zeros((0, 3)), lapse_kind=1)
    out = _check_rhs(g, og, y, label="cyl_3d flat")
    assert np.all(out[(slice(None),) + og.interior()] == 0.0)


@pytest.mark.parametrize("name", ["tiny", "cyl_ragged", "cyl_3d", "spherical"])
def test_radiation_rhs_matches_oracle(name):
    """the eighth-order radiation condition at the pure-outer points"""
    _case("rhs_radiation", name)
    from paper_2505_00097_amd import capi
    g, og = _pair(name, bc_kind=capi.BC_RADIATION)
    kind, _, _ = g.bc_maps()
    k = kind.reshape(og.n[2], og.n[1], og.n[0])
    y = og.apply_bcs(og.brill_lindquist([0.5, 0.3], np.array([(0.1, 0.0, 0.4), (0.0, -0.1, -0.5)])))
    _check_rhs(g, og, y, pts=(k == 0) | (k == 1), label=f"radiation {name}")
    _check_rhs(g, og, y, pts=k == 1, label=f"radiation outer {name}")


@pytest.mark.parametrize("name", ["sph_ragged", "cyl_ragged"])
def test_tile_shape_does_not_change_results(name):
    """the tile walk with five ghost layers: every shape gives the same bits"""
    _case("tiles", name)
    import torch
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    y = to_gpu(og.apply_bcs(wl.smooth_random_state(og.n, seed=3)))
    outs = []
    shapes = [(6, 0, 4), (5, 0, 1), (4, 0, 16)] if og.coord == wl.SINH_CYLINDRICAL else [(6, 0, 4), (5, 1, 1), (4, 2, 4)]
    for lx, ly, band in shapes:
        capi.grid_set_tile(g.h, lx, ly, band)
        r = g.state()
        r.zero_()
        capi.bssn_rhs(g.h, y, r, eta=2.0)
        torch.cuda.synchronize()
        outs.append(to_cpu(r))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def _evolve_pair(g, og, steps, stepper, diss, m, pos):
    """GPU, FP64 oracle and extended-precision oracle evolutions"""
    from paper_2505_00097_amd import capi
    ol = og.twin()
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y)
    ws = g.workspace()
    yo = og.brill_lindquist(m, np.array(pos).reshape(-1, 3))
    yl = ld(yo)
    dt = og.dt()
    gstep = capi.ssprk3_step if stepper == "ssprk3" else capi.rk4_step
    for s in range(steps):
        gstep(g.h, y, ws, dt, eta=2.0, diss=diss)
        for o, v in ((og, yo), (ol, yl)):
            (o.ssprk3_step if stepper == "ssprk3" else o.rk4_step)(v, dt, eta=2.0)
        if s % 10 == 9:
            print("  step", s + 1, flush=True)
    return to_cpu(y), yo, yl


@pytest.mark.parametrize("name,stepper,steps", [("tiny", "rk4", 100), ("cyl_3d", "rk4", 40),
                                                ("cyl_ragged", "ssprk3", 40)])
def test_evolution_matches_oracle(name, stepper, steps):
    _case("evolve", name, stepper, steps)
    g, og = _pair(name)
    out, yo, yl = _evolve_pair(g, og, steps, stepper, (0.0, 0.0), *HEADON)
    check_parity(f"8th order {stepper} {name} {steps} steps", out, yo, yl, (slice(None),) * 3, EVOL_TOL,
                 names=orc.GF_NAMES)


def test_production_numerics_match_oracle():
    """the production head-on numerics of Sec. 4.1 in full: 8th-order
    differences, ninth-order Kreiss-Oliger dissipation 0.99 / 0.3, the
    eighth-order radiation condition and SSPRK3"""
    _case("production", "cyl_ragged", 20)
    from paper_2505_00097_amd import capi
    g, og = _pair("cyl_ragged", bc_kind=capi.BC_RADIATION, diss=DISS)
    out, yo, yl = _evolve_pair(g, og, 20, "ssprk3", DISS, *HEADON)
    check_parity("8th order production cyl_ragged 20 steps", out, yo, yl, (slice(None),) * 3, EVOL_TOL,
                 names=orc.GF_NAMES)


def test_production_numerics_full_size_headon():
    """the head-on workload (SinhCylindrical 128x2x256) with the production
    numerics at 8th order, tuned tile shape, 30 SSPRK3 steps, every point"""
    name = "headon_sinhcylindrical_128x2x256"
    _case("production_full", name, 30)
    import torch  # noqa: F401  (device set up by torch before the library loads)
    from paper_2505_00097_amd import capi
    w = wl.WORKLOADS[name]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"], bc_kind=capi.BC_RADIATION, nghosts=NG)
    og = orc.Grid(w["coord"], w["N"], ampl=w["ampl"], sinhw=w["sinhw"], cfl=w["cfl"], ng=NG, bc_kind=1,
                  diss=DISS)
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y)
    capi.grid_tune(g.h, y, g.state(), diss=DISS)
    print("  tile", capi.grid_get_tile(g.h), flush=True)
    ws = g.workspace()
    yo = og.brill_lindquist(w["masses"], np.array(w["positions"]))
    dt = og.dt()
    for s in range(30):
        capi.ssprk3_step(g.h, y, ws, dt, eta=w["eta"], diss=DISS)
        og.ssprk3_step(yo, dt, eta=w["eta"])
        if s % 5 == 4:
            print("  step", s + 1, flush=True)
    check_parity("8th order production headon full size 30 steps", to_cpu(y), yo, None, (slice(None),) * 3,
                 EVOL_TOL, names=orc.GF_NAMES)


@pytest.mark.parametrize("name", ["tiny", "cyl_3d", "spherical"])
def test_constraints_match_oracle(name):
    _case("constraints", name)
    import torch
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    ol = og.twin()
    I = og.interior()
    groups = [[0], [1, 2, 3], [4, 5, 6]]

    def cons(o, v):
        H, M, C = o.constraints(v)
        return np.concatenate([H[None], M, C])

    for label, y in (("bl", og.brill_lindquist([0.8], [(0.1, 0.0, 0.2)])),
                     ("random", og.apply_bcs(wl.smooth_random_state(og.n, seed=8)))):
        H, M, C = g._empty(1), g._empty(3), g._empty(3)
        for t in (H, M, C):
            t.zero_()
        capi.constraints(g.h, to_gpu(y), H, M, C)
        torch.cuda.synchronize()
        got = np.concatenate([to_cpu(H), to_cpu(M), to_cpu(C)])
        check_parity(f"8th order constraints {name} {label}", got, cons(og, y), cons(ol, ld(y)), I, RHS_TOL,
                     groups=groups)
        H1 = g._empty(1)
        capi.hamiltonian_constraint(g.h, to_gpu(y), H1)
        a, b = to_cpu(H1)[0][I], got[0][I]
        assert np.max(np.abs(a - b)) <= RHS_TOL * np.max(np.abs(b))


@pytest.mark.parametrize("coord,N", [(wl.SINH_SPHERICAL, (5, 5, 2)), (wl.SINH_CYLINDRICAL, (5, 2, 5)),
                                     (wl.SPHERICAL, (5, 5, 4)), (wl.SINH_CYLINDRICAL, (7, 4, 9))])
def test_smallest_grids(coord, N):
    """Grids as narrow as five ghost layers allow: every interior point's
    radius-4 stencils (radius 5 upwinded, and the dissipation) reach the
    outermost ghost layers on both sides; RHS with dissipation and 10 SSPRK3
    steps with the radiation boundary against the oracle."""
    _case("smallest", coord, N)
    import torch  # noqa: F401  (device set up by torch before the library loads)
    from paper_2505_00097_amd import capi
    ampl = (2.0, 2.0, 3.0)
    g = capi.Grid(coord, N, ampl, (0.3,) * 3, nghosts=NG)
    og = orc.Grid(coord, N, ampl=ampl, sinhw=(0.3,) * 3, ng=NG, diss=DISS)
    y = og.apply_bcs(og.brill_lindquist([0.4], [(0.1, 0.0, 0.2)]) + 0.01 * wl.smooth_random_state(og.n, seed=2))
    _check_rhs(g, og, y, diss=DISS, label=f"smallest {coord} {N}")
    gr = capi.Grid(coord, N, ampl, (0.3,) * 3, bc_kind=capi.BC_RADIATION, nghosts=NG)
    ogr = orc.Grid(coord, N, ampl=ampl, sinhw=(0.3,) * 3, ng=NG, diss=DISS, bc_kind=1)
    olr = ogr.twin()
    yg = to_gpu(y)
    yl = ld(y)
    ws = gr.workspace()
    dt = ogr.dt()
    for _ in range(10):
        capi.ssprk3_step(gr.h, yg, ws, dt, eta=2.0, diss=DISS)
        ogr.ssprk3_step(y, dt, eta=2.0)
        olr.ssprk3_step(yl, dt, eta=2.0)
    check_parity(f"8th order smallest {coord} {N} 10 ssprk3 steps", to_cpu(yg), y, yl, (slice(None),) * 3,
                 EVOL_TOL, names=orc.GF_NAMES)


@pytest.mark.parametrize("wname", ["headon_sinhcylindrical_128x2x256", "vacuum3d_sinhspherical_256x128x64"])
def test_rhs_full_size_every_point(wname):
    """the full-size workloads at 8th order with the ninth-order dissipation,
    at the tuned tile shape: the right-hand side at every interior point
    against the oracle"""
    _case("rhs_full", wname)
    import torch  # noqa: F401
    from paper_2505_00097_amd import capi
    w = wl.WORKLOADS[wname]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"], nghosts=NG)
    og = orc.Grid(w["coord"], w["N"], ampl=w["ampl"], sinhw=w["sinhw"], cfl=w["cfl"], ng=NG, diss=DISS)
    y = og.brill_lindquist(w["masses"], w["positions"])
    y = og.apply_bcs(y + 0.05 * wl.smooth_random_state(og.n, seed=3))
    yg = to_gpu(y)
    capi.grid_tune(g.h, yg, g.state(), diss=DISS)
    r = g.state()
    r.zero_()
    capi.bssn_rhs(g.h, yg, r, eta=2.0, diss=DISS)
    out = to_cpu(r)
    del r, yg
    print("  gpu done", flush=True)
    ref = og.rhs(y, eta=2.0)
    print("  oracle done", flush=True)
    refl = og.twin().rhs(ld(y), eta=2.0)
    print("  extended-precision oracle done", flush=True)
    check_parity(f"8th order rhs+ko full size {wname}", out, ref, refl, og.interior(), RHS_TOL,
                 names=orc.GF_NAMES)


def test_ensembles_and_server_run_eighth_order_grids():
    """8th-order jobs in one ensemble with 4th-order twins of the same shapes
    (a size class holding both orders), both boundary kinds, SSPRK3 with
    dissipation and then RK4 without: every job equals its solo steps bit for
    bit. An 8th-order radiation job through the server likewise."""
    _case("ensemble_server")
    import torch
    from paper_2505_00097_amd import capi
    shapes = [(wl.SINH_CYLINDRICAL, (24, 2, 48), (8.0,) * 3, (0.3,) * 3),
              (wl.SINH_SPHERICAL, (20, 8, 4), (6.0,) * 3, (0.3,) * 3),
              (wl.SINH_CYLINDRICAL, (17, 4, 21), (6.0,) * 3, (0.3,) * 3)]
    grids = [capi.Grid(c, N, a, w, 0.5, bc_kind=bc, nghosts=ng) for c, N, a, w in shapes
             for ng in (5, 3) for bc in (capi.BC_EXTRAP, capi.BC_RADIATION)]
    ys = []
    for g in grids:
        y = g.state()
        capi.set_initial_data_brill_lindquist(g.h, *HEADON, y)
        ys.append(y)
    wss = [g.workspace() for g in grids]
    dts = [g.dt for g in grids]
    b = capi.batch_create([g.h for g in grids], eta=2.0, diss=DISS)
    capi.batch_set_integrator(b, capi.SSPRK3)
    capi.batch_set_graph_steps(b, 4)
    for integrator, diss, nsteps in ((capi.SSPRK3, DISS, 9), (capi.RK4, (0.0, 0.0), 5)):
        if integrator == capi.RK4:
            capi.batch_destroy(b)
            b = capi.batch_create([g.h for g in grids], eta=2.0)
        y0 = [y.clone() for y in ys]
        capi.batch_step(b, ys, wss, dts, nsteps=nsteps)
        torch.cuda.synchronize()
        step = capi.ssprk3_step if integrator == capi.SSPRK3 else capi.rk4_step
        for k, (g, y, a) in enumerate(zip(grids, ys, y0)):
            s_ = a.clone()
            ws = g.workspace()
            for _ in range(nsteps):
                step(g.h, s_, ws, g.dt, diss=diss)
            torch.cuda.synchronize()
            assert torch.equal(y, s_), (integrator, k)
    capi.batch_destroy(b)
    c, N, a, w = shapes[0]
    srv = capi.server_create(1e10, max_jobs=2, steps_per_tick=3, keep_results=True, integrator=capi.SSPRK3,
                             diss=DISS)
    try:
        i = capi.server_submit(srv, capi.job_desc(c, N, a, w, 0.5, *HEADON, 8, bc_kind=capi.BC_RADIATION,
                                                  nghosts=NG))
        while capi.server_job_status(srv, i).state != capi.JOB_DONE:
            capi.server_tick(srv)
        g = capi.Grid(c, N, a, w, 0.5, bc_kind=capi.BC_RADIATION, nghosts=NG)
        out = g.state()
        capi.server_fetch(srv, i, out)
        y = g.state()
        capi.set_initial_data_brill_lindquist(g.h, *HEADON, y)
        ws = g.workspace()
        for _ in range(8):
            capi.ssprk3_step(g.h, y, ws, g.dt, diss=DISS)
        torch.cuda.synchronize()
        assert torch.equal(out, y)
    finally:
        capi.server_destroy(srv)
