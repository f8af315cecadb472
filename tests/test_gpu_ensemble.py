"""Ensembles and serving through the C ABI.

The batched kernels run the same per-point device code as bhah_rk4_step, so
every job of a batch, and every job run by the server, must equal its solo
evolution bit for bit, whatever the tile shape, the job mix, the order of
admission or the number of steps per captured graph. The solo path itself is
checked against the oracle elsewhere; one batch job is also checked against
the oracle directly here.
"""
import json

import numpy as np
import pytest

from gpu_helpers import check_parity, to_cpu
from oracle import oracle as orc
from paper_2505_00097_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _case(*a):
    print("CASE", *a, flush=True)


def _small_jobs():
    """Mixed families, ragged sizes, one grid used by two jobs."""
    jobs = wl.batched_jobs(n=3, seed=7)
    for j in jobs:
        j["N"] = (j["N"][0] // 4, 2, j["N"][2] // 4)
    jobs.append(dict(jobs[0], masses=[0.3, 0.2], positions=[(0.0, 0.0, 0.4), (0.0, 0.0, -0.6)]))
    jobs.append(dict(coord=wl.SINH_SPHERICAL, N=(20, 10, 6), ampl=(10.0,) * 3, sinhw=(0.2,) * 3, cfl=0.5,
                     masses=[0.6, 0.4], positions=[(0.7, 0.0, 0.1), (-0.7, 0.0, -0.1)], eta=2.0))
    jobs.append(dict(coord=wl.SPHERICAL, N=(18, 6, 12), ampl=(7.5,) * 3, sinhw=(0.2,) * 3, cfl=0.5,
                     masses=[1.0], positions=[(0.0, 0.0, 0.0)], eta=2.0))
    return jobs


def _setup(jobs):
    from paper_2505_00097_amd import capi
    grids, ys, wss = [], [], []
    cache = {}
    for j in jobs:
        key = (j["coord"], tuple(j["N"]), tuple(j["ampl"]), tuple(j["sinhw"]))
        if key not in cache:
            cache[key] = capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"])
        g = cache[key]
        y = g.state()
        capi.set_initial_data_brill_lindquist(g.h, j["masses"], j["positions"], y)
        grids.append(g)
        ys.append(y)
        wss.append(g.workspace())
    return grids, ys, wss


def _solo(grids, ys0, nsteps, diss=(0.0, 0.0)):
    import torch
    from paper_2505_00097_amd import capi
    out = []
    for g, y0, n in zip(grids, ys0, nsteps):
        y = y0.clone()
        ws = g.workspace()
        for _ in range(n):
            capi.rk4_step(g.h, y, ws, g.dt, diss=diss)
        out.append(y)
    torch.cuda.synchronize()
    return out


def test_batch_matches_solo_bitwise(tmp_path):
    _case("batch mixed families")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _small_jobs()
    grids, ys, wss = _setup(jobs)
    ys0 = [y.clone() for y in ys]
    cache = str(tmp_path / "tiles.json")
    b = capi.batch_create([g.h for g in grids], eta=2.0, tune_cache_path=cache)
    capi.batch_set_graph_steps(b, 5)
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=12)
    torch.cuda.synchronize()
    info = capi.batch_get_info(b)
    assert info.n_active == len(jobs) and info.graph_steps == 5
    assert info.n_classes_tuned == len({(j["coord"], tuple(j["N"])) for j in jobs})
    solo = _solo(grids, ys0, [12] * len(jobs))
    for k, (y, s) in enumerate(zip(ys, solo)):
        assert torch.equal(y, s), k
    entries = json.load(open(cache))["entries"]
    assert len(entries) == info.n_classes_tuned
    for j in range(len(jobs)):
        lx, ly, band = capi.batch_get_tile(b, j)
        assert 3 <= lx <= 6 and 0 <= ly and lx + ly <= 6 and band >= 1
    capi.batch_destroy(b)


def test_batch_with_dissipation_matches_solo_bitwise():
    """Kreiss-Oliger dissipation in the ensemble kernels: every job equals
    its solo evolution with the same strengths, bit for bit."""
    _case("batch dissipation")
    import torch
    from paper_2505_00097_amd import capi
    diss = (0.99, 0.3)
    jobs = _small_jobs()
    grids, ys, wss = _setup(jobs)
    ys0 = [y.clone() for y in ys]
    b = capi.batch_create([g.h for g in grids], eta=2.0, diss=diss)
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=7)
    torch.cuda.synchronize()
    solo = _solo(grids, ys0, [7] * len(jobs), diss=diss)
    plain = _solo(grids, ys0, [7] * len(jobs))
    for k, (y, s, p) in enumerate(zip(ys, solo, plain)):
        assert torch.equal(y, s), k
        assert not torch.equal(y, p), k  # the dissipation is on
    capi.batch_destroy(b)


def test_batch_with_radiation_grids_matches_solo_bitwise():
    """Grids with the Sommerfeld outer boundary in an ensemble, mixed with
    extrapolation grids of the same shapes: each job equals its solo
    evolution bit for bit (outer points evolved by the same device code,
    inner ghosts copied from the one-hop lists)."""
    _case("batch radiation")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _small_jobs()
    grids, ys, wss = _setup(jobs)
    # a radiation-boundary twin of every grid, with the same initial data
    rgrids = [capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], bc_kind=capi.BC_RADIATION)
              for j in jobs]
    rys = [y.clone() for y in ys]
    rwss = [g.workspace() for g in rgrids]
    allg, ally, allw = grids + rgrids, ys + rys, wss + rwss
    y0 = [y.clone() for y in ally]
    b = capi.batch_create([g.h for g in allg], eta=2.0)
    capi.batch_set_graph_steps(b, 3)
    capi.batch_step(b, ally, allw, [g.dt for g in allg], nsteps=7)
    torch.cuda.synchronize()
    solo = _solo(allg, y0, [7] * len(allg))
    for k, (y, s) in enumerate(zip(ally, solo)):
        assert torch.equal(y, s), k
    # the two boundary kinds really differ
    assert not torch.equal(ally[0], ally[len(jobs)])
    capi.batch_destroy(b)


def test_batch_ssprk3_matches_solo_bitwise():
    """SSPRK3 ensembles (two-state stage epilogue in the batched kernel),
    with dissipation and grids of both boundary kinds: each job equals its
    solo bhah_ssprk3_step evolution bit for bit; switching back to RK4
    rebuilds the stages."""
    _case("batch ssprk3")
    import torch
    from paper_2505_00097_amd import capi
    diss = (0.99, 0.3)
    jobs = _small_jobs()
    grids, ys, wss = _setup(jobs)
    rgrids = [capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], bc_kind=capi.BC_RADIATION)
              for j in jobs[:3]]
    allg = grids + rgrids
    ally = ys + [y.clone() for y in ys[:3]]
    allw = wss + [g.workspace() for g in rgrids]
    y0 = [y.clone() for y in ally]
    b = capi.batch_create([g.h for g in allg], eta=2.0, diss=diss)
    capi.batch_set_integrator(b, capi.SSPRK3)
    capi.batch_set_graph_steps(b, 4)
    capi.batch_step(b, ally, allw, [g.dt for g in allg], nsteps=9)
    torch.cuda.synchronize()
    for k, (g, y, a) in enumerate(zip(allg, ally, y0)):
        s = a.clone()
        ws = g.workspace()
        for _ in range(9):
            capi.ssprk3_step(g.h, s, ws, g.dt, diss=diss)
        torch.cuda.synchronize()
        assert torch.equal(y, s), k
    # back to RK4 on the same batch
    capi.batch_set_integrator(b, capi.RK4)
    cur = [y.clone() for y in ally]
    capi.batch_step(b, ally, allw, [g.dt for g in allg], nsteps=2)
    solo = _solo(allg, cur, [2] * len(allg), diss=diss)
    for k, (y, s) in enumerate(zip(ally, solo)):
        assert torch.equal(y, s), k
    with pytest.raises(capi.BhahError, match="integrator"):
        capi.batch_set_integrator(b, 7)
    capi.batch_destroy(b)


def test_server_runs_radiation_jobs_with_ssprk3():
    _case("server radiation")
    import torch
    from paper_2505_00097_amd import capi
    j = _server_jobs()[0]
    srv = capi.server_create(1e10, max_jobs=2, steps_per_tick=3, keep_results=True, integrator=capi.SSPRK3)
    i = capi.server_submit(srv, capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"],
                                              j["positions"], 8, bc_kind=capi.BC_RADIATION))
    while capi.server_job_status(srv, i).state != capi.JOB_DONE:
        capi.server_tick(srv)
    g = capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], bc_kind=capi.BC_RADIATION)
    out = g.state()
    capi.server_fetch(srv, i, out)
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, j["masses"], j["positions"], y)
    ws = g.workspace()
    for _ in range(8):
        capi.ssprk3_step(g.h, y, ws, g.dt)
    torch.cuda.synchronize()
    assert torch.equal(out, y)
    capi.server_destroy(srv)


def test_batch_active_mask_and_swaps():
    _case("batch active mask")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _small_jobs()[:4]
    grids, ys, wss = _setup(jobs)
    ys0 = [y.clone() for y in ys]
    b = capi.batch_create([g.h for g in grids], eta=2.0)
    dts = [g.dt for g in grids]
    capi.batch_step(b, ys, wss, dts, active=[1, 0, 1, 0], nsteps=3)
    capi.batch_step(b, ys, wss, dts, active=[1, 1, 0, 1], nsteps=4)
    # swap job 2's state for a fresh copy: new pointers, same grid
    y2 = ys0[2].clone()
    ys[2] = y2
    capi.batch_step(b, ys, wss, dts, nsteps=2)
    torch.cuda.synchronize()
    solo = _solo(grids, ys0, [9, 6, 2, 6])
    for k, (y, s) in enumerate(zip(ys, solo)):
        assert torch.equal(y, s), k
    capi.batch_destroy(b)


# tile shapes (lx, ly, band) with extent 1 along phi (i2 on SinhSpherical,
# i1 on SinhCylindrical grids), as the stencil reads require
SPH_SHAPES = [(6, 0, 4), (5, 1, 1), (4, 2, 4), (3, 3, 1)]
CYL_SHAPES = [(6, 0, 4), (5, 0, 1), (4, 0, 1), (3, 0, 4)]


def _tile_jobs():
    return [dict(coord=wl.SINH_SPHERICAL, N=(37, 11, 6), ampl=(10.0,) * 3, sinhw=(0.2,) * 3, cfl=0.5,
                 masses=[0.6, 0.4], positions=[(0.7, 0.1, 0.0), (-0.7, 0.0, 0.2)], eta=2.0),
            dict(wl.headon_job(2.0, 1.0, 29), N=(29, 2, 45))]


def _write_cache(path, jobs, shapes):
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    lines = [json.dumps({"arch": arch, "coord": j["coord"], "N": list(j["N"]), "lx": s[0], "ly": s[1],
                         "band": s[2], "us": 1.0}) for j, s in zip(jobs, shapes)]
    path.write_text('{"bhah_tile_cache": 1, "entries": [\n' + ",\n".join(lines) + "\n]}\n")


@pytest.mark.parametrize("k", range(4))
def test_every_tile_shape_covers_each_point_once(tmp_path, k):
    """Force tile shapes through the cache file; ragged extents in all three
    directions must give the solo result exactly."""
    shapes = (SPH_SHAPES[k], CYL_SHAPES[k])
    _case("tile shapes", shapes)
    import torch
    from paper_2505_00097_amd import capi
    jobs = _tile_jobs()
    grids, ys, wss = _setup(jobs)
    ys0 = [y.clone() for y in ys]
    path = tmp_path / "tiles.json"
    _write_cache(path, jobs, shapes)
    b = capi.batch_create([g.h for g in grids], eta=2.0, tune_cache_path=str(path))
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=2)
    torch.cuda.synchronize()
    assert capi.batch_get_info(b).tune_seconds == 0.0
    for j in range(len(jobs)):
        assert capi.batch_get_tile(b, j) == shapes[j]
    solo = _solo(grids, ys0, [2, 2])
    for j, (y, s) in enumerate(zip(ys, solo)):
        assert torch.equal(y, s), (j, shapes)
    capi.batch_destroy(b)


def test_cached_shape_crossing_phi_is_ignored(tmp_path):
    """A cached tile with extent > 1 along phi is rejected and the class is
    tuned instead."""
    _case("tile shape rejected")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _tile_jobs()
    grids, ys, wss = _setup(jobs)
    path = tmp_path / "tiles.json"
    _write_cache(path, jobs, [(4, 0, 4), (5, 1, 1)])
    b = capi.batch_create([g.h for g in grids], eta=2.0, tune_cache_path=str(path))
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=1)
    torch.cuda.synchronize()
    assert capi.batch_get_info(b).tune_seconds > 0.0
    lx, ly, _ = capi.batch_get_tile(b, 0)
    assert lx + ly == 6
    assert capi.batch_get_tile(b, 1)[1] == 0
    capi.batch_destroy(b)


def test_batch_job_against_oracle():
    _case("batch vs oracle")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _small_jobs()
    grids, ys, wss = _setup(jobs)
    b = capi.batch_create([g.h for g in grids], eta=2.0)
    n = 10
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=n)
    torch.cuda.synchronize()
    for k in (0, 4):
        j = jobs[k]
        og = orc.Grid(j["coord"], j["N"], ampl=j["ampl"], sinhw=j["sinhw"], cfl=j["cfl"])
        yo = og.brill_lindquist(j["masses"], j["positions"])
        for _ in range(n):
            og.rk4_step(yo, og.dt(), eta=2.0)
        check_parity(f"batch job {k} rk4 {n} steps", to_cpu(ys[k]).reshape(yo.shape), yo, None, og.interior(), 1e-9,
                     names=orc.GF_NAMES)
    capi.batch_destroy(b)


def test_batch_ensemble_workload_sample():
    """The first 16 jobs of the 64-job ensemble at full size, 2 steps."""
    _case("batch ensemble sample")
    import torch
    from paper_2505_00097_amd import capi
    jobs = wl.batched_jobs()[:16]
    grids, ys, wss = _setup(jobs)
    ys0 = [y.clone() for y in ys]
    b = capi.batch_create([g.h for g in grids], eta=2.0)
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=2)
    torch.cuda.synchronize()
    solo = _solo(grids, ys0, [2] * len(jobs))
    for k, (y, s) in enumerate(zip(ys, solo)):
        assert torch.equal(y, s), k
    capi.batch_destroy(b)


def _server_jobs():
    base = [wl.headon_job(1.5, 1.0, 24), wl.headon_job(3.0, 1.6, 40), wl.headon_job(2.0, 0.9, 24),
            wl.headon_job(6.0, 2.5, 40), wl.headon_job(1.0, 1.2, 24)]
    steps = [7, 12, 3, 20, 0]
    for j, s in zip(base, steps):
        j["steps"] = s
    return base


def test_server_results_same_alone_and_in_mix():
    """Continuous batching: a budget of two state slots of the larger grid
    forces queueing and slot reuse; each fetched result equals the job run
    alone."""
    _case("server mix")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _server_jobs()
    gbig = capi.Grid(jobs[1]["coord"], jobs[1]["N"], jobs[1]["ampl"], jobs[1]["sinhw"], jobs[1]["cfl"])
    slab = 4 * 8 * gbig.info.state_doubles
    budget = 2 * slab
    srv = capi.server_create(budget, max_jobs=3, steps_per_tick=4, keep_results=True)
    ids = []
    for j in jobs:
        d = capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"], j["positions"],
                          j["steps"])
        ids.append(capi.server_submit(srv, d))
    results = {}
    ticks = 0
    while len(results) < len(jobs):
        running, queued = capi.server_tick(srv)
        ticks += 1
        assert ticks < 1000
        for k, i in enumerate(ids):
            st = capi.server_job_status(srv, i)
            if st.state == capi.JOB_DONE and k not in results:
                g = capi.Grid(jobs[k]["coord"], jobs[k]["N"], jobs[k]["ampl"], jobs[k]["sinhw"], jobs[k]["cfl"])
                out = g.state()
                capi.server_fetch(srv, i, out)
                assert capi.server_job_status(srv, i).state == capi.JOB_RELEASED
                assert st.steps_done == jobs[k]["steps"]
                results[k] = (g, out)
    stats = capi.server_get_stats(srv)
    assert stats.done == len(jobs) and stats.running == 0 and stats.queued == 0
    assert stats.peak_held_bytes <= budget and stats.peak_running <= 3
    assert stats.point_steps == sum(j["steps"] * j["N"][0] * j["N"][1] * j["N"][2] for j in jobs)
    for k, j in enumerate(jobs):
        g, out = results[k]
        y = g.state()
        capi.set_initial_data_brill_lindquist(g.h, j["masses"], j["positions"], y)
        (s,) = _solo([g], [y], [j["steps"]])
        assert torch.equal(out, s), k
    with pytest.raises(capi.BhahError):
        capi.server_fetch(srv, ids[0], results[0][1])
    capi.server_destroy(srv)


def test_server_rejects_job_larger_than_budget():
    _case("server budget")
    from paper_2505_00097_amd import capi
    j = wl.headon_job(1.0, 1.0, 32)
    srv = capi.server_create(1e6, max_jobs=2)
    d = capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"], j["positions"], 5)
    with pytest.raises(capi.BhahError, match="budget"):
        capi.server_submit(srv, d)
    capi.server_destroy(srv)


def test_empty_and_zero_step_calls():
    """No active job, zero steps, and a server tick with nothing submitted are
    no-ops; a job asking for zero steps finishes at once with its initial
    data."""
    _case("empty calls")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _small_jobs()[:2]
    grids, ys, wss = _setup(jobs)
    ys0 = [y.clone() for y in ys]
    b = capi.batch_create([g.h for g in grids], eta=2.0)
    capi.batch_step(b, ys, wss, [g.dt for g in grids], active=[0, 0], nsteps=5)
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=0)
    torch.cuda.synchronize()
    for y, y0 in zip(ys, ys0):
        assert torch.equal(y, y0)
    with pytest.raises(capi.BhahError):
        capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=-1)
    capi.batch_destroy(b)
    srv = capi.server_create(1e9, max_jobs=2, keep_results=True)
    assert capi.server_tick(srv) == (0, 0)
    j = jobs[0]
    i = capi.server_submit(srv, capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"],
                                              j["positions"], 0))
    capi.server_tick(srv)
    assert capi.server_job_status(srv, i).state == capi.JOB_DONE
    out = grids[0].state()
    capi.server_fetch(srv, i, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ys0[0])
    capi.server_destroy(srv)


def test_server_target_points_caps_the_running_set():
    """With the running-point target at one job's size, jobs run one at a
    time (continuous admission as each finishes); results still equal the
    solo evolution."""
    _case("server target")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _server_jobs()[:3]
    n_pts = jobs[0]["N"][0] * jobs[0]["N"][1] * jobs[0]["N"][2]
    srv = capi.server_create(1e10, max_jobs=8, steps_per_tick=3, keep_results=True, target_points=n_pts)
    ids = [capi.server_submit(srv, capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"],
                                                 j["positions"], j["steps"])) for j in jobs]
    for _ in range(200):
        running, queued = capi.server_tick(srv)
        assert running <= 1
        if running == 0 and queued == 0:
            break
    st = capi.server_get_stats(srv)
    assert st.done == 3 and st.peak_running == 1
    for k, j in enumerate(jobs):
        g = capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"])
        out = g.state()
        capi.server_fetch(srv, ids[k], out)
        y = g.state()
        capi.set_initial_data_brill_lindquist(g.h, j["masses"], j["positions"], y)
        (s,) = _solo([g], [y], [j["steps"]])
        assert torch.equal(out, s), k
    capi.server_destroy(srv)


def test_server_frees_other_shapes_for_a_job_that_would_not_fit():
    """A budget of one slot of the larger grid: two small jobs run first and
    leave their free slots behind; a large job submitted after they finish
    fits only once those slots are given back, and must still complete (no
    livelock with nothing running and the job queued). Its result equals
    the solo evolution."""
    _case("server reclaim")
    import torch
    from paper_2505_00097_amd import capi
    small = [wl.headon_job(1.5, 1.0, 24), wl.headon_job(2.0, 0.9, 24)]
    big = wl.headon_job(3.0, 1.6, 48)
    gbig = capi.Grid(big["coord"], big["N"], big["ampl"], big["sinhw"], big["cfl"])
    gsmall = capi.Grid(small[0]["coord"], small[0]["N"], small[0]["ampl"], small[0]["sinhw"], small[0]["cfl"])
    slab_big = 4 * 8 * gbig.info.state_doubles
    slab_small = 4 * 8 * gsmall.info.state_doubles
    assert 2 * slab_small <= slab_big  # both small jobs run together
    srv = capi.server_create(slab_big, max_jobs=2, steps_per_tick=4, keep_results=True)

    def desc(j, n):
        return capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"], j["positions"], n)

    ids = [capi.server_submit(srv, desc(j, 5)) for j in small]
    for _ in range(100):
        if capi.server_tick(srv) == (0, 0):
            break
    for i in ids:
        assert capi.server_job_status(srv, i).state == capi.JOB_DONE
    # release both small results: their slots stay held as free slots
    for i, j in zip(ids, small):
        g = capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"])
        capi.server_fetch(srv, i, g.state())
    assert capi.server_get_stats(srv).held_bytes > 0
    ib = capi.server_submit(srv, desc(big, 6))
    for t in range(100):
        if capi.server_tick(srv) == (0, 0):
            break
    st = capi.server_job_status(srv, ib)
    assert st.state == capi.JOB_DONE and st.steps_done == 6
    stats = capi.server_get_stats(srv)
    assert stats.peak_held_bytes <= slab_big and stats.held_bytes <= slab_big
    out = gbig.state()
    capi.server_fetch(srv, ib, out)
    y = gbig.state()
    capi.set_initial_data_brill_lindquist(gbig.h, big["masses"], big["positions"], y)
    (s,) = _solo([gbig], [y], [6])
    assert torch.equal(out, s)
    capi.server_destroy(srv)


def test_server_rejects_bad_lapse_kind_and_keeps_serving():
    """submit rejects lapse_kind outside {0, 1} before anything is queued;
    the other jobs run normally."""
    _case("server lapse_kind")
    from paper_2505_00097_amd import capi
    j = wl.headon_job(1.5, 1.0, 24)
    srv = capi.server_create(1e9, max_jobs=2, steps_per_tick=4)
    bad = capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"], j["positions"], 3)
    bad.lapse_kind = 3
    with pytest.raises(capi.BhahError, match="lapse_kind"):
        capi.server_submit(srv, bad)
    good = capi.job_desc(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"], j["masses"], j["positions"], 3)
    i = capi.server_submit(srv, good)
    for _ in range(50):
        if capi.server_tick(srv) == (0, 0):
            break
    st = capi.server_get_stats(srv)
    assert st.submitted == 1 and st.done == 1 and st.failed == 0 and st.queued == 0
    assert capi.server_job_status(srv, i).state == capi.JOB_RELEASED
    capi.server_destroy(srv)


def test_launch_tuning_leaves_results_unchanged(tmp_path):
    """Launch tuning times graph steps x blocks per CU on copies of the
    states: the jobs still advance exactly the requested steps, bit for bit
    equal to solo steps; a second batch over the same jobs takes the choice
    from the cache file without timing."""
    _case("launch tuning")
    import torch
    from paper_2505_00097_amd import capi
    jobs = _small_jobs()
    grids, ys, wss = _setup(jobs)
    ys0 = [y.clone() for y in ys]
    cache = str(tmp_path / "tiles.json")
    b = capi.batch_create([g.h for g in grids], eta=2.0, tune_cache_path=cache)
    capi.batch_set_launch_tuning(b, True)
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=6)
    torch.cuda.synchronize()
    info = capi.batch_get_info(b)
    assert info.launch_candidates == 12 and not info.launch_from_cache
    assert info.graph_steps in (4, 10, 25) and info.blocks_per_cu in (0, 2, 4, 8)
    assert info.launch_us_per_step > 0 and info.launch_default_us_per_step > 0
    assert info.launch_us_per_step <= info.launch_default_us_per_step
    solo = _solo(grids, ys0, [6] * len(jobs))
    for k, (y, s) in enumerate(zip(ys, solo)):
        assert torch.equal(y, s), k
    capi.batch_destroy(b)
    b2 = capi.batch_create([g.h for g in grids], eta=2.0, tune_cache_path=cache)
    capi.batch_set_launch_tuning(b2, True)
    capi.batch_step(b2, ys, wss, [g.dt for g in grids], nsteps=2)
    torch.cuda.synchronize()
    info2 = capi.batch_get_info(b2)
    assert info2.launch_from_cache and info2.graph_steps == info.graph_steps
    assert info2.blocks_per_cu == info.blocks_per_cu
    solo2 = _solo(grids, solo, [2] * len(jobs))
    for k, (y, s) in enumerate(zip(ys, solo2)):
        assert torch.equal(y, s), k
    capi.batch_destroy(b2)
