"""Parity of the HIP library (through the C ABI) with the CPU oracle.

Tolerances: per right-hand side, every gridfunction within 1e-12 of the
oracle relative to the largest interior magnitude of its tensor -- or, where
larger, within the oracle's own rounding floor on that input (its response
to one-ulp perturbations of the input: second differences on cells of size h
turn input rounding eps |f| into eps |f| / h^2 of output noise, which for
weak-field data on fine sinh cells exceeds 1e-12 of the result); after 100
RK4 steps within 1e-9; integer work (ghost maps) bit-exact; ghost copies
exact.
"""
import numpy as np
import pytest

from gpu_helpers import check_parity, fmt, gf_errors, ld, to_cpu, to_gpu
from oracle import oracle as orc
from paper_2505_00097_amd import workloads as wl

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
EVOL_TOL = 1e-9

GRIDS = {
    "tiny": (wl.SINH_SPHERICAL, (32, 16, 2), (10.0,) * 3, (0.2,) * 3),
    "sph_ragged": (wl.SINH_SPHERICAL, (100, 12, 6), (10.0,) * 3, (0.2,) * 3),
    "cyl_ragged": (wl.SINH_CYLINDRICAL, (70, 2, 140), (20.0,) * 3, (0.2,) * 3),
    "cyl_3d": (wl.SINH_CYLINDRICAL, (20, 8, 30), (4.0, 4.0, 6.0), (0.3, 0.3, 0.4)),
    "spherical": (wl.SPHERICAL, (72, 12, 24), (7.5,) * 3, (0.2,) * 3),
}


def _pair(name):
    import torch  # noqa: F401
    from paper_2505_00097_amd import capi
    coord, N, ampl, w = GRIDS[name]
    return capi.Grid(coord, N, ampl, w), orc.Grid(coord, N, ampl=ampl, sinhw=w)


def _interior(og):
    return og.interior()


def _print_case(*a):
    print("CASE", *a, flush=True)


@pytest.mark.parametrize("name", list(GRIDS))
def test_grid_info_and_maps_match_oracle(name):
    _print_case("maps", name)
    g, og = _pair(name)
    assert g.dt == pytest.approx(og.dt(), rel=1e-14)
    kind, src, par = g.bc_maps()
    rc, okind, osrc, opar = og.bc_maps()
    assert rc == 0
    assert np.array_equal(kind, okind) and np.array_equal(src, osrc) and np.array_equal(par, opar)
    assert g.info.n_pure_outer == np.sum(okind == 1) and g.info.n_inner == np.sum(okind == 2)


@pytest.mark.parametrize("name", ["tiny", "cyl_ragged", "cyl_3d", "sph_ragged"])
def test_apply_bcs_matches_oracle(name):
    _print_case("bcs", name)
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    y0 = wl.smooth_random_state(og.n, seed=11)
    I = (slice(None),) + og.interior()
    ycpu_poison = np.full_like(y0, np.nan)
    ycpu_poison[I] = y0[I]
    og.apply_bcs(ycpu_poison)
    # every ghost starts as NaN on the device too: a ghost the fill misses
    # (or a fill that reads another ghost) stays non-finite
    start = np.full_like(y0, np.nan)
    start[I] = y0[I]
    yg = to_gpu(start)
    capi.apply_bcs(g.h, yg)
    out = to_cpu(yg)
    assert np.all(np.isfinite(out))
    kind, src, par = g.bc_maps()
    k = kind.reshape(og.n[2], og.n[1], og.n[0])
    ref = ycpu_poison
    # copies from interior sources are exact
    interior_src = (k == 2) & (kind[src].reshape(k.shape) == 0)
    assert np.array_equal(out[:, interior_src], ref[:, interior_src])
    # outer ghosts: the library evaluates each as one integer-weighted sum of
    # up to 9 interior values (sum of |weights| at most (10+15+6)^2 = 961 at a
    # corner), the oracle extrapolates layer by layer; both round differently,
    # by at most ~ 961 * 9 * eps relative to the field's magnitude.
    scale = np.max(np.abs(ref), axis=(1, 2, 3))
    err = np.max(np.abs(out - ref), axis=(1, 2, 3)) / scale
    assert np.all(err < 961 * 9 * 2.3e-16), err


@pytest.mark.parametrize("name,m,pos,lapse", [
    ("tiny", [1.0], [(0, 0, 0)], 0),
    ("cyl_ragged", [0.5, 0.5], [(0, 0, 0.5), (0, 0, -0.5)], 0),
    ("sph_ragged", [0.6, 0.4], [(0.7, 0, 0), (-0.7, 0, 0)], 1),
    ("spherical", [], [], 1),
])
def test_initial_data_matches_oracle(name, m, pos, lapse):
    _print_case("id", name)
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y, lapse_kind=lapse)
    out = to_cpu(y)
    ref = og.brill_lindquist(m, np.array(pos).reshape(-1, 3), lapse_kind=lapse)
    I = (slice(None),) + og.interior()
    # interior: same formula, rounding differs by FMA contraction only
    assert np.max(np.abs(out[I] - ref[I])) <= 4 * 2.3e-16 * max(1.0, np.max(np.abs(ref[I])))
    # ghosts: the fill's bound (see test_apply_bcs_matches_oracle)
    assert np.max(np.abs(out - ref)) <= 961 * 9 * 2.3e-16 * max(1.0, np.max(np.abs(ref)))


def _rhs_gpu(g, yc, eta=2.0):
    from paper_2505_00097_amd import capi
    y = to_gpu(yc)
    r = g.state()
    r.zero_()
    aux = g.aux()
    capi.bssn_rhs(g.h, y, r, aux, eta=eta)
    return to_cpu(r), to_cpu(aux)


def _states(name, og):
    """(label, state) inputs for the per-RHS parity."""
    out = []
    if name == "tiny":
        flat = og.brill_lindquist([], np.zeros((0, 3)), lapse_kind=1)
        out.append(("flat", flat))
        bl = og.brill_lindquist([1.0], [(0, 0, 0)])
        out.append(("bl_t0", bl))
        ev = bl.copy()
        for _ in range(10):
            og.rk4_step(ev, og.dt(), eta=2.0)
        out.append(("bl_10_oracle_steps", ev))
    if name == "cyl_ragged":
        out.append(("bl_headon", og.brill_lindquist([0.5, 0.5], [(0, 0, 0.5), (0, 0, -0.5)])))
    # inputs carry valid ghosts, as the right-hand side requires
    out.append(("smooth_random", og.apply_bcs(wl.smooth_random_state(og.n, seed=5))))
    return out


@pytest.mark.parametrize("name", ["tiny", "sph_ragged", "cyl_ragged", "cyl_3d", "spherical"])
def test_rhs_matches_oracle(name):
    g, og = _pair(name)
    ol = og.twin()
    for label, y in _states(name, og):
        _print_case("rhs", name, label)
        ref = og.rhs(y, eta=2.0)
        refl = ol.rhs(ld(y), eta=2.0)
        out, aux = _rhs_gpu(g, y)
        I = og.interior()
        check_parity(f"rhs {name} {label}", out, ref, refl, I, RHS_TOL, names=orc.GF_NAMES)
        if label == "flat":
            assert np.all(out[(slice(None),) + I] == 0.0)
        # the Ricci tensor the right-hand side used
        pts = np.array([og.flat(i0, i1, i2) for i2 in range(3, 3 + og.N[2]) for i1 in range(3, 3 + og.N[1])
                        for i0 in range(3, 3 + og.N[0])])
        ric = og.rhs_points(y, pts, want_ricci=True)[1]
        ricl = ol.rhs_points(ld(y), pts, want_ricci=True)[1]
        gr = np.stack([aux[c].reshape(-1)[pts] for c in range(6)], -1)
        check_parity(f"ricci {name} {label}", gr.T, ric.T, ricl.T, slice(None), RHS_TOL, groups=[range(6)])


DISS = (0.99, 0.3)  # Kreiss-Oliger strengths of the paper's head-on run (gauge, metric)


def _oracle_diss(name):
    coord, N, ampl, w = GRIDS[name]
    return orc.Grid(coord, N, ampl=ampl, sinhw=w, diss=DISS)


@pytest.mark.parametrize("name", ["tiny", "sph_ragged", "cyl_ragged", "cyl_3d", "spherical"])
def test_rhs_with_dissipation_matches_oracle(name):
    """The kernels built with Kreiss-Oliger dissipation (general and two-plane
    variants of every coordinate family) against the oracle's."""
    from paper_2505_00097_amd import capi
    g, og0 = _pair(name)
    og = _oracle_diss(name)
    ol = og.twin()
    for label, y in _states(name, og):
        _print_case("rhs_diss", name, label)
        ref = og.rhs(y, eta=2.0)
        refl = ol.rhs(ld(y), eta=2.0)
        yg = to_gpu(y)
        r = g.state()
        r.zero_()
        capi.bssn_rhs(g.h, yg, r, eta=2.0, diss=DISS)
        out = to_cpu(r)
        I = og.interior()
        check_parity(f"rhs+ko {name} {label}", out, ref, refl, I, RHS_TOL, names=orc.GF_NAMES)
        if label == "smooth_random":  # the dissipation is really on
            plain = og0.rhs(y, eta=2.0)
            assert np.max(np.abs(out - plain)[(slice(None),) + I]) > 1e3 * RHS_TOL * np.max(np.abs(plain))


@pytest.mark.parametrize("name,m,pos,steps", [
    ("cyl_ragged", [0.5, 0.5], [(0, 0, 0.5), (0, 0, -0.5)], 40),
    ("sph_ragged", [0.6, 0.4], [(0.7, 0, 0), (-0.7, 0, 0)], 20),
])
def test_ssprk3_with_dissipation_matches_oracle(name, m, pos, steps):
    """The integrator and dissipation of the paper's production head-on run
    (SSPRK3, Kreiss-Oliger 0.99 / 0.3) against the oracle."""
    _print_case("evolve_ssprk3_diss", name, steps)
    from paper_2505_00097_amd import capi
    g, _ = _pair(name)
    og = _oracle_diss(name)
    ol = og.twin()
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y)
    ws = g.workspace()
    yo = og.brill_lindquist(m, np.array(pos).reshape(-1, 3))
    yl = ld(yo)
    dt = og.dt()
    for _ in range(steps):
        capi.ssprk3_step(g.h, y, ws, dt, eta=2.0, diss=DISS)
        og.ssprk3_step(yo, dt, eta=2.0)
        ol.ssprk3_step(yl, dt, eta=2.0)
    check_parity(f"ssprk3+ko {name} {steps} steps", to_cpu(y), yo, yl, og.interior(), EVOL_TOL,
                 names=orc.GF_NAMES)


def _pair_radiation(name):
    from paper_2505_00097_amd import capi
    coord, N, ampl, w = GRIDS[name]
    return (capi.Grid(coord, N, ampl, w, bc_kind=capi.BC_RADIATION),
            orc.Grid(coord, N, ampl=ampl, sinhw=w, bc_kind=1))


@pytest.mark.parametrize("name", ["tiny", "cyl_ragged", "cyl_3d", "spherical"])
def test_radiation_rhs_matches_oracle(name):
    """With the Sommerfeld outer boundary the right-hand side covers the
    pure-outer points too: both against the oracle."""
    from paper_2505_00097_amd import capi
    g, og = _pair_radiation(name)
    ol = og.twin()
    kind, _, _ = g.bc_maps()
    k = kind.reshape(og.n[2], og.n[1], og.n[0])
    pts = (k == 0) | (k == 1)
    outer = k == 1
    bl = og.apply_bcs(og.brill_lindquist([0.5, 0.3], [(0.1, 0.0, 0.4), (0.0, -0.1, -0.5)]))
    for label, y in (("bl", bl), ("smooth_random", og.apply_bcs(wl.smooth_random_state(og.n, seed=21)))):
        _print_case("rhs_radiation", name, label)
        ref = og.rhs(y, eta=2.0)
        refl = ol.rhs(ld(y), eta=2.0)
        yg = to_gpu(y)
        r = g.state()
        r.zero_()
        capi.bssn_rhs(g.h, yg, r, eta=2.0)
        out = to_cpu(r)
        check_parity(f"rhs radiation {name} {label}", out, ref, refl, pts, RHS_TOL, names=orc.GF_NAMES)
        # the outer points on their own, against their own magnitude
        check_parity(f"rhs radiation outer {name} {label}", out, ref, refl, outer, RHS_TOL, names=orc.GF_NAMES)


@pytest.mark.parametrize("name,steps", [("tiny", 100), ("cyl_ragged", 30)])
def test_radiation_rk4_evolution_matches_oracle(name, steps):
    _print_case("evolve_radiation", name, steps)
    from paper_2505_00097_amd import capi
    g, og = _pair_radiation(name)
    ol = og.twin()
    m, pos = [0.5, 0.5], [(0, 0, 0.5), (0, 0, -0.5)]
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y)
    ws = g.workspace()
    yo = og.brill_lindquist(m, np.array(pos).reshape(-1, 3))
    yl = ld(yo)
    dt = og.dt()
    for _ in range(steps):
        capi.rk4_step(g.h, y, ws, dt, eta=2.0)
        og.rk4_step(yo, dt, eta=2.0)
        ol.rk4_step(yl, dt, eta=2.0)
    # every point, ghosts included
    check_parity(f"rk4 radiation {name} {steps} steps", to_cpu(y), yo, yl, (slice(None),) * 3, EVOL_TOL,
                 names=orc.GF_NAMES)


def test_production_numerics_match_oracle():
    """The head-on run's numerics of Sec. 4.1 at 4th order: SSPRK3, Kreiss-
    Oliger dissipation 0.99 / 0.3 and the Sommerfeld outer boundary."""
    _print_case("evolve_production", "cyl_ragged", 20)
    from paper_2505_00097_amd import capi
    coord, N, ampl, w = GRIDS["cyl_ragged"]
    g = capi.Grid(coord, N, ampl, w, bc_kind=capi.BC_RADIATION)
    og = orc.Grid(coord, N, ampl=ampl, sinhw=w, bc_kind=1, diss=DISS)
    ol = og.twin()
    m, pos = [0.5, 0.5], [(0, 0, 0.5), (0, 0, -0.5)]
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y)
    ws = g.workspace()
    yo = og.brill_lindquist(m, np.array(pos).reshape(-1, 3))
    yl = ld(yo)
    dt = og.dt()
    for _ in range(20):
        capi.ssprk3_step(g.h, y, ws, dt, eta=2.0, diss=DISS)
        og.ssprk3_step(yo, dt, eta=2.0)
        ol.ssprk3_step(yl, dt, eta=2.0)
    check_parity("production cyl_ragged 20 steps", to_cpu(y), yo, yl, (slice(None),) * 3, EVOL_TOL,
                 names=orc.GF_NAMES)


@pytest.mark.parametrize("production", [False, True])
def test_ssprk3_full_size_headon(production):
    """The benchmark's SSPRK3 legs at full size: the head-on workload
    (SinhCylindrical 128x2x256) with SSPRK3 alone, and with the production
    numerics (Kreiss-Oliger 0.99 / 0.3 and the Sommerfeld outer boundary),
    tuned tile shape, 30 steps, against the oracle over every point."""
    name = "headon_sinhcylindrical_128x2x256"
    _print_case("evolve_ssprk3_full", name, production, 30)
    from paper_2505_00097_amd import capi
    w = wl.WORKLOADS[name]
    diss = DISS if production else (0.0, 0.0)
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"],
                  bc_kind=capi.BC_RADIATION if production else capi.BC_EXTRAP)
    og = orc.Grid(w["coord"], w["N"], ampl=w["ampl"], sinhw=w["sinhw"], cfl=w["cfl"],
                  bc_kind=1 if production else 0, diss=diss)
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y)
    capi.grid_tune(g.h, y, g.state(), diss=diss)
    ws = g.workspace()
    yo = og.brill_lindquist(w["masses"], w["positions"])
    dt = og.dt()
    for s in range(30):
        capi.ssprk3_step(g.h, y, ws, dt, eta=w["eta"], diss=diss)
        og.ssprk3_step(yo, dt, eta=w["eta"])
        if s % 5 == 4:
            print("  step", s + 1, flush=True)
    check_parity(f"ssprk3{' production' if production else ''} headon full size 30 steps", to_cpu(y), yo, None,
                 (slice(None),) * 3, EVOL_TOL, names=orc.GF_NAMES)


def test_axisymmetric_evolution_keeps_phi_slices_equal():
    """phi-independent data on an 8-plane SinhSpherical grid (the general
    kernel, phi wrapped): after 20 RK4 steps on the GPU every phi slice is
    bitwise equal and the components with an odd number of phi indices are
    exactly zero."""
    _print_case("axisymmetry")
    import test_oracle_symmetry as sym
    from paper_2505_00097_amd import capi
    coord, N, ampl, w = wl.SINH_SPHERICAL, (16, 8, 8), (6.0,) * 3, (0.3,) * 3
    g = capi.Grid(coord, N, ampl, w)
    og = orc.Grid(coord, N, ampl=ampl, sinhw=w)
    y = to_gpu(sym.axisymmetric_bl(og, [0.6, 0.4], [(0, 0, 0.7), (0, 0, -0.6)]))
    ws = g.workspace()
    for _ in range(20):
        capi.rk4_step(g.h, y, ws, g.dt)
    out = to_cpu(y)
    for k in range(out.shape[1]):
        assert np.array_equal(out[:, k], out[:, og.ng]), k
    for k in sym.ODD_PHI_OR_Z:
        assert np.max(np.abs(out[k])) == 0.0, orc.GF_NAMES[k]


@pytest.mark.parametrize("production", [False, True])
def test_headon_equatorial_mirror_symmetry(production):
    """The full-size head-on workload (equal masses at z = +-0.5) stays
    mirror-symmetric across z = 0 on the GPU: 20 RK4 steps, or 20 steps of
    the production numerics (SSPRK3, Kreiss-Oliger, radiation boundary)."""
    name = "headon_sinhcylindrical_128x2x256"
    _print_case("mirror", name, production)
    import test_oracle_symmetry as sym
    from paper_2505_00097_amd import capi
    w = wl.WORKLOADS[name]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"],
                  bc_kind=capi.BC_RADIATION if production else capi.BC_EXTRAP)
    og = orc.Grid(w["coord"], w["N"], ampl=w["ampl"], sinhw=w["sinhw"], cfl=w["cfl"])
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y)
    ws = g.workspace()
    for _ in range(20):
        if production:
            capi.ssprk3_step(g.h, y, ws, g.dt, eta=w["eta"], diss=DISS)
        else:
            capi.rk4_step(g.h, y, ws, g.dt, eta=w["eta"])
    out = to_cpu(y)
    I = og.interior()
    err = sym.mirror_errors(out, I)
    print("  mirror", fmt(orc.GF_NAMES, err), flush=True)
    assert np.all(err <= 1e-10), fmt(orc.GF_NAMES, err)
    assert np.max(np.abs(out[orc.GF_NAMES.index("vetU2")][I])) > 1e-8


def test_rhs_is_deterministic():
    _print_case("determinism")
    g, og = _pair("sph_ragged")
    y = wl.smooth_random_state(og.n, seed=9)
    a, _ = _rhs_gpu(g, y)
    b, _ = _rhs_gpu(g, y)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("wname", ["headon_sinhcylindrical_128x2x256", "vacuum3d_sinhspherical_256x128x64"])
def test_rhs_full_size_every_point(wname):
    """Full-size workloads at the benchmark's launch configuration (the tuned
    tile shape): the right-hand side at every interior point against the
    oracle."""
    _print_case("rhs_full", wname)
    from paper_2505_00097_amd import capi
    w = wl.WORKLOADS[wname]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"])
    og = orc.Grid(w["coord"], w["N"], ampl=w["ampl"], sinhw=w["sinhw"], cfl=w["cfl"])
    y = og.brill_lindquist(w["masses"], w["positions"])
    y = og.apply_bcs(y + 0.05 * wl.smooth_random_state(og.n, seed=3))
    capi.grid_tune(g.h, to_gpu(y), g.state())
    out, _ = _rhs_gpu(g, y)
    print("  gpu done", flush=True)
    ref = og.rhs(y, eta=2.0)
    print("  oracle done", flush=True)
    refl = og.twin().rhs(ld(y), eta=2.0)
    print("  extended-precision oracle done", flush=True)
    check_parity(f"rhs full size {wname}", out, ref, refl, og.interior(), RHS_TOL, names=orc.GF_NAMES)


def _bl_boxes(og, points, masses, pos):
    """A state that is flat (W = alpha = 1, all else 0) except in the 7^3 index
    box around each point, where it holds Brill-Lindquist W = alpha =
    psi^-2 evaluated at the box points (plain Spherical grid, phi = i2
    wrapped onto the interior planes); the phi ghost planes are copies of
    the interior ones. Every stencil of a listed point reads Brill-Lindquist
    values, and the input costs seconds on the largest grid. Returns the
    state and the boxes (index arrays) it wrote."""
    ng, N2 = og.ng, og.N[2]
    y = og.state()
    y[orc.GF_NAMES.index("cf")] = 1.0
    y[orc.GF_NAMES.index("alpha")] = 1.0
    boxes = []
    for a, b, c in points:
        i0 = np.arange(max(a - 3, 0), min(a + 4, og.n[0]))
        i1 = np.arange(max(b - 3, 0), min(b + 4, og.n[1]))
        i2 = (np.arange(c - 3, c + 4) - ng) % N2 + ng
        r = np.array([og.xx(0, j) for j in i0]) * og.p.ampl[0]
        th = np.array([og.xx(1, j) for j in i1])
        ph = np.array([og.xx(2, j) for j in i2])
        R, TH, PH = np.meshgrid(r, th, ph, indexing="ij")
        x = np.stack([R * np.sin(TH) * np.cos(PH), R * np.sin(TH) * np.sin(PH), R * np.cos(TH)], -1)
        psi = np.ones(R.shape)
        for m, cen in zip(masses, pos):
            psi += m / (2.0 * np.linalg.norm(x - np.asarray(cen), axis=-1))
        box = np.ix_(i2, i1, i0)
        val = np.transpose(psi ** -2, (2, 1, 0))
        y[orc.GF_NAMES.index("cf")][box] = val
        y[orc.GF_NAMES.index("alpha")][box] = val
        boxes.append(box)
    y[:, :ng] = y[:, N2:N2 + ng]
    y[:, N2 + ng:] = y[:, ng:2 * ng]
    return y, boxes


def test_largest_grid_rhs_sampled_and_batch_step():
    """The largest grid the benchmark runs, the paper's 1008x168x336
    Spherical grid (r_max 7.5; 60.3M points with ghosts, close to the 2^26
    points that keep every stencil offset within 31 bits): the right-hand
    side at sampled points (the corners and faces of the index range, the
    last interior point, random ones) against the oracle, and one RK4 step
    of the ensemble path bitwise equal to the solo step. Near the origin
    and the axis of this grid the trK right-hand side is ill-conditioned in
    FP64 (second differences over cells of 1e-3 of the radius); there the
    bar is the FP64 oracle's own error against the extended-precision one."""
    _print_case("largest_grid")
    import torch
    from paper_2505_00097_amd import capi
    N, ampl = (1008, 168, 336), (7.5,) * 3
    masses, pos = [0.5, 0.5], [(0.0, 0.0, 0.5), (0.0, 0.0, -0.5)]
    g = capi.Grid(wl.SPHERICAL, N, ampl, (0.2,) * 3, 0.5)
    og = orc.Grid(wl.SPHERICAL, N, ampl=ampl, sinhw=(0.2,) * 3)
    rng = np.random.default_rng(7)
    ends = [(a, b, c) for a in (0, 1, N[0] - 1) for b in (0, N[1] // 2, N[1] - 1) for c in (0, N[2] - 1)]
    pick = [(3 + a, 3 + b, 3 + c) for a, b, c in ends]
    pick += [(3 + rng.integers(N[0]), 3 + rng.integers(N[1]), 3 + rng.integers(N[2])) for _ in range(100)]
    y, boxes = _bl_boxes(og, pick, masses, pos)
    print("  input ready", flush=True)
    idx = np.array([og.flat(*p) for p in pick])
    yg = to_gpu(y)
    r = g.state()
    capi.bssn_rhs(g.h, yg, r)
    got = r.view(24, -1)[:, torch.from_numpy(idx).to(r.device)].cpu().numpy()[:, None, None, :]
    del r
    ref = og.rhs_points(y, idx).T[:, None, None, :]
    # the extended-precision input: every value the sampled stencils read
    # (the 7^3 boxes), in an otherwise untouched zero array (pages that are
    # never written are never allocated)
    yl = np.zeros(y.shape, dtype=np.longdouble)
    for box in boxes:
        yl[(slice(None),) + box] = y[(slice(None),) + box]
    ng, N2 = og.ng, og.N[2]  # the phi ghost planes, which the oracle reads, as in the FP64 input
    yl[:, :ng] = yl[:, N2:N2 + ng]
    yl[:, N2 + ng:] = yl[:, ng:2 * ng]
    del y
    refl = og.twin().rhs_points(yl, idx).T[:, None, None, :]
    del yl
    assert np.max(np.abs(ref)) > 0.0
    check_parity("rhs largest grid sampled", got, ref, refl, (slice(None),) * 3, RHS_TOL, names=orc.GF_NAMES)
    # the ensemble kernels at this size: one step, bitwise equal to solo
    y1, y2 = yg, yg.clone()
    ws = g.workspace()
    capi.rk4_step(g.h, y1, ws, g.dt)
    b = capi.batch_create([g.h], eta=2.0)
    capi.batch_step(b, [y2], [ws], [g.dt], nsteps=1)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    assert bool(torch.isfinite(y1).all())
    capi.batch_destroy(b)


@pytest.mark.parametrize("name,m,pos,steps", [
    ("tiny", [1.0], [(0, 0, 0)], 100),
    ("cyl_3d", [0.7, 0.3], [(0.3, 0.1, 0.6), (-0.2, 0, -0.5)], 40),
])
def test_rk4_evolution_matches_oracle(name, m, pos, steps):
    _print_case("evolve", name, steps)
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    ol = og.twin()
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y)
    ws = g.workspace()
    yo = og.brill_lindquist(m, np.array(pos).reshape(-1, 3))
    yl = ld(yo)
    dt = og.dt()
    for _ in range(steps):
        capi.rk4_step(g.h, y, ws, dt, eta=2.0)
        og.rk4_step(yo, dt, eta=2.0)
        ol.rk4_step(yl, dt, eta=2.0)
    out = to_cpu(y)
    check_parity(f"rk4 {name} {steps} steps", out, yo, yl, og.interior(), EVOL_TOL, names=orc.GF_NAMES)
    # ghosts too
    check_parity(f"rk4 {name} {steps} steps, every point", out, yo, yl, (slice(None),) * 3, EVOL_TOL,
                 names=orc.GF_NAMES)


@pytest.mark.parametrize("name,m,pos,steps", [
    ("tiny", [1.0], [(0, 0, 0)], 100),
    ("cyl_ragged", [0.5, 0.5], [(0, 0, 0.5), (0, 0, -0.5)], 60),
    ("cyl_3d", [0.7, 0.3], [(0.3, 0.1, 0.6), (-0.2, 0, -0.5)], 40),
])
def test_ssprk3_evolution_matches_oracle(name, m, pos, steps):
    """The SSPRK3 integrator (three stages, two of them mixing y_n with a
    stage state in the kernel epilogue) against the oracle's."""
    _print_case("evolve_ssprk3", name, steps)
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    ol = og.twin()
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, m, pos, y)
    ws = g.workspace()
    yo = og.brill_lindquist(m, np.array(pos).reshape(-1, 3))
    yl = ld(yo)
    dt = og.dt()
    for _ in range(steps):
        capi.ssprk3_step(g.h, y, ws, dt, eta=2.0)
        og.ssprk3_step(yo, dt, eta=2.0)
        ol.ssprk3_step(yl, dt, eta=2.0)
    out = to_cpu(y)
    check_parity(f"ssprk3 {name} {steps} steps", out, yo, yl, og.interior(), EVOL_TOL, names=orc.GF_NAMES)
    check_parity(f"ssprk3 {name} {steps} steps, every point", out, yo, yl, (slice(None),) * 3, EVOL_TOL,
                 names=orc.GF_NAMES)


def test_headon_workload_100_steps_matches_oracle():
    """The head-on workload at full size (SinhCylindrical 128x2x256, two
    punctures), 100 RK4 steps with the tuned tile shape the benchmark uses
    and H at the end, against the oracle."""
    name = "headon_sinhcylindrical_128x2x256"
    _print_case("evolve_full", name, 100)
    from paper_2505_00097_amd import capi
    w = wl.WORKLOADS[name]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"])
    og = orc.Grid(w["coord"], w["N"], ampl=w["ampl"], sinhw=w["sinhw"], cfl=w["cfl"])
    ol = og.twin()
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y)
    capi.grid_tune(g.h, y, g.state())
    ws = g.workspace()
    yo = og.brill_lindquist(w["masses"], w["positions"])
    dt = og.dt()
    assert g.dt == pytest.approx(dt, rel=1e-14)
    for s in range(100):
        capi.rk4_step(g.h, y, ws, dt, eta=w["eta"])
        og.rk4_step(yo, dt, eta=w["eta"])
        if s % 10 == 9:
            print("  step", s + 1, flush=True)
    out = to_cpu(y)
    check_parity("rk4 headon full size 100 steps", out, yo, None, og.interior(), EVOL_TOL, names=orc.GF_NAMES)
    # H on the evolved full-size state (same input on both sides)
    Hg = g._empty(1)
    capi.hamiltonian_constraint(g.h, y, Hg)
    I = og.interior()
    check_parity("H headon after 100 steps", to_cpu(Hg), og.constraints(out)[0][None],
                 ol.constraints(ld(out))[0][None], I, RHS_TOL, groups=[[0]])


@pytest.mark.parametrize("name", ["tiny", "cyl_3d", "sph_ragged"])
def test_hamiltonian_matches_oracle(name):
    _print_case("ham", name)
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    ol = og.twin()
    I = og.interior()
    for label, y in (("bl", og.brill_lindquist([0.8], [(0.1, 0.0, 0.2)])),
                     ("smooth_random", og.apply_bcs(wl.smooth_random_state(og.n, seed=4)))):
        Hg = g._empty(1)
        capi.hamiltonian_constraint(g.h, to_gpu(y), Hg)
        check_parity(f"H {name} {label}", to_cpu(Hg), og.constraints(y)[0][None], ol.constraints(ld(y))[0][None],
                     I, RHS_TOL, groups=[[0]])


def test_batch_matches_solo():
    _print_case("batch")
    import torch
    from paper_2505_00097_amd import capi
    jobs = wl.batched_jobs(n=3, seed=7)
    for j in jobs:
        j["N"] = (j["N"][0] // 4, 2, j["N"][2] // 4)
    grids = [capi.Grid(j["coord"], j["N"], j["ampl"], j["sinhw"], j["cfl"]) for j in jobs]
    ys, wss, solo = [], [], []
    for j, g in zip(jobs, grids):
        y = g.state()
        capi.set_initial_data_brill_lindquist(g.h, j["masses"], j["positions"], y)
        ys.append(y)
        solo.append(y.clone())
        wss.append(g.workspace())
    b = capi.batch_create([g.h for g in grids], eta=2.0)
    capi.batch_step(b, ys, wss, [g.dt for g in grids], nsteps=5)
    for g, y in zip(grids, solo):
        ws = g.workspace()
        for _ in range(5):
            capi.rk4_step(g.h, y, ws, g.dt)
    torch.cuda.synchronize()
    for y, s in zip(ys, solo):
        assert torch.equal(y, s)
    capi.batch_destroy(b)


@pytest.mark.parametrize("name", list(GRIDS))
def test_stage_ghost_fill_equals_full_fill(name):
    """An RK4 step fills copy ghosts inside the stage kernel and the rest in a
    separate pass; re-applying the full boundary fill afterwards must change
    nothing, bit for bit."""
    _print_case("stage ghosts", name)
    import torch
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    y = to_gpu(wl.smooth_random_state(og.n, seed=5))
    capi.apply_bcs(g.h, y)
    ws = g.workspace()
    for _ in range(2):
        capi.rk4_step(g.h, y, ws, g.dt)
    z = y.clone()
    capi.apply_bcs(g.h, z)
    torch.cuda.synchronize()
    assert torch.equal(y, z)


@pytest.mark.parametrize("name", list(GRIDS))
def test_phi_ghost_planes_are_never_read(name):
    """Stencils read phi with the index wrapped onto the interior planes:
    poisoning every phi ghost plane with NaN changes neither the right-hand
    side nor H, bit for bit."""
    _print_case("phi ghosts unread", name)
    import torch
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    y = to_gpu(wl.smooth_random_state(og.n, seed=9))
    capi.apply_bcs(g.h, y)
    z = y.clone()
    N = g.N
    if g.coord == wl.SINH_CYLINDRICAL:
        z[:, :, :3, :] = float("nan")
        z[:, :, 3 + N[1]:, :] = float("nan")
    else:
        z[:, :3, :, :] = float("nan")
        z[:, 3 + N[2]:, :, :] = float("nan")
    r1, r2 = g.state(), g.state()
    r1.zero_()
    r2.zero_()
    capi.bssn_rhs(g.h, y, r1)
    capi.bssn_rhs(g.h, z, r2)
    H1, H2 = g._empty(1).zero_(), g._empty(1).zero_()
    capi.hamiltonian_constraint(g.h, y, H1)
    capi.hamiltonian_constraint(g.h, z, H2)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
    assert torch.equal(H1, H2)


@pytest.mark.parametrize("name", ["sph_ragged", "cyl_ragged", "spherical"])
def test_tile_shape_does_not_change_results(name):
    """Every allowed tile shape of the solo kernel gives the same RK4 step,
    bit for bit, with one wave per tile and again with two (where a two-wave
    kernel is built; elsewhere the one-wave kernel runs); one and two waves
    agree to rounding; bhah_grid_tune picks one shape and mode, and the step
    then equals that mode's, bit for bit; shapes that cross phi are
    rejected."""
    _print_case("solo tiles", name)
    import torch
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    y0 = to_gpu(og.apply_bcs(wl.smooth_random_state(og.n, seed=21)))
    ws = g.workspace()
    shapes = [(6, 0, 4), (5, 0, 1), (4, 0, 4), (3, 0, 1)] if g.coord == wl.SINH_CYLINDRICAL else \
        [(6, 0, 4), (5, 1, 1), (4, 2, 4), (3, 3, 1)]
    refs = {}
    for waves in (1, 2):
        capi.grid_set_waves_per_tile(g.h, waves)
        ref = None
        for shp in shapes:
            capi.grid_set_tile(g.h, *shp)
            assert capi.grid_get_tile(g.h) == shp and capi.grid_get_waves_per_tile(g.h) == waves
            y = y0.clone()
            capi.rk4_step(g.h, y, ws, g.dt)
            torch.cuda.synchronize()
            if ref is None:
                ref = y
            else:
                assert torch.equal(y, ref), (waves, shp)
        refs[waves] = ref
    a, b = to_cpu(refs[1]), to_cpu(refs[2])
    check_parity(f"one vs two waves per tile, rk4 step {name}", b, a, None, (slice(None),) * 3, 1e-13,
                 names=orc.GF_NAMES)
    bad = (5, 1, 1) if g.coord == wl.SINH_CYLINDRICAL else (4, 0, 4)
    with pytest.raises(capi.BhahError):
        capi.grid_set_tile(g.h, *bad)
    capi.grid_set_waves_per_tile(g.h, 1)
    capi.grid_tune(g.h, y0, g.state())
    lx, ly, band = capi.grid_get_tile(g.h)
    assert 3 <= lx <= 6 and lx + ly <= 6 and band >= 1
    waves = capi.grid_get_waves_per_tile(g.h)
    print(f"  tuned: tile {(lx, ly, band)}, {waves} wave(s) per tile", flush=True)
    y = y0.clone()
    capi.rk4_step(g.h, y, ws, g.dt)
    torch.cuda.synchronize()
    assert torch.equal(y, refs[waves])


@pytest.mark.parametrize("coord,N", [(wl.SINH_SPHERICAL, (3, 3, 2)), (wl.SINH_CYLINDRICAL, (3, 2, 3)),
                                     (wl.SPHERICAL, (3, 3, 2))])
def test_smallest_grids(coord, N):
    """Grids one stencil radius wide: every interior point's stencils reach
    the outermost ghost layers on both sides; RHS and 10 RK4 steps against
    the oracle."""
    _print_case("smallest", coord, N)
    from paper_2505_00097_amd import capi
    ampl = (2.0, 2.0, 3.0)
    g = capi.Grid(coord, N, ampl, (0.3,) * 3)
    og = orc.Grid(coord, N, ampl=ampl, sinhw=(0.3,) * 3)
    ol = og.twin()
    y = og.apply_bcs(og.brill_lindquist([0.4], [(0.1, 0.0, 0.2)]) + 0.01 * wl.smooth_random_state(og.n, seed=2))
    out, _ = _rhs_gpu(g, y)
    I = og.interior()
    check_parity(f"rhs smallest {coord} {N}", out, og.rhs(y, eta=2.0), ol.rhs(ld(y), eta=2.0), I, RHS_TOL,
                 names=orc.GF_NAMES)
    yg = to_gpu(y)
    yl = ld(y)
    ws = g.workspace()
    dt = og.dt()
    for _ in range(10):
        capi.rk4_step(g.h, yg, ws, dt)
        og.rk4_step(y, dt, eta=2.0)
        ol.rk4_step(yl, dt, eta=2.0)
    check_parity(f"rk4 smallest {coord} {N} 10 steps", to_cpu(yg), y, yl, I, EVOL_TOL, names=orc.GF_NAMES)


def test_invalid_calls_report_errors():
    _print_case("errors")
    from paper_2505_00097_amd import capi
    g = capi.Grid(wl.SINH_SPHERICAL, (8, 8, 2))
    y = g.state()
    with pytest.raises(capi.BhahError, match="n_punct"):
        capi.set_initial_data_brill_lindquist(g.h, [0.1] * 17, [(0.0, 0.0, 0.0)] * 17, y)
    with pytest.raises(capi.BhahError, match="lapse_kind"):
        capi.set_initial_data_brill_lindquist(g.h, [1.0], [(0.0, 0.0, 0.0)], y, lapse_kind=3)
    with pytest.raises(capi.BhahError, match="shift_variant"):
        gp = capi.GaugeParams(2.0, 1)
        capi._check(capi.lib().bhah_bssn_rhs(g.h, capi.ctypes.byref(gp), capi._ptr(y), capi._ptr(g.state()),
                                             None, capi._stream(None)), "bhah_bssn_rhs")
    for bad in ((-0.1, 0.3), (0.99, float("nan")), (float("inf"), 0.0)):
        with pytest.raises(capi.BhahError, match="dissipation"):
            capi.ssprk3_step(g.h, y, g.workspace(), g.dt, diss=bad)
    # a state pointer that is not aligned to a double is rejected before any launch
    gp = capi.gauge(2.0)
    mis = capi.ctypes.c_void_p(y.data_ptr() + 4)
    rc = capi.lib().bhah_rk4_step(g.h, capi.ctypes.byref(gp), g.dt, mis, capi._ptr(g.workspace()),
                                  capi._stream(None))
    assert rc == capi.EINVAL and "aligned" in capi.last_error()


@pytest.mark.parametrize("name", ["tiny", "cyl_3d", "sph_ragged", "spherical"])
def test_constraints_match_oracle(name):
    """H (Eq. 16), M^i (Eq. 17) and C^i from bhah_constraints against the
    oracle: exactly zero momentum and C^i on Brill-Lindquist data, and within
    the per-RHS bar on evolved and smooth random states (each constraint
    measured against its own largest magnitude)."""
    _print_case("constraints", name)
    import torch
    from paper_2505_00097_amd import capi
    g, og = _pair(name)
    ol = og.twin()
    I = og.interior()
    bl = og.brill_lindquist([0.8], [(0.1, 0.0, 0.2)])
    ev = bl.copy()
    for _ in range(10):
        og.rk4_step(ev, og.dt(), eta=2.0)
    rnd = og.apply_bcs(wl.smooth_random_state(og.n, seed=8))

    def cons(o, v):
        H, M, C = o.constraints(v)
        return np.concatenate([H[None], M, C])

    groups = [[0], [1, 2, 3], [4, 5, 6]]
    for label, y in (("bl", bl), ("evolved", ev), ("random", rnd)):
        H, M, C = g._empty(1), g._empty(3), g._empty(3)
        for t in (H, M, C):
            t.zero_()
        capi.constraints(g.h, to_gpu(y), H, M, C)
        torch.cuda.synchronize()
        got = np.concatenate([to_cpu(H), to_cpu(M), to_cpu(C)])
        if label == "bl":
            assert np.all(got[1:][(slice(None),) + I] == 0.0)
        check_parity(f"constraints {name} {label}", got, cons(og, y), cons(ol, ld(y)), I, RHS_TOL, groups=groups)
    # bhah_hamiltonian_constraint gives the same H up to rounding (another
    # kernel instance: the compiler may contract differently)
    y = to_gpu(ev)
    H1, H2 = g._empty(1), g._empty(1)
    capi.hamiltonian_constraint(g.h, y, H1)
    capi.constraints(g.h, y, H2, None, None)
    a, b = to_cpu(H1)[0][I], to_cpu(H2)[0][I]
    assert np.max(np.abs(a - b)) <= RHS_TOL * np.max(np.abs(a))


def test_probe_peaks_are_plausible():
    """The measured ceilings fall between a sanity floor and the published
    MI355X figures (FP64 vector 78.6 TFLOP/s, HBM 8 TB/s), within 5 %."""
    from paper_2505_00097_amd import capi
    tf, gbps = capi.probe_peaks()
    print(f"probe: fp64 {tf:.1f} TFLOP/s, triad {gbps:.0f} GB/s")
    assert 5.0 < tf < 78.6 * 1.05
    assert 500.0 < gbps < 8000.0 * 1.05


@pytest.mark.parametrize("name,integrator,radiation", [("cyl_ragged", "rk4", False), ("sph_ragged", "rk4", False),
                                                       ("cyl_ragged", "ssprk3", True), ("spherical", "ssprk3", False)])
def test_evolve_equals_single_steps(name, integrator, radiation):
    """bhah_evolve (n steps in one call, phi ghost planes filled only after
    the last) equals n calls of the single-step entry point bit for bit,
    ghosts included; nsteps = 0 changes nothing and nsteps < 0 is refused."""
    _print_case("evolve_n", name, integrator, radiation)
    import torch
    from paper_2505_00097_amd import capi
    coord, N, ampl, w = GRIDS[name]
    g = capi.Grid(coord, N, ampl, w, bc_kind=capi.BC_RADIATION if radiation else capi.BC_EXTRAP)
    diss = DISS if integrator == "ssprk3" else (0.0, 0.0)
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, [0.6, 0.4], [(0.2, 0.0, 0.5), (0.0, 0.1, -0.5)], y)
    y1, y2 = y.clone(), y.clone()
    ws = g.workspace()
    step = capi.ssprk3_step if integrator == "ssprk3" else capi.rk4_step
    for _ in range(7):
        step(g.h, y1, ws, g.dt, diss=diss)
    capi.evolve(g.h, y2, ws, g.dt, 7, integrator=capi.SSPRK3 if integrator == "ssprk3" else capi.RK4, diss=diss)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    y3 = y2.clone()
    capi.evolve(g.h, y3, ws, g.dt, 0)
    torch.cuda.synchronize()
    assert torch.equal(y3, y2)
    with pytest.raises(capi.BhahError, match="nsteps"):
        capi.evolve(g.h, y3, ws, g.dt, -1)
    with pytest.raises(capi.BhahError, match="integrator"):
        capi.evolve(g.h, y3, ws, g.dt, 1, integrator=7)
