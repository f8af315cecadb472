"""Pins of the oracle's Sommerfeld radiation outer boundary (Sec. 3 names the
condition; its form is a reading: every rescaled gridfunction an outgoing
spherical wave about its asymptotic value, d_t f = -v (f - f_inf)/r - v df/dr
at the pure-outer ghost points, f_inf = 1 for alpha and W, v = sqrt(2) for
alpha).

Fixed in closed form, independently of the oracle's stencils and Jacobians:
  - the asymptotic state gives exactly zero;
  - f = f_inf + u(t - r/v)/r solves the condition for every profile u, so
    the discrete right-hand side at the outer points converges to
    u'(-r/v)/r at the order of the differencing (4th);
  - f = f_inf + c/r is stationary: the right-hand side converges to zero.
The data need not solve the BSSN equations: only the outer points, whose
right-hand side is the condition alone, are examined.
"""
import numpy as np
import pytest

import analytic as an
from oracle import oracle as orc

FINF = {"alpha": 1.0, "cf": 1.0}
SPEED = {"alpha": np.sqrt(2.0)}

CASES = [
    (an.SINH_SPHERICAL, (16, 6, 4), (6.0,) * 3, (0.8,) * 3),
    (an.SINH_CYLINDRICAL, (16, 2, 32), (6.0,) * 3, (0.8,) * 3),
    (an.SPHERICAL, (16, 6, 4), (6.0,) * 3, (0.2,) * 3),
]


def _refined(N, coord, f):
    """N with the directions the outer boundary is crossed along refined by f"""
    if coord == an.SINH_CYLINDRICAL:
        return (N[0] * f, N[1], N[2] * f)
    return (N[0] * f, N[1], N[2])


def _outer_rhs(coord, N, ampl, w, field):
    """(rhs, expected, mask of pure-outer points) for gridfunction values
    field(name, r) -> (f, expected d_t f)"""
    g = orc.Grid(coord, N, ampl=ampl, sinhw=w, bc_kind=1)
    _, x, _ = an.mesh(coord, N, ampl, w)
    r = np.linalg.norm(x, axis=-1)
    y = g.state()
    expect = g.state()
    for n in an.GF_NAMES:
        y[an.GF[n]], expect[an.GF[n]] = field(n, r)
    rc, kind, _, _ = g.bc_maps()
    assert rc == 0
    outer = (kind == 1).reshape(g.n[2], g.n[1], g.n[0])
    return g.rhs(y), expect, outer


def test_asymptotic_state_gives_zero():
    for coord, N, ampl, w in CASES:
        rhs, _, outer = _outer_rhs(coord, N, ampl, w, lambda n, r: (np.full_like(r, FINF.get(n, 0.0)), 0 * r))
        assert np.max(np.abs(rhs[:, outer])) <= 1e-13, coord


@pytest.mark.parametrize("case", range(len(CASES)))
def test_outgoing_wave_converges_at_fourth_order(case):
    coord, N, ampl, w = CASES[case]
    s0, sig = -5.5, 2.5

    def field(n, r):
        v = SPEED.get(n, 1.0)
        amp = 1e-2 * (1 + an.GF[n] % 5)  # a different amplitude per gridfunction
        s = -r / v
        u = amp * np.exp(-((s - s0) / sig) ** 2)
        du = -2.0 * (s - s0) / sig ** 2 * u
        return FINF.get(n, 0.0) + u / r, du / r
    errs = []
    for f in (1, 2):
        rhs, ex, outer = _outer_rhs(coord, _refined(N, coord, f), ampl, w, field)
        errs.append(max(np.max(np.abs(rhs[k][outer] - ex[k][outer])) / np.max(np.abs(ex[k][outer]))
                        for k in range(an.NGF)))
    assert errs[1] < 2e-3, errs
    assert errs[0] / errs[1] > 11.0, errs


@pytest.mark.parametrize("case", range(len(CASES)))
def test_static_one_over_r_converges_to_zero(case):
    coord, N, ampl, w = CASES[case]
    errs = []
    for f in (1, 2):
        rhs, _, outer = _outer_rhs(coord, _refined(N, coord, f), ampl, w,
                                   lambda n, r: (FINF.get(n, 0.0) + 0.3 / r, 0 * r))
        errs.append(np.max(np.abs(rhs[:, outer])))
    # scale: each term of the condition is ~ 0.3 / r^2
    assert errs[1] < 1e-2 * 0.3 / ampl[0] ** 2, errs
    assert errs[0] / errs[1] > 12.0, errs


def test_rk4_step_copies_inner_ghosts_and_evolves_outer_points():
    """With the radiation boundary the time integrator advances the outer
    points and refills only the inner ghosts, as parity copies."""
    coord, N, ampl, w = CASES[1]
    g = orc.Grid(coord, N, ampl=ampl, sinhw=w, bc_kind=1)
    ge = orc.Grid(coord, N, ampl=ampl, sinhw=w)
    y0 = ge.brill_lindquist([0.5, 0.5], [(0, 0, 0.8), (0, 0, -0.8)])
    a, b = y0.copy(), y0.copy()
    g.rk4_step(a, g.dt(), eta=2.0)
    ge.rk4_step(b, ge.dt(), eta=2.0)
    rc, kind, src, par = g.bc_maps()
    k = kind.reshape(g.n[2], g.n[1], g.n[0])
    # the outer points now differ from the extrapolated ones
    assert np.max(np.abs(a[:, k == 1] - b[:, k == 1])) > 1e-8
    # inner ghosts: exact copies of their sources, up to the parity sign
    flat = a.reshape(an.NGF, -1)
    inner = np.flatnonzero(kind == 2)
    assert np.all(np.abs(flat[:, inner]) == np.abs(flat[:, src[inner]]))


@pytest.mark.parametrize("stepper,order", [("rk4_step", 4), ("ssprk3_step", 3)])
def test_outer_points_converge_in_time_at_the_integrators_order(stepper, order):
    """The outer points are part of the semi-discrete system, so every stage
    must advance them: the time error at the outer points falls by 2^order
    when dt halves (an integrator that left them behind in some stage would
    be inconsistent there)."""
    coord, N, ampl, w = an.SINH_CYLINDRICAL, (10, 2, 20), (4.0,) * 3, (0.5,) * 3
    g = orc.Grid(coord, N, ampl=ampl, sinhw=w, bc_kind=1)
    y0 = orc.Grid(coord, N, ampl=ampl, sinhw=w).brill_lindquist([0.5, 0.5], [(0, 0, 1.5), (0, 0, -1.5)])
    T = 4 * g.dt()
    rc, kind, _, _ = g.bc_maps()
    outer = (kind == 1).reshape(g.n[2], g.n[1], g.n[0])

    def run(n):
        y = y0.copy()
        for _ in range(n):
            getattr(g, stepper)(y, T / n, eta=2.0)
        return y
    ref = run(64)
    errs = [np.max(np.abs(run(n)[:, outer] - ref[:, outer])) for n in (4, 8)]
    assert errs[0] / errs[1] > 0.7 * 2 ** order, errs
