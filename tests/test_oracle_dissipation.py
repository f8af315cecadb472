"""Pins of the oracle's Kreiss-Oliger dissipation (Sec. 4.1: strengths for the
gauge and the metric variables, operator one order above the differencing).

The dissipation is additive, so the right-hand side with it minus the one
without it is the dissipation term alone, whatever the rest of the equations
do with the data. Its value is fixed in closed form on
  - Fourier modes along one logical direction: the sixth difference of
    cos(theta j) is exactly -64 sin^6(theta/2) cos(theta j);
  - polynomials in the grid index: the sixth difference annihilates degree
    5 and takes j^6 to 6! = 720.
"""
import numpy as np
import pytest

import analytic as an
from oracle import oracle as orc

GRID = (an.SINH_SPHERICAL, (8, 6, 4), (3.0,) * 3, (0.3,) * 3)
GAUGE = {"alpha", "betU0", "betU1", "betU2", "vetU0", "vetU1", "vetU2"}


def _grids(diss):
    coord, N, ampl, w = GRID
    return orc.Grid(coord, N, ampl=ampl, sinhw=w), orc.Grid(coord, N, ampl=ampl, sinhw=w, diss=diss)


def _flat(g):
    y = g.state()
    y[an.GF["cf"]] = 1.0
    y[an.GF["alpha"]] = 1.0
    return y


def _index(g, d):
    """grid index j along direction d at every point (ghosts included)"""
    shape = (g.n[2], g.n[1], g.n[0])
    j = np.arange(g.n[d], dtype=np.float64)
    return np.broadcast_to(j.reshape([-1 if a == 2 - d else 1 for a in range(3)]), shape)


def _dxx(g, d):
    return g.xx(d, g.ng + 1) - g.xx(d, g.ng)


@pytest.mark.parametrize("name", ["alpha", "hDD01", "vetU2", "trK", "lambdaU1", "betU0", "aDD22", "cf"])
@pytest.mark.parametrize("d", [0, 2])
def test_dissipation_of_a_fourier_mode(name, d):
    eps_g, eps_m = 0.99, 0.3
    g0, g1 = _grids((eps_g, eps_m))
    theta, amp = 1.9, 1e-3
    y = _flat(g0)
    mode = amp * np.cos(theta * _index(g0, d) + 0.4)
    y[an.GF[name]] += mode
    diff = g1.rhs(y) - g0.rhs(y)
    I = g0.interior()
    eps = eps_g if name in GAUGE else eps_m
    expect = -eps * np.sin(theta / 2) ** 6 * mode / _dxx(g0, d)
    gi = an.GF[name]
    scale = np.max(np.abs(expect[I]))
    assert np.max(np.abs(diff[gi][I] - expect[I])) <= 1e-10 * scale
    # every other right-hand side is untouched (their fields are constant)
    others = [k for k in range(an.NGF) if k != gi]
    assert np.max(np.abs(diff[others][(slice(None),) + I])) <= 1e-13


def test_dissipation_annihilates_quintics_and_counts_the_sixth_power():
    eps_g, eps_m = 0.7, 0.2
    g0, g1 = _grids((eps_g, eps_m))
    j0, j1, j2 = (_index(g0, d) for d in range(3))
    y = _flat(g0)
    # degree <= 5 in the indices, mixed terms included
    quint = 1e-6 * (j0 ** 5 - 3.0 * j1 ** 4 * j2 + 2.0 * j0 ** 2 * j1 ** 2 * j2 + j2 ** 5 - 7.0 * j0 * j2 ** 3)
    y[an.GF["hDD11"]] += quint
    y[an.GF["betU1"]] += quint
    # a sixth power along i1 only: its sixth difference is 720 everywhere
    y[an.GF["trK"]] += 1e-7 * j1 ** 6
    diff = g1.rhs(y) - g0.rhs(y)
    I = g0.interior()
    for n in ("hDD11", "betU1"):
        assert np.max(np.abs(diff[an.GF[n]][I])) <= 1e-14 * np.max(np.abs(quint)), n  # rounding only
    expect = eps_m * 1e-7 * 720.0 / (64.0 * _dxx(g0, 1))
    assert diff[an.GF["trK"]][I] == pytest.approx(np.full(diff[an.GF["trK"]][I].shape, expect), rel=1e-8)
