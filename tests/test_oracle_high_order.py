"""Pins of the oracle's finite differences of higher order (Sec. 3: the
differencing order N_FD is selectable and needs N_G = N_FD/2 + 1 ghost
layers for the upwinded advection stencils; the production head-on run of
Sec. 4.1 uses N_FD = 8 with ninth-order Kreiss-Oliger dissipation and an
eighth-order radiation condition).

Fixed independently of the oracle's Lagrange-polynomial construction:
  - the centred weights equal the classical closed forms
    d1_j = (-1)^(j+1) (R!)^2 / (j (R-j)! (R+j)!) and d2_j = 2 d1_j / j
    (R = N_FD/2), read off from the response to a unit impulse;
  - every operator is exact on polynomials up to its degree and not one
    degree higher;
  - the dissipation of order 2 N_G - 1 has the Fourier symbol
    -sin^(2 N_G)(theta/2)/h, annihilates polynomials of degree 2 N_G - 1
    and takes j^(2 N_G) to (2 N_G)! / 4^N_G / h;
  - the radiation condition converges at the eighth order on exact
    outgoing waves;
  - the ghost maps with five layers equal the closed-form reflections.
"""
from math import factorial

import numpy as np
import pytest

import analytic as an
from oracle import oracle as orc
from test_oracle_bcs import closed_form_maps
from test_oracle_dissipation import GAUGE, _flat, _index
from test_oracle_fd_geometry import _poly_field
from test_oracle_radiation import FINF, SPEED, _refined


def _grid(ng, coord=an.SINH_CYLINDRICAL, N=(12, 6, 14)):
    return orc.Grid(coord, N, ampl=(3.0,) * 3, sinhw=(0.3,) * 3, ng=ng)


def _h(g, d):
    return g.xx(d, g.ng + 1) - g.xx(d, g.ng)


def _centre(g):
    return tuple(g.ng + n // 2 for n in g.N)


@pytest.mark.parametrize("ng", [3, 4, 5, 6])
def test_centred_weights_equal_closed_forms(ng):
    R = ng - 1
    g = _grid(ng)
    c = _centre(g)
    q = g.flat(*c)
    for k in (0, 2):
        h = _h(g, k)
        d2c = 0.0
        for j in range(1, R + 1):
            f = np.zeros((g.n[2], g.n[1], g.n[0]))
            idx = list(c)
            idx[k] += j
            f[idx[2], idx[1], idx[0]] = 1.0
            d1, d2, _, _ = g.fd_point(f, q)
            w1 = (-1) ** (j + 1) * factorial(R) ** 2 / (j * factorial(R - j) * factorial(R + j))
            assert abs(d1[k] * h - w1) <= 1e-14 * abs(w1), (ng, k, j)
            assert abs(d2[k, k] * h * h - 2.0 * w1 / j) <= 1e-14 * abs(w1), (ng, k, j)
            d2c -= 2.0 * (2.0 * w1 / j)
        # the centre weight of D2 is minus the sum of the others
        f = np.zeros((g.n[2], g.n[1], g.n[0]))
        f[c[2], c[1], c[0]] = 1.0
        _, d2, _, _ = g.fd_point(f, q)
        assert abs(d2[k, k] * h * h - d2c) <= 1e-13 * abs(d2c)
    if ng == 5:  # the eighth-order values themselves
        assert np.allclose([(-1) ** (j + 1) * factorial(4) ** 2 / (j * factorial(4 - j) * factorial(4 + j))
                            for j in range(1, 5)], [4 / 5, -1 / 5, 4 / 105, -1 / 280], rtol=1e-15, atol=0)


@pytest.mark.parametrize("ng", [4, 5])
def test_fd_exact_on_polynomials_up_to_the_order(ng):
    """N_FD = 2 (ng - 1): D, U+-, and the mixed D_k D_l are exact on degree
    N_FD; D2 on degree N_FD + 1 (a symmetric stencil); none one degree
    higher."""
    order = 2 * (ng - 1)
    g = _grid(ng, an.SINH_SPHERICAL, (12, 10, 14))
    rng = np.random.default_rng(11)
    c = _centre(g)
    q = g.flat(*c)
    pt = [g.xx(0, c[0]), g.xx(1, c[1]), g.xx(2, c[2])]
    f, ex = _poly_field(g, (order,) * 3, rng)
    d1, d2, up, dn = g.fd_point(f, q)
    scale = np.max(np.abs(f))
    for k in range(3):
        o = [0, 0, 0]; o[k] = 1
        for v in (d1[k], up[k], dn[k]):
            assert abs(v - ex(pt, o)) < 1e-8 * scale, (k, v, ex(pt, o))
        for l in range(3):
            if l != k:
                o2 = [0, 0, 0]; o2[k] += 1; o2[l] += 1
                assert abs(d2[k, l] - ex(pt, o2)) < 1e-7 * scale
    for k in range(3):
        degs = [0, 0, 0]; degs[k] = order + 1
        f, ex = _poly_field(g, degs, rng)
        d1, d2, up, dn = g.fd_point(f, q)
        s = np.max(np.abs(f))
        o = [0, 0, 0]; o[k] = 2
        assert abs(d2[k, k] - ex(pt, o)) < 1e-7 * s
        o = [0, 0, 0]; o[k] = 1
        for v in (d1[k], up[k], dn[k]):
            assert abs(v - ex(pt, o)) > 1e-11 * s
        degs[k] = order + 2
        f, ex = _poly_field(g, degs, rng)
        _, d2, _, _ = g.fd_point(f, q)
        o = [0, 0, 0]; o[k] = 2
        assert abs(d2[k, k] - ex(pt, o)) > 1e-11 * np.max(np.abs(f))


def test_upwind_stencils_are_shifted_one_point():
    """U+ at N_FD = 8 reads offsets -3..5 only, U- offsets -5..3: an impulse
    at -4 (or +4) leaves it unchanged, one at +5 (or -5) does not."""
    g = _grid(5)
    c = _centre(g)
    q = g.flat(*c)
    for off, changes_up, changes_dn in ((-4, False, True), (4, True, False), (5, True, False),
                                        (-5, False, True), (-3, True, True), (3, True, True)):
        f = np.zeros((g.n[2], g.n[1], g.n[0]))
        f[c[2], c[1], c[0] + off] = 1.0
        _, _, up, dn = g.fd_point(f, q)
        assert (up[0] != 0.0) == changes_up, off
        assert (dn[0] != 0.0) == changes_dn, off


@pytest.mark.parametrize("ng", [3, 5])
@pytest.mark.parametrize("theta", [np.pi, 1.9, 0.7])
def test_dissipation_symbol(ng, theta):
    g = _grid(ng)
    c = _centre(g)
    q = g.flat(*c)
    for d in (0, 2):
        f = np.cos(theta * _index(g, d) + 0.4)
        ko = g.ko_point(f, q)
        expect = -np.sin(theta / 2) ** (2 * ng) * f.ravel()[q] / _h(g, d)
        assert abs(ko[d] - expect) <= 1e-12 / _h(g, d), (d, ko[d], expect)


@pytest.mark.parametrize("ng", [3, 5])
def test_dissipation_annihilates_lower_degrees_and_counts_the_top_power(ng):
    p = ng
    g = _grid(ng)
    c = _centre(g)
    q = g.flat(*c)
    for d in (0, 2):
        j = _index(g, d) - c[d]
        rng = np.random.default_rng(d)
        f = np.polynomial.Polynomial(rng.uniform(-1, 1, 2 * p))(j)  # degree 2p - 1
        assert abs(g.ko_point(f, q)[d]) <= 1e-9 / _h(g, d)
        top = g.ko_point(j ** (2 * p), q)[d]
        expect = factorial(2 * p) / 4.0 ** p / _h(g, d)
        assert abs(top - expect) <= 1e-9 * expect


@pytest.mark.parametrize("name", ["alpha", "hDD01", "vetU2", "betU0", "lambdaU1", "cf"])
def test_eighth_order_dissipation_in_the_rhs(name):
    """the ninth-order operator enters each right-hand side with the gauge or
    the metric strength"""
    eps_g, eps_m = 0.99, 0.3
    coord, N = an.SINH_SPHERICAL, (12, 8, 6)
    g0 = orc.Grid(coord, N, ampl=(3.0,) * 3, sinhw=(0.3,) * 3, ng=5)
    g1 = orc.Grid(coord, N, ampl=(3.0,) * 3, sinhw=(0.3,) * 3, ng=5, diss=(eps_g, eps_m))
    theta, amp, d = 2.3, 1e-3, 0
    y = _flat(g0)
    mode = amp * np.cos(theta * _index(g0, d) + 0.4)
    y[an.GF[name]] += mode
    diff = g1.rhs(y) - g0.rhs(y)
    I = g0.interior()
    eps = eps_g if name in GAUGE else eps_m
    expect = -eps * np.sin(theta / 2) ** 10 * mode / _h(g0, d)
    gi = an.GF[name]
    assert np.max(np.abs(diff[gi][I] - expect[I])) <= 1e-10 * np.max(np.abs(expect[I]))


def _outer_rhs(coord, N, ampl, w, field, ng):
    g = orc.Grid(coord, N, ampl=ampl, sinhw=w, bc_kind=1, ng=ng)
    _, x, _ = an.mesh(coord, N, ampl, w, ng=ng)
    r = np.linalg.norm(x, axis=-1)
    y = g.state()
    expect = g.state()
    for n in an.GF_NAMES:
        y[an.GF[n]], expect[an.GF[n]] = field(n, r)
    rc, kind, _, _ = g.bc_maps()
    assert rc == 0
    outer = (kind == 1).reshape(g.n[2], g.n[1], g.n[0])
    return g.rhs(y), expect, outer


@pytest.mark.parametrize("coord,N,ampl,w", [(an.SINH_SPHERICAL, (16, 6, 4), (6.0,) * 3, (0.8,) * 3),
                                            (an.SINH_CYLINDRICAL, (16, 2, 32), (6.0,) * 3, (0.8,) * 3)])
def test_radiation_converges_at_eighth_order(coord, N, ampl, w):
    """f = f_inf + u(t - r/v)/r: the outer right-hand side converges to
    u'(-r/v)/r with the 9-point stencils of N_G = 5 (ratio 2^8 = 256 when the
    spacing halves; the 5-point stencils of N_G = 3 give 16)."""
    s0, sig = -5.5, 2.5

    def field(n, r):
        v = SPEED.get(n, 1.0)
        amp = 1e-2 * (1 + an.GF[n] % 5)
        s = -r / v
        u = amp * np.exp(-((s - s0) / sig) ** 2)
        du = -2.0 * (s - s0) / sig ** 2 * u
        return FINF.get(n, 0.0) + u / r, du / r
    errs = []
    for f in (1, 2):
        rhs, ex, outer = _outer_rhs(coord, _refined(N, coord, f), ampl, w, field, 5)
        errs.append(max(np.max(np.abs(rhs[k][outer] - ex[k][outer])) / np.max(np.abs(ex[k][outer]))
                        for k in range(an.NGF)))
    assert errs[1] < 1e-4, errs
    assert errs[0] / errs[1] > 100.0, errs


@pytest.mark.parametrize("coord,N", [(an.SINH_SPHERICAL, (12, 8, 8)), (an.SINH_CYLINDRICAL, (10, 2, 12)),
                                     (an.SINH_CYLINDRICAL, (9, 4, 7)), (an.SPHERICAL, (16, 6, 4))])
def test_five_layer_maps_equal_closed_form(coord, N):
    g = orc.Grid(coord, N, ampl=(4.0,) * 3, sinhw=(0.3,) * 3, ng=5)
    rc, kind, src, par = g.bc_maps()
    assert rc == 0
    k2, s2, p2 = closed_form_maps(coord, N, ng=5)
    assert np.array_equal(kind, k2)
    assert np.array_equal(src, s2)
    assert np.array_equal(par, p2)
    inner = np.nonzero(kind == 2)[0]
    assert np.all(np.isin(kind[src[inner]], [0, 1]))
