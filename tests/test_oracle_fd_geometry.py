"""Pins of the oracle's finite differences, coordinates and time step.

FD (Sec. 3, 4th-order stencils): exact on polynomials of the degree the
stencil order fixes, and not exact one degree higher.
Geometry (Sec. 2.2, Eqs. 18-20, 22): the scale factors are sqrt of the flat
metric pulled back to the logical coordinates; their derivatives match
numerical differentiation; the rescaled basis is orthonormal.
Time step: the CFL rule reproduces the paper's 8428 iterations (Sec. 4.2.1).
"""
import json
import os

import numpy as np
import pytest

import analytic as an
from oracle import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _poly_field(g, degs, rng):
    """f = prod_d P_d(xx_d - c_d), random coefficients; returns f on the grid
    and a function giving exact derivatives at a point."""
    ax = g.xx_axes()
    polys = []
    for d in range(3):
        c = np.mean(ax[d])
        coef = rng.uniform(-1, 1, degs[d] + 1)
        polys.append((np.polynomial.Polynomial(coef), c))
    X2, X1, X0 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    Xs = [X0, X1, X2]
    f = np.ones_like(X0)
    for d in range(3):
        P, c = polys[d]
        f = f * P(Xs[d] - c)

    def exact(pt, orders):
        val = 1.0
        for d in range(3):
            P, c = polys[d]
            val *= P.deriv(orders[d])(pt[d] - c) if orders[d] else P(pt[d] - c)
        return val

    return f, exact


@pytest.mark.parametrize("coord,N", [(an.SINH_SPHERICAL, (10, 8, 6)),
                                     (an.SINH_CYLINDRICAL, (8, 6, 10))])
def test_fd_exact_on_polynomials(coord, N):
    g = orc.Grid(coord, N, ampl=(3.0, 3.0, 3.0), sinhw=(0.3, 0.3, 0.3))
    rng = np.random.default_rng(7)
    i0, i1, i2 = 3 + N[0] // 2, 3 + N[1] // 2, 3 + N[2] // 2
    q = g.flat(i0, i1, i2)
    pt = [g.xx(0, i0), g.xx(1, i1), g.xx(2, i2)]
    # degree 4 in every variable: D, U+, U- and the mixed D_kD_l are exact
    f, ex = _poly_field(g, (4, 4, 4), rng)
    d1, d2, up, dn = g.fd_point(f, q)
    scale = np.max(np.abs(f))
    for k in range(3):
        o = [0, 0, 0]; o[k] = 1
        assert abs(d1[k] - ex(pt, o)) < 1e-9 * scale
        assert abs(up[k] - ex(pt, o)) < 1e-9 * scale
        assert abs(dn[k] - ex(pt, o)) < 1e-9 * scale
        for l in range(3):
            if l != k:
                o2 = [0, 0, 0]; o2[k] += 1; o2[l] += 1
                assert abs(d2[k, l] - ex(pt, o2)) < 1e-8 * scale
    # degree 5: the centred second derivative is still exact
    for k in range(3):
        degs = [0, 0, 0]; degs[k] = 5
        f, ex = _poly_field(g, degs, rng)
        d1, d2, up, dn = g.fd_point(f, q)
        o = [0, 0, 0]; o[k] = 2
        assert abs(d2[k, k] - ex(pt, o)) < 1e-8 * np.max(np.abs(f))
        # ... while first derivatives are not (a 4th-order stencil, not higher)
        o = [0, 0, 0]; o[k] = 1
        assert abs(d1[k] - ex(pt, o)) > 1e-12 * np.max(np.abs(f))
        assert abs(up[k] - ex(pt, o)) > 1e-12 * np.max(np.abs(f))
    # degree 6: second derivative not exact either
    for k in range(3):
        degs = [0, 0, 0]; degs[k] = 6
        f, ex = _poly_field(g, degs, rng)
        _, d2, _, _ = g.fd_point(f, q)
        o = [0, 0, 0]; o[k] = 2
        assert abs(d2[k, k] - ex(pt, o)) > 1e-12 * np.max(np.abs(f))


def test_upwind_error_converges_4th_order():
    """U+ and U- of a smooth non-polynomial converge at 4th order (ratio 16
    when the spacing halves)."""
    errs = {"up": [], "dn": []}
    for N in (16, 32):
        g = orc.Grid(an.SINH_CYLINDRICAL, (N, 2, N), ampl=(2.0, 2.0, 2.0), sinhw=(0.5, 0.5, 0.5))
        ax = g.xx_axes()
        X2, X1, X0 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        f = np.sin(2.0 * X0 + 0.3) * np.cos(1.7 * X2)
        j0 = 3 + N // 2
        j2 = 3 + N // 4
        _, _, up, dn = g.fd_point(f, g.flat(j0, 3, j2))
        exact = 2.0 * np.cos(2.0 * ax[0][j0] + 0.3) * np.cos(1.7 * ax[2][j2])
        errs["up"].append(abs(up[0] - exact))
        errs["dn"].append(abs(dn[0] - exact))
    # sample points are not nested here, so only the order of magnitude
    for k in errs:
        assert 8.0 < errs[k][0] / errs[k][1] < 40.0


@pytest.mark.parametrize("coord", [an.SINH_SPHERICAL, an.SINH_CYLINDRICAL, an.SPHERICAL])
def test_scale_factors_are_flat_metric(coord):
    """S_i = |d x / d xx^i| and the pulled-back flat metric is diagonal
    (Sec. 2.2: gammahat_ij = diag(S_i^2)); d S and dd S agree with numerical
    differentiation of S; the rescaled basis is orthonormal."""
    g = orc.Grid(coord, (8, 8, 8), ampl=(4.0, 4.0, 5.0), sinhw=(0.25, 0.25, 0.35))
    rng = np.random.default_rng(11)
    lo_hi = an.domain(coord)
    for _ in range(12):
        xx = np.array([rng.uniform(lo + 0.1 * (hi - lo), hi - 0.1 * (hi - lo)) for lo, hi in lo_hi])
        S, dS, ddS = g.scalefactors(xx)
        J = np.zeros((3, 3))
        h = 1e-5
        for i in range(3):
            e = np.zeros(3); e[i] = h
            J[i] = (-g.cart(xx + 2 * e) + 8 * g.cart(xx + e) - 8 * g.cart(xx - e) + g.cart(xx - 2 * e)) / (12 * h)
        metric = J @ J.T
        assert np.allclose(metric, np.diag(S ** 2), rtol=1e-8, atol=1e-8 * np.max(S ** 2))
        # numerical derivatives of S
        for k in range(3):
            e = np.zeros(3); e[k] = h
            Sp2, Sp1, Sm1, Sm2 = (g.scalefactors(xx + 2 * e)[0], g.scalefactors(xx + e)[0],
                                  g.scalefactors(xx - e)[0], g.scalefactors(xx - 2 * e)[0])
            num = (-Sp2 + 8 * Sp1 - 8 * Sm1 + Sm2) / (12 * h)
            assert np.allclose(dS[:, k], num, rtol=1e-7, atol=1e-7 * np.max(np.abs(S)))
            dSp2, dSp1, dSm1, dSm2 = (g.scalefactors(xx + 2 * e)[1], g.scalefactors(xx + e)[1],
                                      g.scalefactors(xx - e)[1], g.scalefactors(xx - 2 * e)[1])
            num2 = (-dSp2 + 8 * dSp1 - 8 * dSm1 + dSm2) / (12 * h)
            assert np.allclose(ddS[:, :, k], num2, rtol=1e-6, atol=1e-6 * np.max(np.abs(dS)) + 1e-9)
        E = g.basis(xx)
        assert np.allclose(E @ E.T, np.eye(3), atol=1e-14)
        assert np.allclose(E, J / S[:, None], atol=1e-8)


def test_oracle_coordinates_match_definitions():
    for coord, N in [(an.SINH_SPHERICAL, (6, 4, 4)), (an.SINH_CYLINDRICAL, (5, 4, 6)), (an.SPHERICAL, (4, 4, 4))]:
        ampl, w = (3.0, 3.0, 2.0), (0.3, 0.3, 0.4)
        g = orc.Grid(coord, N, ampl=ampl, sinhw=w)
        (X0, X1, X2), x, E = an.mesh(coord, N, ampl, w)
        for (i2, i1, i0) in [(0, 0, 0), (2, 3, 1), (x.shape[0] - 1, x.shape[1] - 1, x.shape[2] - 1)]:
            xx = np.array([X0[i2, i1, i0], X1[i2, i1, i0], X2[i2, i1, i0]])
            assert np.allclose([g.xx(0, i0), g.xx(1, i1), g.xx(2, i2)], xx, atol=1e-15)
            assert np.allclose(g.cart(xx), x[i2, i1, i0], rtol=1e-14, atol=1e-14)
            assert np.allclose(g.basis(xx), E[i2, i1, i0], atol=1e-14)


def test_dt_rule_reproduces_paper_iteration_count():
    fx = json.load(open(os.path.join(GOLDEN, "single_node_iterations.json")))
    g = orc.Grid(orc.SPHERICAL, fx["N"], ampl=(fx["r_max"],) * 3, cfl=fx["cfl"])
    dt = g.dt()
    iters = fx["t_final"] / dt
    assert int(np.floor(iters)) == fx["iterations"], iters
    # the limiting spacing is r_min sin(theta_min) dphi
    N = fx["N"]
    rmin = fx["r_max"] * 0.5 / N[0]
    assert dt == pytest.approx(fx["cfl"] * rmin * np.sin(np.pi / (2 * N[1])) * 2 * np.pi / N[2], rel=1e-14)


def test_dt_at_tiny_config():
    # SinhSpherical 32x16x2, AMPL 10, SINHW 0.2, CFL 0.5: dt = 0.5 r_min dtheta
    g = orc.Grid(orc.SINH_SPHERICAL, (32, 16, 2), ampl=(10.0,) * 3, sinhw=(0.2,) * 3)
    rmin = 10.0 * np.sinh(0.5 / 32 / 0.2) / np.sinh(5.0)
    assert g.dt() == pytest.approx(0.5 * rmin * np.pi / 16, rel=1e-13)
