"""Pins of the oracle's ghost-zone fill (Sec. 3, ghost-point classes, Fig. 1,
and the ordered boundary steps).

- The oracle classifies ghosts by the Cartesian round trip; the same maps
  follow from closed-form index reflections (restated here from the symmetry
  of the coordinates: r -> -r is (r, pi - theta, phi + pi), theta -> -theta is
  (r, -theta, phi + pi), rho -> -rho is (rho, phi + pi, z), phi periodic).
- Inner ghosts and their sources are the same Cartesian point.
- Parities: e~_(d)(dst) = p_d e~_(d)(src) for the rescaled basis of Sec. 2.2.
- Constant Cartesian scalar/vector/tensor fields are reproduced exactly at
  every ghost; fields quadratic in the grid indices are reproduced exactly
  at outer-boundary ghosts (quadratic extrapolation), corners included.
"""
import numpy as np
import pytest

import analytic as an
from oracle import oracle as orc

GRIDS = [
    # (coord, N, ampl, sinhw) -- the tiny and head-on workloads plus odd shapes
    (an.SINH_SPHERICAL, (32, 16, 2), (10.0,) * 3, (0.2,) * 3),
    (an.SINH_CYLINDRICAL, (128, 2, 256), (20.0,) * 3, (0.2,) * 3),
    (an.SINH_SPHERICAL, (12, 8, 8), (5.0,) * 3, (0.3,) * 3),
    (an.SINH_SPHERICAL, (16, 10, 6), (5.0,) * 3, (0.3,) * 3),
    (an.SINH_CYLINDRICAL, (20, 6, 24), (4.0, 4.0, 6.0), (0.3, 0.3, 0.4)),
    (an.SINH_CYLINDRICAL, (9, 4, 7), (4.0, 4.0, 6.0), (0.3, 0.3, 0.4)),
    (an.SPHERICAL, (72, 12, 24), (7.5,) * 3, (0.2,) * 3),
]


def closed_form_maps(coord, N, ng=3):
    n = [N[d] + 2 * ng for d in range(3)]
    I2, I1, I0 = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    j0, j1, j2 = I0.copy(), I1.copy(), I2.copy()
    par = np.zeros(I0.shape, dtype=np.int64)
    if coord == an.SINH_CYLINDRICAL:
        m = j0 < ng
        j0 = np.where(m, 2 * ng - 1 - j0, j0)
        j1 = np.where(m, j1 + N[1] // 2, j1)
        par = np.where(m, par ^ 0b011, par)
        j1 = ng + np.mod(j1 - ng, N[1])
    else:
        m = j0 < ng
        j0 = np.where(m, 2 * ng - 1 - j0, j0)
        j1 = np.where(m, N[1] + 2 * ng - 1 - j1, j1)
        j2 = np.where(m, j2 + N[2] // 2, j2)
        par = np.where(m, par ^ 0b101, par)
        lo = j1 < ng
        hi = j1 >= N[1] + ng
        j1 = np.where(lo, 2 * ng - 1 - j1, np.where(hi, 2 * (N[1] + ng) - 1 - j1, j1))
        j2 = np.where(lo | hi, j2 + N[2] // 2, j2)
        par = np.where(lo | hi, par ^ 0b110, par)
        j2 = ng + np.mod(j2 - ng, N[2])
    interior = ((I0 >= ng) & (I0 < N[0] + ng) & (I1 >= ng) & (I1 < N[1] + ng)
                & (I2 >= ng) & (I2 < N[2] + ng))
    same = (j0 == I0) & (j1 == I1) & (j2 == I2)
    kind = np.where(interior, 0, np.where(same, 1, 2))
    flat = (I2 * n[1] + I1) * n[0] + I0
    src = np.where(kind == 2, (j2 * n[1] + j1) * n[0] + j0, flat)
    par = np.where(kind == 2, par, 0)
    return kind.ravel(), src.ravel(), par.ravel()


@pytest.mark.parametrize("coord,N,ampl,w", GRIDS)
def test_maps_round_trip_equals_closed_form(coord, N, ampl, w):
    g = orc.Grid(coord, N, ampl=ampl, sinhw=w)
    rc, kind, src, par = g.bc_maps()
    assert rc == 0  # every source is an interior or an outer-boundary point
    k2, s2, p2 = closed_form_maps(coord, N)
    assert np.array_equal(kind, k2)
    assert np.array_equal(src, s2)
    assert np.array_equal(par, p2)
    # sources are interior or pure outer (one hop)
    inner = np.nonzero(kind == 2)[0]
    assert np.all(np.isin(kind[src[inner]], [0, 1]))
    # same Cartesian point, and e~(dst) = p e~(src) componentwise
    _, x, E = an.mesh(coord, N, ampl, w)
    xf = x.reshape(-1, 3)
    Ef = E.reshape(-1, 3, 3)
    assert np.max(np.abs(xf[inner] - xf[src[inner]])) <= 1e-13 * max(ampl)
    sign = 1.0 - 2.0 * ((par[inner, None] >> np.arange(3)) & 1)
    assert np.max(np.abs(Ef[inner] - sign[:, :, None] * Ef[src[inner]])) < 1e-13


def test_boundary_point_counts_of_the_workloads():
    expect = {  # (pure outer, inner) ghost counts
        (an.SINH_SPHERICAL, (32, 16, 2)): (96, 5568),
        (an.SINH_CYLINDRICAL, (128, 2, 256)): (3108, 212220),
    }
    for (coord, N), (nout, ninn) in expect.items():
        g = orc.Grid(coord, N, ampl=(10.0,) * 3)
        _, kind, _, _ = g.bc_maps()
        assert np.sum(kind == 1) == nout
        assert np.sum(kind == 2) == ninn


def test_boundary_point_counts_large_spherical():
    k, _, _ = closed_form_maps(an.SINH_SPHERICAL, (256, 128, 64))
    assert np.sum(k == 1) == 3 * 128 * 64
    assert np.sum(k == 2) == 335832


def _fill_frame_fields(coord, N, ampl, w, rng):
    """State whose every point holds the rescaled components of constant
    Cartesian fields: scalars, two vectors and two symmetric tensors."""
    _, x, E = an.mesh(coord, N, ampl, w)
    y = np.zeros((an.NGF,) + x.shape[:-1])
    for name in ("alpha", "cf", "trK"):
        y[an.GF[name]] = rng.uniform(-1, 1)
    for base in ("vetU0", "betU0", "lambdaU0"):
        vf = an.to_frame_vec(E, rng.uniform(-1, 1, 3))
        for i in range(3):
            y[an.GF[base] + i] = vf[..., i]
    for base in ("hDD00", "aDD00"):
        T = rng.uniform(-1, 1, (3, 3))
        T = T + T.T
        Tf = an.to_frame_sym(E, np.broadcast_to(T, x.shape[:-1] + (3, 3)))
        for c, (i, j) in enumerate(an.SYM):
            y[an.GF[base] + c] = Tf[..., i, j]
    return y


@pytest.mark.parametrize("coord,N,ampl,w", [GRIDS[0], GRIDS[2], GRIDS[4], GRIDS[5],
                                            (an.SINH_CYLINDRICAL, (32, 2, 64), (20.0,) * 3, (0.2,) * 3)])
def test_constant_cartesian_fields_reproduced_at_every_ghost(coord, N, ampl, w):
    rng = np.random.default_rng(3)
    g = orc.Grid(coord, N, ampl=ampl, sinhw=w)
    exact = _fill_frame_fields(coord, N, ampl, w, rng)
    y = np.full_like(exact, np.nan)
    I = g.interior()
    y[(slice(None),) + I] = exact[(slice(None),) + I]
    g.apply_bcs(y)
    assert np.all(np.isfinite(y))
    assert np.max(np.abs(y - exact)) < 1e-13


@pytest.mark.parametrize("coord,N,ampl,w", [GRIDS[0], GRIDS[3], GRIDS[4], GRIDS[5]])
def test_extrapolation_exact_for_quadratics(coord, N, ampl, w):
    rng = np.random.default_rng(5)
    g = orc.Grid(coord, N, ampl=ampl, sinhw=w)
    n = g.n
    I2, I1, I0 = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    c = rng.uniform(-1, 1, 10)
    q = (c[0] + c[1] * I0 + c[2] * I1 + c[3] * I2 + c[4] * I0 * I0 + c[5] * I1 * I1
         + c[6] * I2 * I2 + c[7] * I0 * I1 + c[8] * I0 * I2 + c[9] * I1 * I2)
    y = np.full((an.NGF,) + q.shape, np.nan)
    I = g.interior()
    y[:, I[0], I[1], I[2]] = q[I]
    g.apply_bcs(y)
    _, kind, _, _ = g.bc_maps()
    outer = (kind == 1).reshape(q.shape)
    assert np.any(outer)
    scale = np.max(np.abs(q))
    for gf in range(an.NGF):
        assert np.max(np.abs(y[gf][outer] - q[outer])) < 1e-12 * scale
