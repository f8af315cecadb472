"""Symmetry invariants of the discrete evolution (oracle).

Axisymmetry: data that do not depend on phi keep every phi slice bitwise
equal under the RK4 evolution (phi derivatives of equal values vanish
exactly, the reference metric of the spherical family does not depend on
phi, and the inner ghost maps only move values between equal slices), and the
components with an odd number of phi indices stay exactly zero.

Equatorial symmetry: head-on data symmetric under z -> -z stay symmetric:
components with an odd number of z indices change sign under the mirror,
the others do not. The mirrored stencils sum in a different order, so this
holds to rounding: for one right-hand side of exactly mirror-symmetric
input, to the extended-precision build's rounding (1e-16) and to 1e-13 in
FP64; to 1e-10 of each field after a short evolution of the head-on data
(a wrong sign or index breaks it at order one).

Both fail for a wrong index or parity sign anywhere in the right-hand side,
the ghost maps or the integrator.
"""
import numpy as np

import analytic as an
from gpu_helpers import gf_errors
from oracle import oracle as orc

ODD_PHI_OR_Z = [an.GF[n] for n in ("hDD02", "hDD12", "aDD02", "aDD12", "lambdaU2", "vetU2", "betU2")]


def axisymmetric_bl(og, masses, pos):
    """Brill-Lindquist data on the z axis made exactly phi-independent: one
    phi slice copied to all of them (phi is i2 on the spherical family)."""
    y = og.brill_lindquist(masses, np.array(pos))
    y[:] = y[:, og.ng:og.ng + 1, :, :]
    return og.apply_bcs(y)


def mirror_errors(y, interior):
    """per gridfunction: max |f(z) - s f(-z)| over interior points over max |f|
    (z is i2 on the cylindrical family; s = -1 for one z index)"""
    out = []
    for k in range(an.NGF):
        f = y[k]
        s = -1.0 if k in ODD_PHI_OR_Z else 1.0
        scale = np.max(np.abs(f[interior]))
        d = np.max(np.abs(f - s * f[::-1, :, :])[interior])
        out.append(d / scale if scale > 0 else d)
    return np.array(out)


def test_axisymmetric_evolution_keeps_phi_slices_equal():
    og = orc.Grid(an.SINH_SPHERICAL, (16, 8, 8), ampl=(6.0,) * 3, sinhw=(0.3,) * 3)
    y = axisymmetric_bl(og, [0.6, 0.4], [(0, 0, 0.7), (0, 0, -0.6)])
    for _ in range(10):
        og.rk4_step(y, og.dt(), eta=2.0)
    for k in range(y.shape[1]):
        assert np.array_equal(y[:, k], y[:, og.ng]), k
    for k in ODD_PHI_OR_Z:
        assert np.max(np.abs(y[k])) == 0.0, an.GF_NAMES[k]
    # the evolution is not trivial: the lapse collapses, K and the shift grow
    assert np.max(np.abs(y[an.GF["trK"]])) > 1e-3 and np.max(np.abs(y[an.GF["vetU0"]])) > 1e-7


def test_equatorial_mirror_symmetry_of_rhs_and_evolution():
    og = orc.Grid(an.SINH_CYLINDRICAL, (24, 2, 48), ampl=(20.0,) * 3, sinhw=(0.2,) * 3)
    y = og.brill_lindquist([0.5, 0.5], np.array([(0, 0, 0.5), (0, 0, -0.5)]))
    I = og.interior()
    # one right-hand side of the initial data made exactly mirror-symmetric
    # (the data are symmetric to one ulp, which the operator's second
    # differences on fine cells amplify to 1e-12): symmetric to the
    # rounding of each build
    ys = y.copy()
    for k in range(an.NGF):
        s = -1.0 if k in ODD_PHI_OR_Z else 1.0
        ys[k] = 0.5 * (ys[k] + s * ys[k][::-1])
    assert np.all(mirror_errors(ys, I) == 0.0)
    assert np.all(mirror_errors(og.twin().rhs(ys.astype(np.longdouble), eta=2.0), I) <= 1e-16)
    assert np.all(mirror_errors(og.rhs(ys, eta=2.0), I) <= 1e-13)
    for _ in range(20):
        og.rk4_step(y, og.dt(), eta=2.0)
    assert np.all(mirror_errors(y, I) <= 1e-10)
    # odd components are nonzero off the plane (the test has teeth)
    assert np.max(np.abs(y[an.GF["vetU2"]][I])) > 1e-8
