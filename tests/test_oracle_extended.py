"""Pins of the extended-precision build of the oracle (the same C source
compiled with long double, the reference of the GPU parity tests).

The closed-form pins of the right-hand side (flat space, Brill-Lindquist,
the textbook Ricci tensor, the pure-gauge shift) also run on this build
(test_oracle_rhs_pins.py). Here: it computes the same discrete operator as
the FP64 build (agreement to FP64 rounding on a smooth state, identical
structural zeros), and it really carries more digits where FP64 loses them:
a second difference of large values on fine cells (Sec. 3's centred
stencils), whose cancellation error FP64 amplifies and x87 long double (64
significand bits against 53) shrinks about 2^11-fold.
"""
import numpy as np
import pytest

import analytic as an
from oracle import oracle as orc
from paper_2505_00097_amd import workloads as wl


def test_extended_build_uses_a_wider_type():
    assert np.finfo(np.longdouble).nmant >= 63
    g = orc.Grid(an.SINH_SPHERICAL, (6, 4, 2), ampl=(2.0,) * 3, ld=True)
    assert g.dtype == np.longdouble and g.state().dtype == np.longdouble


@pytest.mark.parametrize("coord,N", [(an.SINH_SPHERICAL, (10, 8, 6)), (an.SINH_CYLINDRICAL, (8, 6, 10)),
                                     (an.SPHERICAL, (8, 6, 6))])
def test_second_difference_cancellation_is_smaller_in_extended_precision(coord, N):
    """f = C + a (i0 - j)^2 along i0 with C = 1, a = 1e-6: the centred second
    difference is exact on quadratics, so D2 f equals D2 of a (i0 - j)^2
    alone; the gap between the two is the cancellation error of the build
    (about Sum|w| ulp(C) / (2 a): 3e-10 relative in FP64, 1.5e-13 in long
    double). The spacing cancels in the comparison."""
    errs = {}
    for ld in (False, True):
        g = orc.Grid(coord, N, ampl=(3.0,) * 3, sinhw=(0.3,) * 3, ld=ld)
        ft = np.longdouble if ld else np.float64
        i0 = np.arange(g.n[0], dtype=ft)
        j = ft(3 + N[0] // 2)
        quad = ft(1e-6) * (i0 - j) ** 2
        shape = (g.n[2], g.n[1], g.n[0])
        f_big = np.broadcast_to(ft(1.0) + quad, shape).copy()
        f_small = np.broadcast_to(quad, shape).copy()
        q = g.flat(int(j), 3 + N[1] // 2, 3 + N[2] // 2)
        big = g.fd_point(f_big, q)[1][0, 0]
        small = g.fd_point(f_small, q)[1][0, 0]
        errs[ld] = float(abs(big - small) / abs(small))
    assert errs[False] > 1e-11, errs  # FP64 loses digits here ...
    assert errs[True] < 1e-11, errs  # ... long double keeps them
    assert errs[True] < 1e-2 * errs[False], errs


@pytest.mark.parametrize("coord,N,ampl", [(an.SINH_SPHERICAL, (12, 8, 6), (10.0,) * 3),
                                          (an.SINH_CYLINDRICAL, (12, 2, 16), (20.0,) * 3),
                                          (an.SPHERICAL, (8, 6, 6), (7.5,) * 3)])
def test_extended_and_fp64_builds_agree_to_fp64_rounding(coord, N, ampl):
    """The same FP64 input (a smooth random state, ghosts filled) through
    both builds: right-hand sides agree to FP64 rounding (relative to each
    gridfunction's largest magnitude), differ somewhere (two builds, not
    one), and zero exactly in the same places; so do the constraints."""
    g64 = orc.Grid(coord, N, ampl=ampl)
    gld = g64.twin()
    y = g64.apply_bcs(np.ascontiguousarray(wl.smooth_random_state(tuple(g64.n), seed=11)))
    r64, rld = g64.rhs(y, eta=2.0), gld.rhs(gld.vec(y), eta=2.0)
    I = (slice(None),) + g64.interior()
    a, b = r64[I].reshape(24, -1), rld[I].reshape(24, -1)
    scale = np.max(np.abs(b), axis=1)
    rel = np.max(np.abs(a - b), axis=1) / np.where(scale > 0, scale, 1.0)
    assert np.all(rel < 1e-12), rel
    assert np.max(rel) > 0.0
    assert np.array_equal(a == 0.0, b == 0.0)
    H64, Hld = g64.constraints(y)[0][g64.interior()], gld.constraints(gld.vec(y))[0][g64.interior()]
    assert np.max(np.abs(H64 - Hld)) < 1e-12 * np.max(np.abs(Hld))
