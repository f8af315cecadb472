"""Pin of the whole evolution system: the continuum BSSN system with this
gauge preserves the constraints (Eqs. 16, 17 and C^i = Lambdabar^i - Delta^i,
Sec. 2.1), so after evolving constraint-satisfying data the discrete
constraints must converge to zero at the scheme's order. A dropped or wrong
term anywhere in Eqs. 7-15 leaves a resolution-independent violation.

The data are Brill-Lindquist punctures placed outside the grid, so the
fields are smooth everywhere on it; the lapse is precollapsed (psi^-2), which
makes every term of the system active within a short time.
"""
import numpy as np

import analytic as an
from oracle import oracle as orc


def test_constraints_converge_after_evolution():
    coord, Nc, ampl, w = an.SINH_CYLINDRICAL, (12, 2, 24), (2.0,) * 3, (0.4,) * 3
    m, pos = [1.0, 0.5], [(0, 0, 2.7), (0, 0, -2.6)]
    nsteps = 8
    dt = orc.Grid(coord, Nc, ampl=ampl, sinhw=w).dt()
    errs = []
    for fine in (False, True):
        N = tuple(n * 3 if n > 2 else n for n in Nc) if fine else Nc
        g = orc.Grid(coord, N, ampl=ampl, sinhw=w)
        y = g.brill_lindquist(m, pos)
        H0, M0, C0 = g.constraints(y)
        for _ in range(nsteps * (3 if fine else 1)):
            g.rk4_step(y, dt / 3 if fine else dt, eta=2.0)
        # the evolution has switched on every variable
        I = g.interior()
        for name in ("trK", "aDD00", "aDD02", "hDD00", "lambdaU0", "lambdaU2", "vetU2", "betU2"):
            assert np.max(np.abs(y[an.GF[name]][I])) > 1e-5, name
        H, M, C = g.constraints(y)
        c, f = an.common_points(Nc, ratio=tuple(3 if n > 2 else 1 for n in Nc))
        idx = np.ix_(*(f if fine else c)[::-1])
        _, x, _ = an.mesh(coord, N, ampl, w)
        xs = x[idx]
        reg = (np.sqrt(xs[..., 0] ** 2 + xs[..., 1] ** 2) < 1.0) & (np.abs(xs[..., 2]) < 1.0)
        errs.append(np.array([np.max(np.abs(H[idx])[reg]), np.max(np.abs(M[0][idx])[reg]),
                              np.max(np.abs(M[2][idx])[reg]), np.max(np.abs(C[0][idx])[reg]),
                              np.max(np.abs(C[2][idx])[reg])]))
    ratio = errs[0] / errs[1]
    assert np.all(ratio > 40.0), (errs, ratio)
