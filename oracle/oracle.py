"""ctypes binding of the CPU oracle (oracle/bssn_oracle.c). TEST INFRASTRUCTURE.

Two builds of the same C source: the FP64 oracle (liboracle.so, numpy
float64 arrays) and its extended-precision twin (liboracle_ld.so, numpy
longdouble arrays: x87 80-bit), the yardstick for FP64 rounding error.
Arrays are in the state layout y[24][n2][n1][n0] (i0 fastest).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")
LIBPATH_LD = os.path.join(HERE, "liboracle_ld.so")

NGF = 24
GF_NAMES = ["aDD00", "aDD01", "aDD02", "aDD11", "aDD12", "aDD22", "alpha",
            "betU0", "betU1", "betU2", "cf", "hDD00", "hDD01", "hDD02", "hDD11",
            "hDD12", "hDD22", "lambdaU0", "lambdaU1", "lambdaU2", "trK",
            "vetU0", "vetU1", "vetU2"]
GF = {n: i for i, n in enumerate(GF_NAMES)}

SINH_SPHERICAL, SINH_CYLINDRICAL, SPHERICAL = 0, 1, 2


class OracleParams(ctypes.Structure):
    _fields_ = [("coord", ctypes.c_int), ("N", ctypes.c_int * 3), ("ng", ctypes.c_int),
                ("ampl", ctypes.c_double * 3), ("sinhw", ctypes.c_double * 3),
                ("cfl", ctypes.c_double), ("diss_gauge", ctypes.c_double),
                ("diss_metric", ctypes.c_double), ("bc_kind", ctypes.c_int)]


_libs = {}


def lib(ld=False):
    """The FP64 oracle, or with ld=True its extended-precision build."""
    if ld not in _libs:
        path = LIBPATH_LD if ld else LIBPATH
        if not os.path.exists(path):
            from .build_oracle import build
            build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(OracleParams)
        fl = ctypes.c_longdouble if ld else ctypes.c_double
        dp = ctypes.POINTER(fl)
        ip = ctypes.POINTER(ctypes.c_int)
        llp = ctypes.POINTER(ctypes.c_longlong)
        sig = {
            "oracle_check": (ctypes.c_int, [P]),
            "oracle_xx": (fl, [P, ctypes.c_int, ctypes.c_int]),
            "oracle_scalefactors": (None, [P, dp, dp, dp, dp]),
            "oracle_xx_to_cart": (None, [P, dp, dp]),
            "oracle_rescaled_basis": (None, [P, dp, dp]),
            "oracle_dt": (fl, [P]),
            "oracle_bc_maps": (ctypes.c_int, [P, ip, ip, ip]),
            "oracle_apply_bcs": (ctypes.c_int, [P, dp]),
            "oracle_id_brill_lindquist": (ctypes.c_int, [P, ctypes.c_int, dp, dp, ctypes.c_int, dp]),
            "oracle_rhs": (ctypes.c_int, [P, fl, dp, dp]),
            "oracle_rhs_points": (ctypes.c_int, [P, fl, dp, ctypes.c_int, llp, dp, dp]),
            "oracle_constraints": (ctypes.c_int, [P, dp, dp, dp, dp]),
            "oracle_rk4_step": (ctypes.c_int, [P, fl, fl, dp]),
            "oracle_ssprk3_step": (ctypes.c_int, [P, fl, fl, dp]),
            "oracle_fd_point": (ctypes.c_int, [P, dp, ctypes.c_longlong, dp, dp, dp, dp]),
            "oracle_ko_point": (ctypes.c_int, [P, dp, ctypes.c_longlong, dp]),
            "oracle_num_threads": (ctypes.c_int, []),
            "oracle_set_num_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _libs[ld] = L
    return _libs[ld]


def _dp(a, ld=False):
    if a is None:
        return None
    ft = np.longdouble if ld else np.float64
    assert a.dtype == ft and a.flags.c_contiguous, (a.dtype, ft)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble if ld else ctypes.c_double))


class Grid:
    """A grid description for the oracle (host arrays only)."""

    def __init__(self, coord, N, ampl=(10.0, 10.0, 10.0), sinhw=(0.2, 0.2, 0.2), cfl=0.5, ng=3,
                 diss=(0.0, 0.0), bc_kind=0, ld=False):
        """diss: Kreiss-Oliger strengths (gauge, metric); (0, 0) is off.
        bc_kind: 0 extrapolated outer ghosts, 1 Sommerfeld radiation.
        ld: evaluate in extended precision (arrays are numpy longdouble)."""
        self.ld = bool(ld)
        self.dtype = np.longdouble if self.ld else np.float64
        self.L = lib(self.ld)
        self.p = OracleParams()
        self.p.bc_kind = int(bc_kind)
        self.p.diss_gauge = float(diss[0])
        self.p.diss_metric = float(diss[1])
        self.p.coord = int(coord)
        for d in range(3):
            self.p.N[d] = int(N[d])
            self.p.ampl[d] = float(ampl[d])
            self.p.sinhw[d] = float(sinhw[d])
        self.p.ng = int(ng)
        self.p.cfl = float(cfl)
        if self.L.oracle_check(ctypes.byref(self.p)) != 0:
            raise ValueError("oracle: unsupported grid parameters")
        self._args = (coord, tuple(N), tuple(ampl), tuple(sinhw), cfl, ng, tuple(diss), bc_kind)
        self.coord = int(coord)
        self.N = tuple(int(n) for n in N)
        self.ng = int(ng)
        self.n = tuple(n + 2 * ng for n in self.N)
        self.npts = self.n[0] * self.n[1] * self.n[2]

    def twin(self, ld=True):
        """The same grid and numerics in the other build (ld=True: the
        extended-precision reference)."""
        coord, N, ampl, sinhw, cfl, ng, diss, bc_kind = self._args
        return Grid(coord, N, ampl=ampl, sinhw=sinhw, cfl=cfl, ng=ng, diss=diss, bc_kind=bc_kind, ld=ld)

    # -- shapes ----------------------------------------------------------
    def state(self, fill=0.0):
        return np.full((NGF, self.n[2], self.n[1], self.n[0]), fill, dtype=self.dtype)

    def gf(self, count=1):
        return np.zeros((count, self.n[2], self.n[1], self.n[0]), dtype=self.dtype)

    def _a(self, a):
        return _dp(a, self.ld)

    def vec(self, v):
        """v as a contiguous array of this build's floating type"""
        return np.ascontiguousarray(v, dtype=self.dtype)

    def interior(self):
        g = self.ng
        return (slice(g, g + self.N[2]), slice(g, g + self.N[1]), slice(g, g + self.N[0]))

    # -- coordinates -----------------------------------------------------
    def xx(self, d, j):
        return self.L.oracle_xx(ctypes.byref(self.p), d, j)

    def xx_axes(self):
        return [np.array([self.xx(d, j) for j in range(self.n[d])]) for d in range(3)]

    def scalefactors(self, xx):
        xx = self.vec(xx)
        S = self.vec(np.zeros(3)); dS = self.vec(np.zeros(9)); ddS = self.vec(np.zeros(27))
        self.L.oracle_scalefactors(ctypes.byref(self.p), self._a(xx), self._a(S), self._a(dS), self._a(ddS))
        return S, dS.reshape(3, 3), ddS.reshape(3, 3, 3)

    def cart(self, xx):
        xx = self.vec(xx)
        x = self.vec(np.zeros(3))
        self.L.oracle_xx_to_cart(ctypes.byref(self.p), self._a(xx), self._a(x))
        return x

    def basis(self, xx):
        xx = self.vec(xx)
        e = self.vec(np.zeros(9))
        self.L.oracle_rescaled_basis(ctypes.byref(self.p), self._a(xx), self._a(e))
        return e.reshape(3, 3)

    def dt(self):
        return self.L.oracle_dt(ctypes.byref(self.p))

    # -- boundary maps / fill --------------------------------------------
    def bc_maps(self):
        kind = np.zeros(self.npts, dtype=np.int32)
        src = np.zeros(self.npts, dtype=np.int32)
        par = np.zeros(self.npts, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        rc = self.L.oracle_bc_maps(ctypes.byref(self.p), kind.ctypes.data_as(ip),
                                  src.ctypes.data_as(ip), par.ctypes.data_as(ip))
        return rc, kind, src, par

    def apply_bcs(self, y):
        rc = self.L.oracle_apply_bcs(ctypes.byref(self.p), self._a(y))
        if rc:
            raise RuntimeError("oracle_apply_bcs failed")
        return y

    def brill_lindquist(self, masses, positions, lapse_kind=0):
        m = self.vec(masses).reshape(-1)
        pos = self.vec(positions).reshape(-1)
        y = self.state()
        rc = self.L.oracle_id_brill_lindquist(ctypes.byref(self.p), len(m), self._a(m), self._a(pos),
                                             int(lapse_kind), self._a(y))
        if rc:
            raise RuntimeError("oracle_id_brill_lindquist failed")
        return y

    # -- right-hand sides / constraints ---------------------------------
    def rhs(self, y, eta=2.0, out=None):
        if out is None:
            out = self.state()
        rc = self.L.oracle_rhs(ctypes.byref(self.p), float(eta), self._a(y), self._a(out))
        if rc:
            raise RuntimeError("oracle_rhs failed")
        return out

    def rhs_points(self, y, idx, eta=2.0, want_ricci=False):
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros((len(idx), NGF), dtype=self.dtype)
        ric = np.zeros((len(idx), 6), dtype=self.dtype) if want_ricci else None
        rc = self.L.oracle_rhs_points(ctypes.byref(self.p), float(eta), self._a(y), len(idx),
                                     idx.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                     self._a(out), self._a(ric))
        if rc:
            raise RuntimeError("oracle_rhs_points failed")
        return (out, ric) if want_ricci else out

    def constraints(self, y):
        H = self.gf(1)
        M = self.gf(3)
        C = self.gf(3)
        rc = self.L.oracle_constraints(ctypes.byref(self.p), self._a(y), self._a(H), self._a(M), self._a(C))
        if rc:
            raise RuntimeError("oracle_constraints failed")
        return H[0], M, C

    def rk4_step(self, y, dt, eta=2.0):
        rc = self.L.oracle_rk4_step(ctypes.byref(self.p), float(eta), float(dt), self._a(y))
        if rc:
            raise RuntimeError("oracle_rk4_step failed")
        return y

    def ssprk3_step(self, y, dt, eta=2.0):
        rc = self.L.oracle_ssprk3_step(ctypes.byref(self.p), float(eta), float(dt), self._a(y))
        if rc:
            raise RuntimeError("oracle_ssprk3_step failed")
        return y

    def fd_point(self, f, idx):
        f = self.vec(f)
        d1, d2, up, dn = (self.vec(np.zeros(k)) for k in (3, 9, 3, 3))
        rc = self.L.oracle_fd_point(ctypes.byref(self.p), self._a(f), int(idx), self._a(d1), self._a(d2),
                                   self._a(up), self._a(dn))
        if rc:
            raise RuntimeError("oracle_fd_point failed")
        return d1, d2.reshape(3, 3), up, dn

    def ko_point(self, f, idx):
        """Kreiss-Oliger operator (unit strength) of f at flat index idx along
        each direction."""
        f = self.vec(f)
        ko = self.vec(np.zeros(3))
        if self.L.oracle_ko_point(ctypes.byref(self.p), self._a(f), int(idx), self._a(ko)):
            raise RuntimeError("oracle_ko_point failed")
        return ko

    def flat(self, i0, i1, i2):
        return (i2 * self.n[1] + i1) * self.n[0] + i0


def num_threads():
    return lib().oracle_num_threads()


def set_num_threads(n):
    for ld in (False, True):
        lib(ld).oracle_set_num_threads(int(n))
