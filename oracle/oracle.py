"""ctypes binding of the CPU oracle (oracle/bssn_oracle.c). TEST INFRASTRUCTURE.

Arrays are numpy float64 in the state layout y[24][n2][n1][n0] (i0 fastest).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

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


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from .build_oracle import build
            build()
        L = ctypes.CDLL(LIBPATH)
        P = ctypes.POINTER(OracleParams)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        llp = ctypes.POINTER(ctypes.c_longlong)
        sig = {
            "oracle_check": (ctypes.c_int, [P]),
            "oracle_xx": (ctypes.c_double, [P, ctypes.c_int, ctypes.c_int]),
            "oracle_scalefactors": (None, [P, dp, dp, dp, dp]),
            "oracle_xx_to_cart": (None, [P, dp, dp]),
            "oracle_rescaled_basis": (None, [P, dp, dp]),
            "oracle_dt": (ctypes.c_double, [P]),
            "oracle_bc_maps": (ctypes.c_int, [P, ip, ip, ip]),
            "oracle_apply_bcs": (ctypes.c_int, [P, dp]),
            "oracle_id_brill_lindquist": (ctypes.c_int, [P, ctypes.c_int, dp, dp, ctypes.c_int, dp]),
            "oracle_rhs": (ctypes.c_int, [P, ctypes.c_double, dp, dp]),
            "oracle_rhs_points": (ctypes.c_int, [P, ctypes.c_double, dp, ctypes.c_int, llp, dp, dp]),
            "oracle_constraints": (ctypes.c_int, [P, dp, dp, dp, dp]),
            "oracle_rk4_step": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double, dp]),
            "oracle_ssprk3_step": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double, dp]),
            "oracle_fd_point": (ctypes.c_int, [P, dp, ctypes.c_longlong, dp, dp, dp, dp]),
            "oracle_ko_point": (ctypes.c_int, [P, dp, ctypes.c_longlong, dp]),
            "oracle_num_threads": (ctypes.c_int, []),
            "oracle_set_num_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Grid:
    """A grid description for the oracle (host arrays only)."""

    def __init__(self, coord, N, ampl=(10.0, 10.0, 10.0), sinhw=(0.2, 0.2, 0.2), cfl=0.5, ng=3,
                 diss=(0.0, 0.0), bc_kind=0):
        """diss: Kreiss-Oliger strengths (gauge, metric); (0, 0) is off.
        bc_kind: 0 extrapolated outer ghosts, 1 Sommerfeld radiation."""
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
        if lib().oracle_check(ctypes.byref(self.p)) != 0:
            raise ValueError("oracle: unsupported grid parameters")
        self.coord = int(coord)
        self.N = tuple(int(n) for n in N)
        self.ng = int(ng)
        self.n = tuple(n + 2 * ng for n in self.N)
        self.npts = self.n[0] * self.n[1] * self.n[2]

    # -- shapes ----------------------------------------------------------
    def state(self, fill=0.0):
        return np.full((NGF, self.n[2], self.n[1], self.n[0]), fill, dtype=np.float64)

    def gf(self, count=1):
        return np.zeros((count, self.n[2], self.n[1], self.n[0]), dtype=np.float64)

    def interior(self):
        g = self.ng
        return (slice(g, g + self.N[2]), slice(g, g + self.N[1]), slice(g, g + self.N[0]))

    # -- coordinates -----------------------------------------------------
    def xx(self, d, j):
        return lib().oracle_xx(ctypes.byref(self.p), d, j)

    def xx_axes(self):
        return [np.array([self.xx(d, j) for j in range(self.n[d])]) for d in range(3)]

    def scalefactors(self, xx):
        xx = np.ascontiguousarray(xx, dtype=np.float64)
        S = np.zeros(3); dS = np.zeros(9); ddS = np.zeros(27)
        lib().oracle_scalefactors(ctypes.byref(self.p), _dp(xx), _dp(S), _dp(dS), _dp(ddS))
        return S, dS.reshape(3, 3), ddS.reshape(3, 3, 3)

    def cart(self, xx):
        xx = np.ascontiguousarray(xx, dtype=np.float64)
        x = np.zeros(3)
        lib().oracle_xx_to_cart(ctypes.byref(self.p), _dp(xx), _dp(x))
        return x

    def basis(self, xx):
        xx = np.ascontiguousarray(xx, dtype=np.float64)
        e = np.zeros(9)
        lib().oracle_rescaled_basis(ctypes.byref(self.p), _dp(xx), _dp(e))
        return e.reshape(3, 3)

    def dt(self):
        return lib().oracle_dt(ctypes.byref(self.p))

    # -- boundary maps / fill --------------------------------------------
    def bc_maps(self):
        kind = np.zeros(self.npts, dtype=np.int32)
        src = np.zeros(self.npts, dtype=np.int32)
        par = np.zeros(self.npts, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        rc = lib().oracle_bc_maps(ctypes.byref(self.p), kind.ctypes.data_as(ip),
                                  src.ctypes.data_as(ip), par.ctypes.data_as(ip))
        return rc, kind, src, par

    def apply_bcs(self, y):
        rc = lib().oracle_apply_bcs(ctypes.byref(self.p), _dp(y))
        if rc:
            raise RuntimeError("oracle_apply_bcs failed")
        return y

    def brill_lindquist(self, masses, positions, lapse_kind=0):
        m = np.ascontiguousarray(masses, dtype=np.float64).reshape(-1)
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1)
        y = self.state()
        rc = lib().oracle_id_brill_lindquist(ctypes.byref(self.p), len(m), _dp(m), _dp(pos),
                                             int(lapse_kind), _dp(y))
        if rc:
            raise RuntimeError("oracle_id_brill_lindquist failed")
        return y

    # -- right-hand sides / constraints ---------------------------------
    def rhs(self, y, eta=2.0, out=None):
        if out is None:
            out = self.state()
        rc = lib().oracle_rhs(ctypes.byref(self.p), float(eta), _dp(y), _dp(out))
        if rc:
            raise RuntimeError("oracle_rhs failed")
        return out

    def rhs_points(self, y, idx, eta=2.0, want_ricci=False):
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros((len(idx), NGF))
        ric = np.zeros((len(idx), 6)) if want_ricci else None
        rc = lib().oracle_rhs_points(ctypes.byref(self.p), float(eta), _dp(y), len(idx),
                                     idx.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                     _dp(out), _dp(ric))
        if rc:
            raise RuntimeError("oracle_rhs_points failed")
        return (out, ric) if want_ricci else out

    def constraints(self, y):
        H = self.gf(1)
        M = self.gf(3)
        C = self.gf(3)
        rc = lib().oracle_constraints(ctypes.byref(self.p), _dp(y), _dp(H), _dp(M), _dp(C))
        if rc:
            raise RuntimeError("oracle_constraints failed")
        return H[0], M, C

    def rk4_step(self, y, dt, eta=2.0):
        rc = lib().oracle_rk4_step(ctypes.byref(self.p), float(eta), float(dt), _dp(y))
        if rc:
            raise RuntimeError("oracle_rk4_step failed")
        return y

    def ssprk3_step(self, y, dt, eta=2.0):
        rc = lib().oracle_ssprk3_step(ctypes.byref(self.p), float(eta), float(dt), _dp(y))
        if rc:
            raise RuntimeError("oracle_ssprk3_step failed")
        return y

    def fd_point(self, f, idx):
        f = np.ascontiguousarray(f, dtype=np.float64)
        d1 = np.zeros(3); d2 = np.zeros(9); up = np.zeros(3); dn = np.zeros(3)
        rc = lib().oracle_fd_point(ctypes.byref(self.p), _dp(f), int(idx), _dp(d1), _dp(d2),
                                   _dp(up), _dp(dn))
        if rc:
            raise RuntimeError("oracle_fd_point failed")
        return d1, d2.reshape(3, 3), up, dn

    def ko_point(self, f, idx):
        """Kreiss-Oliger operator (unit strength) of f at flat index idx along
        each direction."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        ko = np.zeros(3)
        if lib().oracle_ko_point(ctypes.byref(self.p), _dp(f), int(idx), _dp(ko)):
            raise RuntimeError("oracle_ko_point failed")
        return ko

    def flat(self, i0, i1, i2):
        return (i2 * self.n[1] + i1) * self.n[0] + i0


def num_threads():
    return lib().oracle_num_threads()


def set_num_threads(n):
    lib().oracle_set_num_threads(int(n))
