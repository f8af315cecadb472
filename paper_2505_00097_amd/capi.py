"""Thin ctypes binding of libbhah.so (include/bhah.h).

Argument marshalling only: torch tensors supply device memory and streams;
every step of the evolution runs in the library's HIP kernels. The library
must have been built (paper_2505_00097_amd/build.py); there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbhah.so")

NUM_GFS = 24
NUM_AUX_GFS = 9
SINH_SPHERICAL, SINH_CYLINDRICAL, SPHERICAL = 0, 1, 2
OK, EINVAL, EDEVICE, ENOMEM = 0, -1, -2, -3
BC_EXTRAP, BC_RADIATION = 0, 1  # outer boundary kinds (bhah_grid_params.bc_kind)
RK4, SSPRK3 = 0, 1  # integrators of ensembles and the server
GF_NAMES = ["aDD00", "aDD01", "aDD02", "aDD11", "aDD12", "aDD22", "alpha",
            "betU0", "betU1", "betU2", "cf", "hDD00", "hDD01", "hDD02", "hDD11",
            "hDD12", "hDD22", "lambdaU0", "lambdaU1", "lambdaU2", "trK",
            "vetU0", "vetU1", "vetU2"]


class GridParams(ctypes.Structure):
    _fields_ = [("coord", ctypes.c_int), ("N", ctypes.c_int * 3), ("nghosts", ctypes.c_int),
                ("ampl", ctypes.c_double * 3), ("sinhw", ctypes.c_double * 3),
                ("cfl", ctypes.c_double), ("bc_kind", ctypes.c_int)]


class GaugeParams(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("shift_variant", ctypes.c_int), ("diss_gauge", ctypes.c_double),
                ("diss_metric", ctypes.c_double)]


class GridInfo(ctypes.Structure):
    _fields_ = [("n_total", ctypes.c_int * 3), ("n_points", ctypes.c_longlong),
                ("n_interior", ctypes.c_longlong), ("state_doubles", ctypes.c_longlong),
                ("aux_doubles", ctypes.c_longlong), ("workspace_doubles", ctypes.c_longlong),
                ("n_pure_outer", ctypes.c_longlong), ("n_inner", ctypes.c_longlong),
                ("dxx", ctypes.c_double * 3), ("xxmin", ctypes.c_double * 3), ("dt", ctypes.c_double)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_active", ctypes.c_int), ("n_tiles", ctypes.c_int), ("n_chunks", ctypes.c_int),
                ("graph_steps", ctypes.c_int), ("rhs_blocks", ctypes.c_int),
                ("n_classes_tuned", ctypes.c_int), ("tune_seconds", ctypes.c_double),
                ("blocks_per_cu", ctypes.c_int), ("launch_us_per_step", ctypes.c_double),
                ("launch_default_us_per_step", ctypes.c_double), ("launch_tune_seconds", ctypes.c_double),
                ("launch_candidates", ctypes.c_int), ("launch_from_cache", ctypes.c_int)]


class ServerParams(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_double), ("max_jobs", ctypes.c_int),
                ("steps_per_tick", ctypes.c_int), ("keep_results", ctypes.c_int),
                ("target_points", ctypes.c_longlong),
                ("gauge", GaugeParams), ("tune_cache_path", ctypes.c_char_p), ("integrator", ctypes.c_int)]


class JobDesc(ctypes.Structure):
    _fields_ = [("grid", GridParams), ("n_punct", ctypes.c_int), ("masses", ctypes.c_double * 16),
                ("pos", (ctypes.c_double * 3) * 16), ("lapse_kind", ctypes.c_int),
                ("nsteps", ctypes.c_longlong)]


class JobStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("steps_done", ctypes.c_longlong),
                ("interior_points", ctypes.c_longlong), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("done", ctypes.c_longlong),
                ("running", ctypes.c_longlong), ("queued", ctypes.c_longlong),
                ("point_steps", ctypes.c_longlong), ("busy_seconds", ctypes.c_double),
                ("elapsed_seconds", ctypes.c_double), ("step_ms_p50", ctypes.c_double),
                ("step_ms_p99", ctypes.c_double), ("job_s_p50", ctypes.c_double),
                ("job_s_p99", ctypes.c_double), ("held_bytes", ctypes.c_double),
                ("peak_held_bytes", ctypes.c_double), ("peak_running", ctypes.c_int),
                ("failed", ctypes.c_longlong)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_RELEASED, JOB_FAILED = 0, 1, 2, 3, 4


class BhahError(RuntimeError):
    pass


_lib = None
_vp = ctypes.c_void_p
_SIGS = {
    "bhah_last_error": (ctypes.c_char_p, []),
    "bhah_grid_create": (ctypes.c_int, [ctypes.POINTER(GridParams), ctypes.POINTER(_vp)]),
    "bhah_grid_destroy": (None, [_vp]),
    "bhah_grid_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(GridInfo)]),
    "bhah_grid_get_bc_maps": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "bhah_set_initial_data_brill_lindquist": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "bhah_apply_bcs": (ctypes.c_int, [_vp, _vp, _vp]),
    "bhah_bssn_rhs": (ctypes.c_int, [_vp, ctypes.POINTER(GaugeParams), _vp, _vp, _vp, _vp]),
    "bhah_rk4_step": (ctypes.c_int, [_vp, ctypes.POINTER(GaugeParams), ctypes.c_double, _vp, _vp, _vp]),
    "bhah_rk4_step_noalloc": (ctypes.c_int, [_vp, ctypes.POINTER(GaugeParams), ctypes.c_double, _vp, _vp]),
    "bhah_evolve": (ctypes.c_int, [_vp, ctypes.POINTER(GaugeParams), ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   _vp, _vp, _vp]),
    "bhah_hamiltonian_constraint": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "bhah_constraints": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "bhah_grid_set_tile": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "bhah_grid_get_tile": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "bhah_grid_set_waves_per_tile": (ctypes.c_int, [_vp, ctypes.c_int]),
    "bhah_grid_get_waves_per_tile": (ctypes.c_int, [_vp, _vp]),
    "bhah_grid_tune": (ctypes.c_int, [_vp, ctypes.POINTER(GaugeParams), _vp, _vp, _vp]),
    "bhah_batch_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(GaugeParams), ctypes.c_char_p,
                                         ctypes.POINTER(_vp)]),
    "bhah_batch_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "bhah_batch_set_graph_steps": (ctypes.c_int, [_vp, ctypes.c_int]),
    "bhah_batch_set_blocks_per_cu": (ctypes.c_int, [_vp, ctypes.c_int]),
    "bhah_batch_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(BatchInfo)]),
    "bhah_batch_set_launch_tuning": (ctypes.c_int, [_vp, ctypes.c_int]),
    "bhah_batch_get_tile": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "bhah_batch_destroy": (None, [_vp]),
    "bhah_server_create": (ctypes.c_int, [ctypes.POINTER(ServerParams), _vp, ctypes.POINTER(_vp)]),
    "bhah_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(JobDesc), ctypes.POINTER(ctypes.c_longlong)]),
    "bhah_server_tick": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "bhah_server_job_status": (ctypes.c_int, [_vp, ctypes.c_longlong, ctypes.POINTER(JobStatus)]),
    "bhah_server_fetch": (ctypes.c_int, [_vp, ctypes.c_longlong, _vp]),
    "bhah_server_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ServerStats)]),
    "bhah_server_destroy": (None, [_vp]),
    "bhah_probe_peaks": (ctypes.c_int, [_vp, _vp, _vp]),
    "bhah_ssprk3_step": (ctypes.c_int, [_vp, ctypes.POINTER(GaugeParams), ctypes.c_double, _vp, _vp, _vp]),
    "bhah_batch_set_integrator": (ctypes.c_int, [_vp, ctypes.c_int]),
}


def lib():
    """Load libbhah.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with paper_2505_00097_amd/build.py")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != OK:
        msg = lib().bhah_last_error().decode(errors="replace")
        raise BhahError(f"{what} failed ({rc}): {msg}")


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return _vp(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def last_error():
    return lib().bhah_last_error().decode(errors="replace")


def gauge(eta=2.0, diss=(0.0, 0.0)):
    """diss: Kreiss-Oliger strengths (gauge, metric); (0, 0) is off."""
    return GaugeParams(float(eta), 0, float(diss[0]), float(diss[1]))


# ---- the C ABI, one Python function per entry point ----------------------
def grid_create(coord, N, ampl=(10.0, 10.0, 10.0), sinhw=(0.2, 0.2, 0.2), cfl=0.5, bc_kind=0, nghosts=3):
    """nghosts 3: 4th-order differences; 5: 8th order."""
    p = GridParams()
    p.coord = int(coord)
    for d in range(3):
        p.N[d] = int(N[d])
        p.ampl[d] = float(ampl[d])
        p.sinhw[d] = float(sinhw[d])
    p.nghosts = int(nghosts)
    p.cfl = float(cfl)
    p.bc_kind = int(bc_kind)
    h = _vp()
    _check(lib().bhah_grid_create(ctypes.byref(p), ctypes.byref(h)), "bhah_grid_create")
    return h


def grid_destroy(h):
    lib().bhah_grid_destroy(h)


def grid_get_info(h):
    info = GridInfo()
    _check(lib().bhah_grid_get_info(h, ctypes.byref(info)), "bhah_grid_get_info")
    return info


def grid_get_bc_maps(h, n_points):
    import numpy as np
    kind = np.zeros(n_points, dtype=np.int32)
    src = np.zeros(n_points, dtype=np.int32)
    par = np.zeros(n_points, dtype=np.int32)
    _check(lib().bhah_grid_get_bc_maps(h, kind.ctypes.data, src.ctypes.data, par.ctypes.data),
           "bhah_grid_get_bc_maps")
    return kind, src, par


def set_initial_data_brill_lindquist(h, masses, positions, y, lapse_kind=0, stream=None):
    n = len(masses)
    m = (ctypes.c_double * max(n, 1))(*[float(v) for v in masses])
    flat = [float(c) for p in positions for c in p]
    pos = (ctypes.c_double * max(3 * n, 1))(*flat)
    _check(lib().bhah_set_initial_data_brill_lindquist(h, n, m, pos, int(lapse_kind), _ptr(y), _stream(stream)),
           "bhah_set_initial_data_brill_lindquist")


def apply_bcs(h, y, stream=None):
    _check(lib().bhah_apply_bcs(h, _ptr(y), _stream(stream)), "bhah_apply_bcs")


def bssn_rhs(h, y, rhs, aux=None, eta=2.0, diss=(0.0, 0.0), stream=None):
    gp = gauge(eta, diss)
    _check(lib().bhah_bssn_rhs(h, ctypes.byref(gp), _ptr(y), _ptr(rhs), _ptr(aux), _stream(stream)),
           "bhah_bssn_rhs")


def rk4_step(h, y, workspace, dt, eta=2.0, diss=(0.0, 0.0), stream=None):
    gp = gauge(eta, diss)
    _check(lib().bhah_rk4_step(h, ctypes.byref(gp), float(dt), _ptr(y), _ptr(workspace), _stream(stream)),
           "bhah_rk4_step")


def ssprk3_step(h, y, workspace, dt, eta=2.0, diss=(0.0, 0.0), stream=None):
    gp = gauge(eta, diss)
    _check(lib().bhah_ssprk3_step(h, ctypes.byref(gp), float(dt), _ptr(y), _ptr(workspace), _stream(stream)),
           "bhah_ssprk3_step")


def rk4_step_noalloc(h, y, dt, eta=2.0, diss=(0.0, 0.0), stream=None):
    gp = gauge(eta, diss)
    _check(lib().bhah_rk4_step_noalloc(h, ctypes.byref(gp), float(dt), _ptr(y), _stream(stream)),
           "bhah_rk4_step_noalloc")


NOALLOC_MAX_POINTS = 294912


def evolve(h, y, workspace, dt, nsteps, integrator=RK4, eta=2.0, diss=(0.0, 0.0), stream=None):
    gp = gauge(eta, diss)
    _check(lib().bhah_evolve(h, ctypes.byref(gp), int(integrator), float(dt), int(nsteps), _ptr(y), _ptr(workspace),
                             _stream(stream)), "bhah_evolve")


def hamiltonian_constraint(h, y, H, stream=None):
    _check(lib().bhah_hamiltonian_constraint(h, _ptr(y), _ptr(H), _stream(stream)),
           "bhah_hamiltonian_constraint")


def constraints(h, y, H=None, M=None, C=None, stream=None):
    _check(lib().bhah_constraints(h, _ptr(y), _ptr(H), _ptr(M), _ptr(C), _stream(stream)), "bhah_constraints")


def grid_set_tile(h, lx, ly, band):
    _check(lib().bhah_grid_set_tile(h, int(lx), int(ly), int(band)), "bhah_grid_set_tile")


def grid_get_tile(h):
    lx, ly, band = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().bhah_grid_get_tile(h, ctypes.byref(lx), ctypes.byref(ly), ctypes.byref(band)),
           "bhah_grid_get_tile")
    return lx.value, ly.value, band.value


def grid_set_waves_per_tile(h, waves):
    _check(lib().bhah_grid_set_waves_per_tile(h, int(waves)), "bhah_grid_set_waves_per_tile")


def grid_get_waves_per_tile(h):
    w = ctypes.c_int()
    _check(lib().bhah_grid_get_waves_per_tile(h, ctypes.byref(w)), "bhah_grid_get_waves_per_tile")
    return w.value


def grid_tune(h, y, rhs, eta=2.0, diss=(0.0, 0.0), stream=None):
    gp = gauge(eta, diss)
    _check(lib().bhah_grid_tune(h, ctypes.byref(gp), _ptr(y), _ptr(rhs), _stream(stream)), "bhah_grid_tune")


def probe_peaks(stream=None):
    """Measured (FP64 TFLOP/s, HBM GB/s) of the current device."""
    tf, gb = ctypes.c_double(), ctypes.c_double()
    _check(lib().bhah_probe_peaks(ctypes.byref(tf), ctypes.byref(gb), _stream(stream)), "bhah_probe_peaks")
    return tf.value, gb.value


def batch_create(grid_handles, eta=2.0, tune_cache_path=None, diss=(0.0, 0.0)):
    n = len(grid_handles)
    arr = (_vp * n)(*[g.value for g in grid_handles])
    gp = gauge(eta, diss)
    b = _vp()
    path = tune_cache_path.encode() if tune_cache_path else None
    _check(lib().bhah_batch_create(arr, n, ctypes.byref(gp), path, ctypes.byref(b)), "bhah_batch_create")
    return b


def batch_step(b, ys, wss, dts, active=None, nsteps=1, stream=None):
    n = len(ys)
    yp = (_vp * n)(*[t.data_ptr() for t in ys])
    wp = (_vp * n)(*[t.data_ptr() for t in wss])
    dp = (ctypes.c_double * n)(*[float(d) for d in dts])
    ap = None if active is None else (ctypes.c_ubyte * n)(*[1 if a else 0 for a in active])
    _check(lib().bhah_batch_step(b, yp, wp, dp, ap, int(nsteps), _stream(stream)), "bhah_batch_step")


def batch_set_graph_steps(b, steps):
    _check(lib().bhah_batch_set_graph_steps(b, int(steps)), "bhah_batch_set_graph_steps")


def batch_set_integrator(b, integrator):
    _check(lib().bhah_batch_set_integrator(b, int(integrator)), "bhah_batch_set_integrator")


def batch_set_blocks_per_cu(b, blocks_per_cu):
    _check(lib().bhah_batch_set_blocks_per_cu(b, int(blocks_per_cu)), "bhah_batch_set_blocks_per_cu")


def batch_set_launch_tuning(b, on=True):
    _check(lib().bhah_batch_set_launch_tuning(b, 1 if on else 0), "bhah_batch_set_launch_tuning")


def batch_get_info(b):
    info = BatchInfo()
    _check(lib().bhah_batch_get_info(b, ctypes.byref(info)), "bhah_batch_get_info")
    return info


def batch_get_tile(b, j):
    lx, ly, band = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().bhah_batch_get_tile(b, int(j), ctypes.byref(lx), ctypes.byref(ly), ctypes.byref(band)),
           "bhah_batch_get_tile")
    return lx.value, ly.value, band.value


def batch_destroy(b):
    lib().bhah_batch_destroy(b)


def server_create(budget_bytes, max_jobs, steps_per_tick=10, keep_results=False, eta=2.0,
                  tune_cache_path=None, stream=None, target_points=0, diss=(0.0, 0.0), integrator=RK4):
    p = ServerParams(float(budget_bytes), int(max_jobs), int(steps_per_tick), 1 if keep_results else 0,
                     int(target_points), gauge(eta, diss), tune_cache_path.encode() if tune_cache_path else None,
                     int(integrator))
    s = _vp()
    _check(lib().bhah_server_create(ctypes.byref(p), _stream(stream), ctypes.byref(s)), "bhah_server_create")
    return s


def job_desc(coord, N, ampl, sinhw, cfl, masses, positions, nsteps, lapse_kind=0, bc_kind=0, nghosts=3):
    d = JobDesc()
    d.grid = GridParams(int(coord), (ctypes.c_int * 3)(*N), int(nghosts), (ctypes.c_double * 3)(*ampl),
                        (ctypes.c_double * 3)(*sinhw), float(cfl), int(bc_kind))
    d.n_punct = len(masses)
    for i, (m, x) in enumerate(zip(masses, positions)):
        d.masses[i] = float(m)
        for k in range(3):
            d.pos[i][k] = float(x[k])
    d.lapse_kind = int(lapse_kind)
    d.nsteps = int(nsteps)
    return d


def server_submit(s, desc):
    i = ctypes.c_longlong()
    _check(lib().bhah_server_submit(s, ctypes.byref(desc), ctypes.byref(i)), "bhah_server_submit")
    return i.value


def server_tick(s):
    r, q = ctypes.c_int(), ctypes.c_int()
    _check(lib().bhah_server_tick(s, ctypes.byref(r), ctypes.byref(q)), "bhah_server_tick")
    return r.value, q.value


def server_job_status(s, job_id):
    st = JobStatus()
    _check(lib().bhah_server_job_status(s, int(job_id), ctypes.byref(st)), "bhah_server_job_status")
    return st


def server_fetch(s, job_id, dst):
    _check(lib().bhah_server_fetch(s, int(job_id), _ptr(dst)), "bhah_server_fetch")


def server_get_stats(s):
    st = ServerStats()
    _check(lib().bhah_server_get_stats(s, ctypes.byref(st)), "bhah_server_get_stats")
    return st


def server_destroy(s):
    lib().bhah_server_destroy(s)


# ---- convenience wrapper ------------------------------------------------
class Grid:
    """A grid on the current device plus helpers to allocate its arrays."""

    def __init__(self, coord, N, ampl=(10.0, 10.0, 10.0), sinhw=(0.2, 0.2, 0.2), cfl=0.5, bc_kind=0, nghosts=3):
        self.h = grid_create(coord, N, ampl, sinhw, cfl, bc_kind, nghosts)
        self.info = grid_get_info(self.h)
        self.coord = int(coord)
        self.N = tuple(int(n) for n in N)
        self.n = tuple(self.info.n_total[d] for d in range(3))
        self.dt = self.info.dt

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            grid_destroy(h)
            self.h = None

    def _empty(self, count):
        import torch
        return torch.empty((count, self.n[2], self.n[1], self.n[0]), dtype=torch.float64, device="cuda")

    def state(self):
        return self._empty(NUM_GFS)

    def aux(self):
        return self._empty(NUM_AUX_GFS)

    def workspace(self):
        import torch
        return torch.empty(self.info.workspace_doubles, dtype=torch.float64, device="cuda")

    def bc_maps(self):
        return grid_get_bc_maps(self.h, self.info.n_points)
