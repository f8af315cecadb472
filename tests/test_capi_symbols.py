"""The C-ABI library loads on the host and exports every function that
include/*.h declares (no compute calls: no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(bhah_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("bhah_grid_create", "bhah_set_initial_data_brill_lindquist", "bhah_apply_bcs",
              "bhah_bssn_rhs", "bhah_rk4_step", "bhah_hamiltonian_constraint"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2505_00097_amd import capi
    if not os.path.exists(capi.LIBPATH):
        pytest.fail("libbhah.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(capi.LIBPATH)
    for n in sorted(_declared()):
        assert hasattr(L, n), n
    # the binding exposes the same names
    for n in _declared():
        assert hasattr(capi, n[len("bhah_"):]), n


def test_binding_has_no_cpu_fallback():
    import paper_2505_00097_amd.capi as capi
    src = open(capi.__file__).read()
    assert "oracle" not in src


def test_grid_create_reports_errors_without_gpu():
    """Parameter validation happens before any device call."""
    from paper_2505_00097_amd import capi
    with pytest.raises(capi.BhahError, match="nghosts|N_phi|coord"):
        p = capi.GridParams()
        p.coord = 7
        p.nghosts = 3
        h = ctypes.c_void_p()
        capi._check(capi.lib().bhah_grid_create(ctypes.byref(p), ctypes.byref(h)), "bhah_grid_create")
