"""The allocation-free RK4 entry point (bhah_rk4_step_noalloc) against the
workspace entry point it mirrors (bhah_rk4_step): bit for bit on two calls
in a row, the second on a smaller grid (the shared device array keeps the
first call's contents), with the radiation boundary and dissipation too;
a grid larger than the array is refused before any launch."""
import pytest

from paper_2505_00097_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _state(capi, w, bc_kind, diss):
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"], bc_kind=bc_kind)
    y = g.state()
    capi.set_initial_data_brill_lindquist(g.h, w["masses"], w["positions"], y)
    ws = g.workspace()
    for _ in range(2):  # a state with every field nonzero
        capi.rk4_step(g.h, y, ws, g.dt, diss=diss)
    return g, y


def test_noalloc_step_equals_workspace_step():
    import torch
    from paper_2505_00097_amd import capi
    cases = [("headon_sinhcylindrical_128x2x256", capi.BC_EXTRAP, (0.0, 0.0)),
             ("tiny_sinhspherical_32x16x2", capi.BC_EXTRAP, (0.0, 0.0)),
             ("tiny_sinhspherical_32x16x2", capi.BC_RADIATION, (0.99, 0.3))]
    for name, bc, diss in cases:
        print("CASE noalloc", name, bc, diss, flush=True)
        w = wl.WORKLOADS[name]
        g, y = _state(capi, w, bc, diss)
        assert g.info.n_points <= capi.NOALLOC_MAX_POINTS
        y1, y2 = y.clone(), y.clone()
        capi.rk4_step(g.h, y1, g.workspace(), g.dt, diss=diss)
        capi.rk4_step_noalloc(g.h, y2, g.dt, diss=diss)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2), name
        # a second step from the array's leftover contents
        capi.rk4_step(g.h, y1, g.workspace(), g.dt, diss=diss)
        capi.rk4_step_noalloc(g.h, y2, g.dt, diss=diss)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2), name


def test_noalloc_refuses_a_grid_above_the_limit():
    from paper_2505_00097_amd import capi
    w = wl.WORKLOADS["vacuum3d_sinhspherical_256x128x64"]
    g = capi.Grid(w["coord"], w["N"], w["ampl"], w["sinhw"], w["cfl"])
    assert g.info.n_points > capi.NOALLOC_MAX_POINTS
    y = g.state()
    with pytest.raises(capi.BhahError, match="BHAH_NOALLOC_MAX_POINTS"):
        capi.rk4_step_noalloc(g.h, y, g.dt)
