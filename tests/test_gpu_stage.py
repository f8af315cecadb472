"""The LDS-staged phase 1 of the right-hand-side kernel (tiles of 64 points
along i0) against the per-lane gathers of the other tile shapes. Both take
the same arithmetic on the same values, so the right-hand side, the Ricci
output and whole RK4 and SSPRK3 steps are bitwise equal. On two-phi-plane
grids every phase-1 stencil is staged; on the others the mixed pairs (0, 1)
and (0, 2) are. The cases cover ragged row tiles (lanes past the grid
compute a clamped point and store nothing), dissipation, 8th order where a
staged form is built, and the paired epilogue (full tiles) beside the
per-lane one (ragged tiles). The staged kernel is checked against the
oracle by the parity tests, which run at the tuned tiles."""
import pytest

from paper_2505_00097_amd import workloads as wl
import test_gpu_parity as tp

pytestmark = pytest.mark.gpu

KO = (0.99, 0.3)


def _tiles(coord):
    """Row tiles (staged) first, then shapes that gather; every tile has
    extent 1 along phi (i1 on SinhCylindrical grids, i2 otherwise)."""
    if coord == wl.SINH_CYLINDRICAL:
        return [(6, 0, 1), (5, 0, 1), (3, 0, 1)]
    return [(6, 0, 1), (5, 1, 1), (3, 3, 1)]


def _grid(name, ng):
    from paper_2505_00097_amd import capi
    coord, N, ampl, w = tp.GRIDS[name]
    return capi.Grid(coord, N, ampl, w, nghosts=ng)


@pytest.mark.parametrize("name,ng,diss", [
    ("tiny", 3, (0.0, 0.0)), ("tiny", 3, KO), ("tiny", 5, (0.0, 0.0)), ("tiny", 5, KO),
    ("cyl_ragged", 3, (0.0, 0.0)), ("cyl_ragged", 3, KO), ("cyl_ragged", 5, (0.0, 0.0)), ("cyl_ragged", 5, KO),
    ("sph_ragged", 3, (0.0, 0.0)), ("sph_ragged", 3, KO),
    ("cyl_3d", 3, (0.0, 0.0)), ("cyl_3d", 3, KO),
    ("spherical", 3, (0.0, 0.0)), ("spherical", 3, KO)])
def test_staged_rhs_bitwise_equals_gathers(name, ng, diss):
    tp._print_case("staged rhs", name, ng, diss)
    import torch
    from paper_2505_00097_amd import capi
    g = _grid(name, ng)
    y = torch.from_numpy(wl.smooth_random_state(g.n, seed=5)).cuda()
    tiles = _tiles(g.coord)
    outs = []
    for tile in tiles:
        capi.grid_set_tile(g.h, *tile)
        r = g.state()
        r.zero_()
        a = g.aux()
        a.zero_()
        capi.bssn_rhs(g.h, y, r, a, diss=diss)
        torch.cuda.synchronize()
        outs.append((r.cpu(), a.cpu()))
    assert torch.isfinite(outs[0][0]).all()
    for tile, (r, a) in zip(tiles[1:], outs[1:]):
        assert torch.equal(r, outs[0][0]), tile
        assert torch.equal(a, outs[0][1]), tile


@pytest.mark.parametrize("name", ["cyl_ragged", "cyl_3d", "spherical"])
def test_staged_steps_bitwise_equal_gathers(name):
    """RK4 and SSPRK3 steps (the stage combinations of the epilogue, SSPRK3
    mixing two states) with dissipation, at every tile shape."""
    tp._print_case("staged steps", name)
    import torch
    from paper_2505_00097_amd import capi
    g = _grid(name, 3)
    y0 = torch.from_numpy(wl.smooth_random_state(g.n, seed=6)).cuda()
    ws = g.workspace()
    for step in (capi.rk4_step, capi.ssprk3_step):
        ref = None
        for tile in _tiles(g.coord):
            capi.grid_set_tile(g.h, *tile)
            y = y0.clone()
            step(g.h, y, ws, g.dt, diss=KO)
            torch.cuda.synchronize()
            if ref is None:
                ref = y
                assert torch.isfinite(ref).all()
            else:
                assert torch.equal(y, ref), (step.__name__, tile)
