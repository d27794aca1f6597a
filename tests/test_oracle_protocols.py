"""Pins for the grid-to-grid protocols of Sec. V on synthetic seafloor.

Grid A fills rows midway between successive recorded rows; grid B records
every other node of a fine truth grid, removes a random fraction of the
recorded nodes and interpolates every unrecorded fine node.  These tests fix
the geometry of both cases against closed forms (midpoint rows, nodes that
coincide) and the oracle's behaviour on them, so that the GPU protocol runs
are compared with an oracle whose inputs are known to be laid out right.
"""
import numpy as np
import pytest

from gen import grid_a_case, grid_b_case


def _og(orc, g):
    return orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def test_grid_a_rows_lie_midway(orc):
    """Bilinear at a destination row is the mean of the two recorded rows
    around it (the x coordinate falls on a node), and Catmull-Rom at the
    midpoint of an interior row pair is (-P0 + 9 P1 + 9 P2 - P3) / 16."""
    src, v, dst = grid_a_case(5000)
    assert src.ny == dst.ny + 1 and src.nx == dst.nx
    assert dst.nx * dst.ny >= 5000
    r = v.astype(np.float64)
    bil = orc.bilinear(_og(orc, src), r, _og(orc, dst))
    np.testing.assert_allclose(bil, 0.5 * (r[:-1] + r[1:]), rtol=0, atol=1e-9)
    cub = orc.bicubic(_og(orc, src), r, _og(orc, dst))
    mid = (-r[:-3] + 9.0 * r[1:-2] + 9.0 * r[2:-1] - r[3:]) / 16.0
    np.testing.assert_allclose(cub[1:-1], mid, rtol=0, atol=1e-9)


def test_grid_a_large_cases_repeat_one_patch():
    src, v, dst = grid_a_case(3_000_000, patch=512)
    assert v.shape == (src.ny, src.nx) and v.dtype == np.float32
    np.testing.assert_array_equal(v[:512, :512], v[512:1024, 512:1024])
    _, v_small, _ = grid_a_case(200_000, patch=512)
    np.testing.assert_array_equal(v[:400, :400], v_small[:400, :400])


@pytest.mark.parametrize("frac", [0.0, 0.01, 0.1])
def test_grid_b_removal_and_masks(frac):
    c = grid_b_case(96, frac)
    nc = 48
    m = nc * nc
    assert c["removed"].sum() == int(round(frac * m))
    assert np.isnan(c["coarse"]).sum() == c["removed"].sum()
    # interpolated points: every fine node that was not recorded
    assert c["interp"].sum() == 96 * 96 - (m - c["removed"].sum())
    np.testing.assert_array_equal(c["interp"][::2, ::2], c["removed"])
    # recorded nodes carry the truth at the coinciding fine node
    ok = ~c["removed"]
    np.testing.assert_array_equal(c["coarse"][ok], c["truth"][::2, ::2][ok].astype(np.float32))
    np.testing.assert_array_equal(c["z"], c["truth"][::2, ::2][ok])
    # the scattered copy sits exactly on the fine node centres
    t = c["truth_spec"]
    b = np.rint((c["x"] - t.x0) / t.dx - 0.5).astype(int)
    a = np.rint((c["y"] - t.y0) / t.dy - 0.5).astype(int)
    np.testing.assert_array_equal(c["x"], t.x0 + (b + 0.5) * t.dx)
    assert (a % 2 == 0).all() and (b % 2 == 0).all()
    np.testing.assert_array_equal(c["z"], c["truth"][a, b])


def test_grid_b_seeded_and_truth_reuse():
    a = grid_b_case(64, 0.05)
    b = grid_b_case(64, 0.05, truth=a["truth"])
    np.testing.assert_array_equal(a["removed"], b["removed"])
    c = grid_b_case(64, 0.1, truth=a["truth"])
    assert c["removed"].sum() > a["removed"].sum()
    with pytest.raises(ValueError):
        grid_b_case(64, 0.05, truth=a["truth"][:10])


def test_grid_b_coarse_nodes_map_onto_fine_nodes(orc):
    """Resampling the recorded grid onto the fine grid returns each recorded
    value at its own fine node, and a plane is reproduced at every fine node
    inside the recorded hull by bilinear and Catmull-Rom (both reproduce
    linear fields; Catmull-Rom only where its four taps are inside the grid,
    since edge-clamped taps bend it), whatever the node spacing."""
    c = grid_b_case(64, 0.0)
    cs, ts = c["coarse_spec"], c["truth_spec"]
    v = c["coarse"].astype(np.float64)
    bil = orc.bilinear(_og(orc, cs), v, _og(orc, ts))
    np.testing.assert_array_equal(bil[::2, ::2], v)
    xs = cs.x0 + (np.arange(cs.nx) + 0.5) * cs.dx
    ys = cs.y0 + (np.arange(cs.ny) + 0.5) * cs.dy
    plane = -4000.0 + 0.37 * xs[None, :] - 0.21 * ys[:, None]
    fx = ts.x0 + (np.arange(ts.nx) + 0.5) * ts.dx
    fy = ts.y0 + (np.arange(ts.ny) + 0.5) * ts.dy
    want = -4000.0 + 0.37 * fx[None, :] - 0.21 * fy[:, None]
    # the last fine row and column lie beyond the last recorded node
    got = orc.bilinear(_og(orc, cs), plane, _og(orc, ts))
    np.testing.assert_allclose(got[:-1, :-1], want[:-1, :-1], rtol=0, atol=1e-9)
    # fine node j sits at coarse coordinate j / 2: taps in range for 2 <= j < 2 nc - 4
    got = orc.bicubic(_og(orc, cs), plane, _og(orc, ts))
    k = slice(2, 2 * cs.nx - 4)
    np.testing.assert_allclose(got[k, k], want[k, k], rtol=0, atol=1e-9)


def test_grid_b_idw_fill_with_no_removal_hits_recorded_nodes(orc):
    """With nothing removed, IDW from the recorded nodes returns each recorded
    value exactly at its own fine node (a hit) and fills every other fine node
    from the recorded nodes within the radius."""
    c = grid_b_case(64, 0.0)
    t = c["truth_spec"]
    og = orc.Grid(t.x0, t.y0, t.dx, t.dy, t.nx, t.ny)
    z, cnt, nn = orc.idw(og, c["x"], c["y"], c["z"], 3.0 * t.dx)
    np.testing.assert_array_equal(z[::2, ::2], c["truth"][::2, ::2])
    assert (cnt > 0).all()
