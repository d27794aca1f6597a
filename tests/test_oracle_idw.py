"""Pins of the FP64 oracle's IDW and nearest-neighbour search (CPU only).

Each test checks the oracle against something other than itself: closed forms,
invariants, brute force against binned search, or scipy's cKDTree.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.spatial import cKDTree

from gen import uniform_field, small_swath


def _grid(orc, g):
    return orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def _nodes(grid):
    xs, ys = grid.node_xy()
    X, Y = np.meshgrid(xs, ys)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def _clear_of_boundary(tree, nodes, r, rel=1e-9):
    """Nodes with no sounding within rel*r of the disk boundary (where the
    lattice predicate and a float64 predicate could disagree)."""
    inner = tree.query_ball_point(nodes, r * (1 - rel), return_length=True)
    outer = tree.query_ball_point(nodes, r * (1 + rel), return_length=True)
    return inner == outer


# ------------------------------------------------------------ closed forms --

def test_constant_field_is_exact(orc):
    x, y, z, g = uniform_field(n=3000, seed=11, extent=200.0, nodes=48)
    z = np.full_like(z, -4321.125)
    grid = _grid(orc, g)
    out, cnt, _ = orc.idw(grid, x, y, z, radius=9.0, power=2.0, min_pts=1)
    ok = ~np.isnan(out)
    assert ok.sum() > 0.9 * out.size
    assert np.all(out[ok] == -4321.125)
    assert np.all(np.isnan(out[cnt == 0]))


@pytest.mark.parametrize("power", [1.0, 2.0, 3.0])
def test_two_points_closed_form(orc, power):
    # one node at (1, 1); soundings at distance 0.5 and 1.5 on a line
    grid = orc.Grid(0.0, 0.0, 2.0, 2.0, 1, 1)
    x = np.array([1.5, 1.0 - 1.5])
    y = np.array([1.0, 1.0])
    z = np.array([-100.0, -130.0])
    out, cnt, nn = orc.idw(grid, x, y, z, radius=2.0, power=power)
    w1, w2 = 0.5 ** -power, 1.5 ** -power
    expect = (w1 * z[0] + w2 * z[1]) / (w1 + w2)
    assert cnt[0, 0] == 2 and nn[0, 0] == 0
    assert out[0, 0] == pytest.approx(expect, rel=1e-15, abs=0)


def test_equal_distances_give_mean(orc):
    grid = orc.Grid(0.0, 0.0, 2.0, 2.0, 1, 1)
    ang = np.deg2rad([0.0, 90.0, 180.0, 270.0])
    x = 1.0 + 0.75 * np.cos(ang)
    y = 1.0 + 0.75 * np.sin(ang)
    z = np.array([-10.0, -20.0, -40.0, -50.0])
    out, cnt, _ = orc.idw(grid, x, y, z, radius=1.0)
    assert cnt[0, 0] == 4
    assert out[0, 0] == pytest.approx(-30.0, rel=1e-14)


def test_single_neighbour_returns_its_depth(orc):
    grid = orc.Grid(0.0, 0.0, 2.0, 2.0, 1, 1)
    x, y, z = np.array([1.3, 9.0]), np.array([0.4, 9.0]), np.array([-77.7, -1.0])
    out, cnt, nn = orc.idw(grid, x, y, z, radius=2.0, power=3.0)
    assert cnt[0, 0] == 1 and nn[0, 0] == 0 and out[0, 0] == -77.7


def test_hit_returns_sounding_and_beats_min_pts(orc):
    grid = orc.Grid(10.0, 20.0, 2.0, 2.0, 4, 3)
    xs, ys = grid.node_xy()
    # sounding exactly on node (1, 2); two soundings exactly on node (0, 0)
    x = np.array([xs[2], xs[0], xs[0], xs[0] + 0.7])
    y = np.array([ys[1], ys[0], ys[0], ys[0]])
    z = np.array([-5.0, -7.0, -8.0, -100.0])
    out, cnt, nn = orc.idw(grid, x, y, z, radius=1.0, power=2.0, min_pts=5)
    assert out[1, 2] == -5.0
    assert out[0, 0] == -7.5          # mean of the coincident pair
    assert nn[0, 0] == 1              # lowest index among the tie at D^2 = 0
    assert np.isnan(out[2, 3])        # nothing in range, min_pts not met


def test_large_power_tends_to_nearest(orc):
    x, y, z, g = uniform_field(n=4000, seed=12, extent=300.0, nodes=30)
    grid = _grid(orc, g)
    out, cnt, nn = orc.idw(grid, x, y, z, radius=15.0, power=80.0)
    tree = cKDTree(np.stack([x, y], 1))
    d, _ = tree.query(_nodes(grid), k=2)
    clear = (d[:, 1] > 1.3 * d[:, 0]) & (d[:, 1] < 15.0)
    o = out.ravel()[clear]
    near = z[nn.ravel()[clear]]
    assert clear.sum() > 100
    assert np.max(np.abs(o - near)) < 1e-3


def test_k1_equals_nearest_depth(orc):
    x, y, z, g = uniform_field(n=5000, seed=13, extent=300.0, nodes=40)
    grid = _grid(orc, g)
    out, cnt, nn = orc.idw(grid, x, y, z, radius=12.0, max_pts=1)
    tree = cKDTree(np.stack([x, y], 1))
    d, i = tree.query(_nodes(grid), k=2)
    have = d[:, 0] <= 12.0 * (1 - 1e-9)
    uniq = have & (d[:, 1] > d[:, 0] * (1 + 1e-9))
    assert np.all(nn.ravel()[uniq] == i[uniq, 0])
    assert np.all(out.ravel()[have] == z[nn.ravel()[have]])


# ----------------------------------------------------------- invariants ----

def test_bounds_and_counts_vs_kdtree(orc):
    s = small_swath(nodes=96, pings=60, beams=64, n_lines=3, seed=21)
    grid = _grid(orc, s.grid)
    out, cnt, nn = orc.idw(grid, s.x, s.y, s.z, radius=s.radius, power=2.0)
    tree = cKDTree(np.stack([s.x, s.y], 1))
    nodes = _nodes(grid)
    members = tree.query_ball_point(nodes, s.radius)
    clear = _clear_of_boundary(tree, nodes, s.radius)
    o, c = out.ravel(), cnt.ravel()
    checked = 0
    for k in np.nonzero(clear)[0]:
        m = members[k]
        assert c[k] == len(m)
        if m:
            zz = s.z[m]
            assert zz.min() <= o[k] <= zz.max()
            checked += 1
        else:
            assert math.isnan(o[k])
    assert checked > 1000


def test_cap_equals_uncapped_on_k_nearest(orc):
    x, y, z, g = uniform_field(n=6000, seed=14, extent=200.0, nodes=20)
    grid = _grid(orc, g)
    k = 5
    out, cnt, _ = orc.idw(grid, x, y, z, radius=10.0, max_pts=k, power=2.0)
    tree = cKDTree(np.stack([x, y], 1))
    nodes = _nodes(grid)
    d, i = tree.query(nodes, k=k + 1)
    tested = 0
    for q in range(nodes.shape[0]):
        if not (d[q, k] <= 10.0 * (1 - 1e-9)) or d[q, k] <= d[q, k - 1] * (1 + 1e-9):
            continue  # fewer than k+1 in range, or a tie at the cap boundary
        a, b = divmod(q, grid.nx)
        sub = i[q, :k]
        one = orc.Grid(grid.x0 + b * grid.dx, grid.y0 + a * grid.dy, grid.dx,
                       grid.dy, 1, 1)
        ref, rc, _ = orc.idw(one, x[sub], y[sub], z[sub], radius=10.0, power=2.0)
        assert cnt[a, b] == k and rc[0, 0] == k
        assert out[a, b] == pytest.approx(ref[0, 0], rel=1e-14)
        tested += 1
    assert tested > 200


def test_min_pts_gives_nan(orc):
    x, y, z, g = uniform_field(n=400, seed=15, extent=200.0, nodes=40)
    grid = _grid(orc, g)
    out, cnt, _ = orc.idw(grid, x, y, z, radius=8.0, min_pts=3)
    assert np.all(np.isnan(out[cnt < 3]))
    assert np.all(~np.isnan(out[cnt >= 3]))
    assert (cnt < 3).sum() > 50 and (cnt >= 3).sum() > 50


def test_invalid_soundings_are_dropped(orc):
    x, y, z, g = uniform_field(n=3000, seed=16, extent=200.0, nodes=32)
    grid = _grid(orc, g)
    ref, rc, rn = orc.idw(grid, x, y, z, radius=8.0)
    bad_x = np.insert(x, [5, 100, 2000], [np.nan, 10.0, np.inf])
    bad_y = np.insert(y, [5, 100, 2000], [10.0, 10.0, 10.0])
    bad_z = np.insert(z, [5, 100, 2000], [-1.0, np.nan, -1.0])
    out, cnt, nn = orc.idw(grid, bad_x, bad_y, bad_z, radius=8.0)
    assert np.array_equal(out, ref, equal_nan=True) and np.array_equal(cnt, rc)
    keep = np.ones(bad_x.size, bool)
    keep[[5, 101, 2002]] = False
    remap = np.nonzero(keep)[0]
    assert np.array_equal(np.where(nn >= 0, remap[np.maximum(rn, 0)], -1), nn)


def test_soundings_outside_grid_contribute(orc):
    grid = orc.Grid(0.0, 0.0, 2.0, 2.0, 3, 3)
    x, y, z = np.array([-3.0]), np.array([1.0]), np.array([-9.0])   # 4 m left of node (0,0)
    out, cnt, nn = orc.idw(grid, x, y, z, radius=4.0)
    assert cnt[0, 0] == 1 and out[0, 0] == -9.0 and cnt[0, 1] == 0
    out, cnt, nn = orc.idw(grid, x, y, z, radius=4.0, bin_log2=18)
    assert cnt[0, 0] == 1 and out[0, 0] == -9.0


# -------------------------------------------------------- nearest / ties ---

def test_nearest_tie_breaks_on_lowest_index(orc):
    grid = orc.Grid(0.0, 0.0, 2.0, 2.0, 1, 1)          # node at (1, 1)
    x = np.array([9.0, 2.0, 1.0, 0.0, 1.0])
    y = np.array([9.0, 1.0, 2.0, 1.0, 0.0])             # four at distance 1
    z = np.array([0.0, -1.0, -2.0, -3.0, -4.0])
    for b in (-1, 16, 18):
        idx, zz = orc.nearest(grid, x, y, z, radius=1.0, bin_log2=b)
        assert idx[0, 0] == 1 and zz[0, 0] == -1.0
    out, cnt, nn = orc.idw(grid, x, y, z, radius=1.0)
    assert nn[0, 0] == 1 and cnt[0, 0] == 4 and out[0, 0] == pytest.approx(-2.5, rel=1e-15)
    # radius is inclusive: exactly on the circle is a member
    out, cnt, nn = orc.idw(grid, x, y, z, radius=1.0, max_pts=2)
    assert cnt[0, 0] == 2 and out[0, 0] == pytest.approx(-1.5, rel=1e-15)


def test_nearest_matches_kdtree(orc):
    s = small_swath(nodes=80, pings=50, beams=48, n_lines=3, seed=22)
    grid = _grid(orc, s.grid)
    idx, zz = orc.nearest(grid, s.x, s.y, s.z, radius=6.0, bin_log2=18)
    tree = cKDTree(np.stack([s.x, s.y], 1))
    d, i = tree.query(_nodes(grid), k=2)
    uniq = (d[:, 0] <= 6.0 * (1 - 1e-9)) & (d[:, 1] > d[:, 0] * (1 + 1e-9))
    empty = d[:, 0] > 6.0 * (1 + 1e-9)
    assert uniq.sum() > 1000
    assert np.all(idx.ravel()[uniq] == i[uniq, 0])
    assert np.all(zz.ravel()[uniq] == s.z[i[uniq, 0]])
    assert np.all(idx.ravel()[empty] == -1) and np.all(np.isnan(zz.ravel()[empty]))


# ------------------------------------------------- binned == brute force ---

@settings(max_examples=60, deadline=None)
@given(n=st.integers(0, 120), seed=st.integers(0, 2**31 - 1),
       snap=st.sampled_from([0.25, 0.5, 1.0, 2.0 ** -16]),
       bin_log2=st.integers(16, 20), kcap=st.sampled_from([0, 1, 3, 7]),
       radius=st.sampled_from([1.0, 2.5, 3.0, 6.0]),
       min_pts=st.integers(0, 3))
def test_binned_equals_brute_force(orc, n, seed, snap, bin_log2, kcap, radius, min_pts):
    rng = np.random.default_rng(seed)
    grid = orc.Grid(-3.0, 5.0, 1.5, 2.0, 9, 7)
    # lattice-snapped coordinates, including points outside the grid, so that
    # equal distances and D^2 == R^2 occur
    x = np.round(rng.uniform(-12.0, 22.0, n) / snap) * snap
    y = np.round(rng.uniform(-5.0, 28.0, n) / snap) * snap
    z = -np.round(rng.uniform(10.0, 20.0, n), 1)
    if n > 4:
        x[: n // 4] = np.round(x[: n // 4])         # more exact ties
        z[n // 5] = np.nan
    a = orc.idw(grid, x, y, z, radius=radius, max_pts=kcap, min_pts=min_pts, bin_log2=-1)
    b = orc.idw(grid, x, y, z, radius=radius, max_pts=kcap, min_pts=min_pts, bin_log2=bin_log2)
    for u, v in zip(a, b):
        assert np.array_equal(u, v, equal_nan=True)
    i1, z1 = orc.nearest(grid, x, y, z, radius=radius, bin_log2=-1)
    i2, z2 = orc.nearest(grid, x, y, z, radius=radius, bin_log2=bin_log2)
    assert np.array_equal(i1, i2) and np.array_equal(z1, z2, equal_nan=True)
    assert np.array_equal(i1, a[2])


def test_sampled_nodes_match_full_grid(orc):
    s = small_swath(nodes=64, pings=40, beams=40, n_lines=2, seed=23)
    grid = _grid(orc, s.grid)
    full = orc.idw(grid, s.x, s.y, s.z, radius=6.0, max_pts=16, bin_log2=19)
    nodes = np.array([0, 5, 63, 64 * 64 - 1, 1000, 2047])
    part = orc.idw(grid, s.x, s.y, s.z, radius=6.0, max_pts=16, bin_log2=19, nodes=nodes)
    for f, p in zip(full, part):
        assert np.array_equal(f.ravel()[nodes], p, equal_nan=True)


@pytest.mark.parametrize("kcap,snap", [(0, 0.0), (3, 0.0), (5, 0.25)])
def test_selected_set_bounds_by_brute_force(orc, kcap, snap):
    """orc_idw_bounds against a brute-force statement written here: lattice
    D^2 in int64 for every (node, sounding), the closed disk, the first k by
    (D^2, index), then min and max of their depths; and every O1 value lies
    within them (the clamp of step 6)."""
    rng = np.random.default_rng(71 + kcap)
    g = orc.Grid(10.0, -5.0, 1.5, 2.0, 17, 13)
    n = 600
    x = g.x0 + rng.uniform(-4, g.nx * g.dx + 4, n)
    y = g.y0 + rng.uniform(-4, g.ny * g.dy + 4, n)
    if snap:
        x = g.x0 + np.round((x - g.x0) / snap) * snap
        y = g.y0 + np.round((y - g.y0) / snap) * snap
    z = -3000.0 + rng.normal(0.0, 25.0, n)
    r = 3.0
    lo, hi = orc.idw_bounds(g, x, y, z, r, max_pts=kcap, bin_log2=17)
    X = np.rint((x - g.x0) * 65536.0).astype(np.int64)
    Y = np.rint((y - g.y0) * 65536.0).astype(np.int64)
    R = int(round(r * 65536.0))
    for a in range(g.ny):
        for b in range(g.nx):
            Xn = int(round((b + 0.5) * g.dx * 65536.0))
            Yn = int(round((a + 0.5) * g.dy * 65536.0))
            d2 = (X - Xn) ** 2 + (Y - Yn) ** 2
            mem = np.flatnonzero(d2 <= R * R)
            order = mem[np.lexsort((mem, d2[mem]))]
            if kcap:
                order = order[:kcap]
            if order.size == 0:
                assert np.isnan(lo[a, b]) and np.isnan(hi[a, b])
            else:
                assert lo[a, b] == z[order].min() and hi[a, b] == z[order].max()
    v, _, _ = orc.idw(g, x, y, z, r, 2.0, 1, kcap, bin_log2=17)
    ok = ~np.isnan(v)
    assert np.array_equal(ok, ~np.isnan(lo))
    assert np.all(v[ok] >= lo[ok]) and np.all(v[ok] <= hi[ok])
