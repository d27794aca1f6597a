"""Pins of the oracle's ordinary-kriging resample (CPU).

The paper prints no worked example for kriging; the pins are properties of
ordinary kriging with a variogram of no nugget: it interpolates the data
exactly, its weights sum to one (a constant shift passes through), for a
range far below the node spacing every off-node point gets the mean of its
window (all pairwise variogram values equal), an independent dense solver
gives the same weights, and invalid neighbours fall back to bilinear.
"""
import numpy as np
import pytest


def _grid(orc, nx=12, ny=10, dx=2.0, dy=3.0, x0=50.0, y0=-20.0):
    return orc.Grid(x0, y0, dx, dy, nx, ny)


def _field(g, seed=1):
    rng = np.random.default_rng(seed)
    return rng.normal(-4200.0, 30.0, (g.ny, g.nx))


def test_interpolates_the_data(orc):
    g = _grid(orc)
    src = _field(g)
    out = orc.kriging(g, src, g, 9.0)
    np.testing.assert_allclose(out, src, rtol=0, atol=1e-9)


def test_weights_sum_to_one(orc):
    g = _grid(orc)
    d = orc.Grid(g.x0 + 0.3, g.y0 - 0.7, 0.9, 1.1, 25, 24)
    src = _field(g, 2)
    a = orc.kriging(g, src, d, 7.0)
    b = orc.kriging(g, src + 123.25, d, 7.0)
    np.testing.assert_allclose(b - a, 123.25, rtol=0, atol=1e-8)
    c = orc.kriging(g, np.full((g.ny, g.nx), -3333.5), d, 7.0)
    np.testing.assert_allclose(c, -3333.5, rtol=0, atol=1e-9)


def test_tiny_range_gives_the_window_mean(orc):
    g = _grid(orc)
    # destination points midway between source nodes: every distance to a
    # window node is at least half a spacing, far beyond the range
    d = orc.Grid(g.x0 + g.dx / 2, g.y0 + g.dy / 2, g.dx, g.dy, g.nx - 1, g.ny - 1)
    src = _field(g, 3)
    out = orc.kriging(g, src, d, 1e-3)
    for a in range(d.ny):
        for b in range(d.nx):
            u, w = b + 0.5, a + 0.5              # source index coordinates
            wx = min(max(int(np.floor(u + 0.5)) - 2, 0), g.nx - 5)
            wy = min(max(int(np.floor(w + 0.5)) - 2, 0), g.ny - 5)
            want = src[wy:wy + 5, wx:wx + 5].mean()
            assert out[a, b] == pytest.approx(want, rel=0, abs=1e-9)


def test_matches_an_independent_dense_solve(orc):
    g = _grid(orc, nx=9, ny=8)
    d = orc.Grid(g.x0 - 1.0, g.y0 + 0.4, 1.3, 1.7, 15, 14)
    src = _field(g, 4)
    rng_m = 8.5
    out = orc.kriging(g, src, d, rng_m)
    for a in range(0, d.ny, 3):
        for b in range(0, d.nx, 2):
            xd = d.x0 + (b + 0.5) * d.dx
            yd = d.y0 + (a + 0.5) * d.dy
            u = min(max((xd - g.x0) / g.dx - 0.5, 0.0), g.nx - 1.0)
            w = min(max((yd - g.y0) / g.dy - 0.5, 0.0), g.ny - 1.0)
            wx = min(max(int(np.floor(u + 0.5)) - 2, 0), g.nx - 5)
            wy = min(max(int(np.floor(w + 0.5)) - 2, 0), g.ny - 5)
            jj, ii = np.meshgrid(np.arange(5), np.arange(5))
            px = ((wx + jj) * g.dx).ravel()
            py = ((wy + ii) * g.dy).ravel()
            gam = lambda h: 1.0 - np.exp(-h / rng_m)
            K = np.ones((26, 26))
            K[:25, :25] = gam(np.hypot(px[:, None] - px[None, :], py[:, None] - py[None, :]))
            K[25, 25] = 0.0
            rhs = np.ones(26)
            rhs[:25] = gam(np.hypot(px - u * g.dx, py - w * g.dy))
            lam = np.linalg.solve(K, rhs)
            want = lam[:25] @ src[wy:wy + 5, wx:wx + 5].ravel()
            assert out[a, b] == pytest.approx(want, rel=1e-11)


def test_invalid_neighbour_falls_back_to_bilinear(orc):
    g = _grid(orc)
    d = orc.Grid(g.x0, g.y0, g.dx / 2, g.dy / 2, 2 * g.nx, 2 * g.ny)
    src = _field(g, 5)
    holed = src.copy()
    holed[4, 6] = np.nan
    krig_clean = orc.kriging(g, src, d, 6.0)
    krig = orc.kriging(g, holed, d, 6.0)
    bil = orc.bilinear(g, holed, d)
    changed = ~(krig == krig_clean)
    # windows whose 5 x 5 nodes hold the hole: centres within 2 nodes, more near
    # an edge where windows move inward; 2 destination nodes per source node
    assert 0 < changed.sum() <= 14 * 14
    assert np.array_equal(krig[changed], bil[changed], equal_nan=True)
    assert np.isnan(krig).sum() == np.isnan(bil).sum() > 0


def test_grid_under_five_nodes_is_bilinear(orc):
    g = _grid(orc, nx=4, ny=9)
    d = orc.Grid(g.x0, g.y0, 0.7, 1.1, 11, 24)
    src = _field(g, 6)
    assert np.array_equal(orc.kriging(g, src, d, 5.0), orc.bilinear(g, src, d))


@pytest.mark.parametrize("u,v,wx,wy", [
    (0.3, 0.2, 0, 0),       # nearest node 0: the window [-2, 2] moves in to [0, 4]
    (2.49, 1.6, 0, 0),      # nearest node 2 / 2: window [0, 4]
    (2.51, 2.7, 1, 1),      # nearest node 3 / 3: window [1, 5]
    (6.2, 4.4, 4, 2),       # interior: nearest 6 / 4, windows [4, 8] / [2, 6]
    (8.4, 7.3, 6, 5),       # nearest 8 / 7: [6, 10] / [5, 9] -- the last full windows
    (8.6, 8.6, 7, 5),       # nearest 9 / 9: moved in to [7, 11] / [5, 9]
    (10.9, 9.0, 7, 5),      # the last nodes: windows end at the edge
])
def test_edge_window_literal(orc, u, v, wx, wy):
    """The 5 x 5 neighbourhood at and near the grid edges, written out per case
    (not recomputed): centred on the nearest source node and moved inward so
    that it stays on the grid (12 x 10 source nodes).  With a range far below
    the spacing every window node is equally uncorrelated with the point, so
    the kriged value is the window's mean, and the test field gives each
    window a different mean (a window left partly outside the grid with
    clamped indices, or centred on the floor node, fails)."""
    g = _grid(orc)
    jj, ii = np.meshgrid(np.arange(g.nx, dtype=np.float64), np.arange(g.ny, dtype=np.float64))
    src = -4000.0 + jj * jj + 100.0 * ii * ii
    d = orc.Grid(g.x0 + (u + 0.5) * g.dx - 0.5, g.y0 + (v + 0.5) * g.dy - 0.5, 1.0, 1.0, 1, 1)
    out = orc.kriging(g, src, d, 1e-3)[0, 0]
    want = src[wy:wy + 5, wx:wx + 5].mean()
    assert out == pytest.approx(want, rel=0, abs=1e-9)
