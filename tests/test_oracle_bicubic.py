"""Pins of the oracle's Catmull-Rom resample with bilinear fallback (CPU).

The paper prints no worked example for the cubic; the pins are the spline's
closed-form properties: it passes through the samples, its midpoint weights
are (-1, 9, 9, -1) / 16, it reproduces quadratics (and their tensor products)
away from the clamped edges, a constant field stays exact, and a node that
sees a NaN among its 16 taps takes the bilinear value instead.
"""
import numpy as np
import pytest


def _grids(orc, nx=24, ny=20, dx=2.0, dy=3.0, x0=100.0, y0=-50.0):
    return orc.Grid(x0, y0, dx, dy, nx, ny)


def test_passes_through_the_samples(orc):
    g = _grids(orc)
    rng = np.random.default_rng(3)
    src = rng.normal(-4000.0, 50.0, (g.ny, g.nx))
    out = orc.bicubic(g, src, g)
    assert np.array_equal(out, src)


def test_midpoint_weights(orc):
    # destination nodes half a source cell away in x and y: t = s = 1/2
    g = _grids(orc)
    d = orc.Grid(g.x0 + g.dx / 2, g.y0 + g.dy / 2, g.dx, g.dy, g.nx - 1, g.ny - 1)
    rng = np.random.default_rng(4)
    src = rng.normal(0.0, 10.0, (g.ny, g.nx))
    out = orc.bicubic(g, src, d)
    w = np.array([-1.0, 9.0, 9.0, -1.0]) / 16.0
    for a in range(1, g.ny - 2):
        for b in range(1, g.nx - 2):
            block = src[a - 1:a + 3, b - 1:b + 3]
            want = w @ block @ w
            assert out[a, b] == pytest.approx(want, rel=1e-13, abs=1e-12)


@pytest.mark.parametrize("field", ["quadratic", "biquadratic"])
def test_reproduces_quadratics_in_the_interior(orc, field):
    g = _grids(orc, nx=30, ny=26)
    d = orc.Grid(g.x0, g.y0, g.dx / 3.0, g.dy / 2.5, 90, 65)
    jj, ii = np.meshgrid(np.arange(g.nx, dtype=np.float64), np.arange(g.ny, dtype=np.float64))

    def f(u, v):  # u, v: source index coordinates
        if field == "quadratic":
            return 3.0 + 0.5 * u - 0.25 * v + 0.125 * u * u - 0.0625 * v * v + 0.03125 * u * v
        return (1.0 + 0.5 * u + 0.25 * u * u) * (2.0 - 0.125 * v + 0.0625 * v * v)

    src = f(jj, ii)
    out = orc.bicubic(g, src, d)
    # index coordinate of each destination node (the bilinear's mapping)
    u = (d.x0 + (np.arange(d.nx) + 0.5) * d.dx - g.x0) / g.dx - 0.5
    v = (d.y0 + (np.arange(d.ny) + 0.5) * d.dy - g.y0) / g.dy - 0.5
    inner_u = (u >= 1.0) & (u <= g.nx - 3.0)
    inner_v = (v >= 1.0) & (v <= g.ny - 3.0)
    want = f(u[None, :], v[:, None])
    sel = inner_v[:, None] & inner_u[None, :]
    assert sel.sum() > 1000
    np.testing.assert_allclose(out[sel], want[sel], rtol=1e-12, atol=1e-12)
    # a cubic is not reproduced: the test can tell a wrong kernel from a right one
    src3 = jj ** 3
    out3 = orc.bicubic(g, src3, d)
    assert np.abs(out3[sel] - (u[None, :] ** 3 + 0 * v[:, None])[sel]).max() > 1e-3


def test_constant_field_everywhere(orc):
    g = _grids(orc)
    d = orc.Grid(g.x0 - 7.0, g.y0 + 1.0, 0.7, 1.3, 80, 60)
    src = np.full((g.ny, g.nx), -2750.25)
    assert np.all(orc.bicubic(g, src, d) == -2750.25)


def test_nan_tap_falls_back_to_bilinear(orc):
    g = _grids(orc)
    d = orc.Grid(g.x0, g.y0, g.dx / 2, g.dy / 2, 2 * g.nx, 2 * g.ny)
    rng = np.random.default_rng(5)
    clean = rng.normal(-3000.0, 20.0, (g.ny, g.nx))
    holed = clean.copy()
    holed[9, 11] = np.nan
    cub_clean = orc.bicubic(g, clean, d)
    cub = orc.bicubic(g, holed, d)
    bil = orc.bilinear(g, holed, d)
    changed = ~(cub == cub_clean)
    # the NaN reaches the destination nodes whose 4 x 4 footprint holds it:
    # at most 4 source cells per axis around it, i.e. 8 destination nodes
    rows, cols = np.nonzero(changed)
    assert 0 < rows.size <= 64
    assert rows.max() - rows.min() <= 7 and cols.max() - cols.min() <= 7
    # there the value is exactly the bilinear one (NaN when a corner is)
    assert np.array_equal(cub[changed], bil[changed], equal_nan=True)
    assert np.isnan(cub[changed]).sum() == np.isnan(bil).sum() > 0
    assert np.isfinite(cub[changed]).sum() > 0


def _one_node_at(orc, g, u, v):
    """Destination grid of one node at source index coordinates (u, v)."""
    return orc.Grid(g.x0 + (u + 0.5) * g.dx - 0.5, g.y0 + (v + 0.5) * g.dy - 0.5, 1.0, 1.0, 1, 1)


def test_edge_intervals_use_clamped_taps(orc):
    """First and last source intervals (reading of Sec. III-B at the border:
    taps beyond the grid repeat the edge node).  At t = 1/2 in the first
    interval the taps are (P0, P0, P1, P2), so the cubic's midpoint weights
    (-1, 9, 9, -1)/16 give (8 P0 + 9 P1 - P2)/16; in the last interval the taps
    are (P[n-3], P[n-2], P[n-1], P[n-1]): (-P[n-3] + 9 P[n-2] + 8 P[n-1])/16.
    Written out by hand; a mirrored edge ((9 P0 + 8 P1 - P2)/16) or a linear
    extrapolation ((7 P0 + 10 P1 - P2)/16) of the outside tap fails."""
    g = orc.Grid(10.0, 20.0, 2.0, 4.0, 7, 1)     # one row: the y cubic is the identity
    p = np.array([[-4000.0, -4016.0, -3992.0, -4040.0, -3980.0, -4008.0, -4064.0]])
    first = orc.bicubic(g, p, _one_node_at(orc, g, 0.5, 0.0))[0, 0]
    assert first == (8 * -4000.0 + 9 * -4016.0 - (-3992.0)) / 16
    last = orc.bicubic(g, p, _one_node_at(orc, g, 5.5, 0.0))[0, 0]
    assert last == (-(-3980.0) + 9 * -4008.0 + 8 * -4064.0) / 16
    # the interior midpoint for contrast: (-P1 + 9 P2 + 9 P3 - P4)/16
    mid = orc.bicubic(g, p, _one_node_at(orc, g, 2.5, 0.0))[0, 0]
    assert mid == (-(-4016.0) + 9 * -3992.0 + 9 * -4040.0 - (-3980.0)) / 16
    # beyond the outermost nodes the coordinate is clamped: the edge value
    assert orc.bicubic(g, p, _one_node_at(orc, g, -0.4, 0.0))[0, 0] == -4000.0
    assert orc.bicubic(g, p, _one_node_at(orc, g, 6.3, 0.0))[0, 0] == -4064.0


def test_corner_interval_is_the_product_of_edge_weights(orc):
    """At the lower-left corner, midway in both axes, the value is the tensor
    product of the first-interval weights (8, 9, -1, 0)/16 on the 3 x 3 corner
    block; the upper-right corner uses (0, -1, 9, 8)/16."""
    g = orc.Grid(0.0, 0.0, 1.0, 1.0, 5, 6)
    rng = np.random.default_rng(8)
    src = np.round(rng.normal(-3000.0, 20.0, (g.ny, g.nx)))   # integers: exact sums
    wf = np.array([8.0, 9.0, -1.0]) / 16
    lo = orc.bicubic(g, src, _one_node_at(orc, g, 0.5, 0.5))[0, 0]
    assert lo == pytest.approx(wf @ src[0:3, 0:3] @ wf, rel=1e-15, abs=0)
    wl = np.array([-1.0, 9.0, 8.0]) / 16
    hi = orc.bicubic(g, src, _one_node_at(orc, g, g.nx - 1.5, g.ny - 1.5))[0, 0]
    assert hi == pytest.approx(wl @ src[g.ny - 3:, g.nx - 3:] @ wl, rel=1e-15, abs=0)
