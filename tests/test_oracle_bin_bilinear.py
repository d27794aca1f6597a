"""Pins of the oracle's binning (counting sort) and bilinear resample (CPU)."""
import json
import os

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from gen import small_swath, uniform_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- binning --

@pytest.mark.parametrize("bin_log2", [16, 18, 19, 21])
def test_binning_is_a_stable_sort_into_correct_boxes(orc, bin_log2):
    s = small_swath(nodes=128, pings=80, beams=64, n_lines=3, seed=31, x0=250.0, y0=-40.0)
    x, y, z = s.x.copy(), s.y.copy(), s.z.copy()
    x[7], z[11], y[13] = np.nan, np.inf, -np.inf
    x[17] = 1e30                                      # far away
    grid = orc.Grid(s.grid.x0, s.grid.y0, s.grid.dx, s.grid.dy, s.grid.nx, s.grid.ny)
    cs, perm, n_bad, n_out = orc.bin_points(grid, x, y, z, s.radius, bin_log2)
    nbx, nby, h = orc.bin_dims(grid, s.radius, bin_log2)
    assert cs.shape[0] == nbx * nby + 1 and cs[0] == 0 and np.all(np.diff(cs) >= 0)
    assert n_bad == 3
    assert perm.shape[0] + n_bad + n_out == x.shape[0]
    assert np.unique(perm).shape[0] == perm.shape[0]
    finite = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    assert np.all(finite[perm])
    # bin of each placed sounding, from the cell_start ranges
    bid = np.repeat(np.arange(nbx * nby), np.diff(cs))
    key = bid.astype(np.int64) * (1 << 32) + perm
    assert np.all(np.diff(key) > 0)                   # sorted by (bin, index)
    # each sounding lies in its bin's box (metres, half a lattice unit slack)
    B = 2.0 ** bin_log2 / 65536.0
    bx, by = bid % nbx, bid // nbx
    lo_x = grid.x0 + (bx - h) * B - 2.0 ** -17
    lo_y = grid.y0 + (by - h) * B - 2.0 ** -17
    px, py = x[perm], y[perm]
    assert np.all(px >= lo_x) and np.all(px < lo_x + B + 2.0 ** -16)
    assert np.all(py >= lo_y) and np.all(py < lo_y + B + 2.0 ** -16)
    # every dropped finite sounding is out of reach of every node
    dropped = np.setdiff1d(np.nonzero(finite)[0], perm)
    assert dropped.shape[0] == n_out and n_out > 0
    xs, ys = grid.node_xy()
    nodes = np.stack(np.meshgrid(xs, ys), -1).reshape(-1, 2)
    d, _ = cKDTree(nodes).query(np.stack([x[dropped], y[dropped]], 1))
    assert np.all(d > s.radius)


def test_binning_stability_with_duplicates(orc):
    grid = orc.Grid(0.0, 0.0, 1.0, 1.0, 8, 8)
    x = np.array([3.2, 0.1, 3.2, 3.2, 7.9, 0.1])
    y = np.array([4.1, 0.2, 4.1, 4.1, 7.9, 0.2])
    z = -np.arange(6.0)
    cs, perm, nb, no = orc.bin_points(grid, x, y, z, 1.0, 16)
    # same position -> same bin -> ascending original index
    pos = {int(i): k for k, i in enumerate(perm)}
    assert pos[0] < pos[2] < pos[3] and pos[1] < pos[5]
    assert nb == 0 and no == 0


# --------------------------------------------------------------- bilinear --

def test_bilinear_golden_cell(orc):
    with open(os.path.join(GOLDEN, "bilinear_cell.json")) as f:
        g = json.load(f)
    # 2x2 source grid with unit spacing, nodes at 0.5 and 1.5: the unit cell
    # (x1, x2) = (0, 1) in index coordinates
    src = orc.Grid(0.0, 0.0, 1.0, 1.0, 2, 2)
    vals = np.array([[g["Q11"], g["Q21"]], [g["Q12"], g["Q22"]]])
    dst = orc.Grid(g["x"] + 0.5 - 0.5, g["y"] + 0.5 - 0.5, 1.0, 1.0, 1, 1)
    out = orc.bilinear(src, vals, dst)
    assert out[0, 0] == g["expected"]


def test_bilinear_reproduces_bilinear_functions(orc):
    src = orc.Grid(100.0, -50.0, 2.0, 3.0, 40, 30)
    xs, ys = src.node_xy()
    X, Y = np.meshgrid(xs, ys)
    f = lambda X, Y: 3.0 - 0.25 * X + 0.5 * Y + 0.01 * X * Y  # noqa: E731
    dst = orc.Grid(100.0, -50.0, 0.7, 1.1, 110, 80)
    out = orc.bilinear(src, f(X, Y), dst)
    dx, dy = dst.node_xy()
    DX, DY = np.meshgrid(dx, dy)
    inner = (DX >= xs[0]) & (DX <= xs[-1]) & (DY >= ys[0]) & (DY <= ys[-1])
    ref = f(DX, DY)
    assert inner.sum() > 5000
    assert np.max(np.abs(out[inner] - ref[inner]) / np.abs(ref[inner]).max()) < 1e-13


@pytest.mark.parametrize("shape", [((37, 23), (74, 46)), ((16, 16), (32, 32)),
                                   ((20, 13), (31, 50)), ((9, 9), (4, 5))])
def test_bilinear_matches_torch_interpolate(orc, shape):
    (sh, sw), (dh, dw) = shape
    rng = np.random.default_rng(sh * 100 + dw)
    v = -5000.0 + rng.normal(0, 300.0, (sh, sw))
    ext_x, ext_y = 2.0 * sw, 2.0 * sh
    src = orc.Grid(0.0, 0.0, 2.0, 2.0, sw, sh)
    dst = orc.Grid(0.0, 0.0, ext_x / dw, ext_y / dh, dw, dh)
    out = orc.bilinear(src, v, dst)
    ref = torch.nn.functional.interpolate(torch.from_numpy(v)[None, None], size=(dh, dw),
                                          mode="bilinear", align_corners=False)[0, 0].numpy()
    assert np.max(np.abs(out - ref)) < 1e-9


def test_bilinear_holes_propagate(orc):
    src = orc.Grid(0.0, 0.0, 2.0, 2.0, 12, 10)
    v = np.full((10, 12), -100.0)
    v[4, 6] = np.nan
    dst = orc.Grid(0.0, 0.0, 1.0, 1.0, 24, 20)
    out = orc.bilinear(src, v, dst)
    # a 2x upsample reads source node (i, j) from destination nodes 2i-1 .. 2i+2
    nan = np.isnan(out)
    assert nan.sum() == 16
    assert np.all(nan[7:11, 11:15])
    assert np.all(out[~nan] == -100.0)


def test_bilinear_constant_field(orc):
    src = orc.Grid(5.0, 5.0, 3.0, 3.0, 7, 5)
    dst = orc.Grid(0.0, 0.0, 0.9, 1.3, 33, 21)
    out = orc.bilinear(src, np.full((5, 7), -2750.5), dst)
    assert np.max(np.abs(out + 2750.5)) < 1e-12


def test_oracle_is_deterministic_across_threads(orc):
    x, y, z, g = uniform_field(n=8000, seed=41, extent=400.0, nodes=64)
    grid = orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    a = orc.idw(grid, x, y, z, radius=15.0, max_pts=9, bin_log2=19, nthreads=1)
    b = orc.idw(grid, x, y, z, radius=15.0, max_pts=9, bin_log2=19, nthreads=4)
    for u, w in zip(a, b):
        assert np.array_equal(u, w, equal_nan=True)
