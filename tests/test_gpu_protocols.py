"""GPU runs of the grid-to-grid protocols of Sec. V against the oracle.

Grid A (rows midway between recorded rows) for the three resamplers, and
grid B (every other node of a fine truth grid recorded, a random fraction of
those removed, every unrecorded fine node interpolated) for the three
resamplers and the scattered IDW path.  Values are compared node by node with
the oracle on the same inputs (NaN patterns exactly, finite values to 1e-5
relative), and so are the protocol's error metrics (MAE, RMSE against the
truth over the interpolated nodes, holes excluded and counted).
"""
import numpy as np
import pytest
import torch

from gen import grid_a_case, grid_b_case

pytestmark = pytest.mark.gpu

REL = 1e-5
KRIG_RANGE_CELLS = 3.0


@pytest.fixture(scope="module")
def ag():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22675_amd as ag
    ag.load_library()
    return ag


def _og(orc, g):
    return orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def _resample(ag, method, src, s, d, range_m=None):
    out = torch.empty((d.ny, d.nx), dtype=torch.float32, device="cuda")
    t = torch.from_numpy(np.ascontiguousarray(src, dtype=np.float32)).cuda()
    if method == "kriging":
        ag.auv_resample_kriging(t, s, out, d, range_m)
    else:
        getattr(ag, f"auv_resample_{method}")(t, s, out, d)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _oracle(orc, method, src, s, d, range_m=None):
    args = (_og(orc, s), np.asarray(src, dtype=np.float64), _og(orc, d))
    if method == "kriging":
        return orc.kriging(*args, range_m)
    return getattr(orc, method)(*args)


def _assert_close(out, ref, label):
    assert np.array_equal(np.isnan(out), np.isnan(ref)), f"{label}: hole patterns differ"
    ok = ~np.isnan(ref)
    if ok.any():
        err = np.max(np.abs(out[ok] - ref[ok]) / np.abs(ref[ok]))
        assert err <= REL, f"{label}: max rel err {err:.3e}"


def _metrics(est, truth, interp):
    v = est[interp]
    t = truth[interp]
    ok = ~np.isnan(v)
    e = v[ok] - t[ok]
    return {"holes": int((~ok).sum()), "mae": float(np.abs(e).mean()),
            "rmse": float(np.sqrt((e * e).mean()))}


def _assert_metrics_agree(out, ref, truth, interp):
    """Same holes; |MAE_out - MAE_ref| is at most the mean node difference
    (triangle inequality) and |RMSE_out - RMSE_ref| at most its RMS
    (Minkowski), with a little slack for the metric sums themselves."""
    mo = _metrics(out, truth, interp)
    mr = _metrics(ref, truth, interp)
    assert mo["holes"] == mr["holes"]
    ok = interp & ~np.isnan(ref)
    d = out[ok] - ref[ok]
    assert abs(mo["mae"] - mr["mae"]) <= np.abs(d).mean() + 1e-9 * mr["mae"]
    assert abs(mo["rmse"] - mr["rmse"]) <= np.sqrt((d * d).mean()) + 1e-9 * mr["rmse"]
    return mo


@pytest.mark.parametrize("method", ["bilinear", "bicubic", "kriging"])
@pytest.mark.parametrize("points", [1000, 70_000])
def test_grid_a_parity(ag, orc, method, points):
    s, v, d = grid_a_case(points)
    rm = KRIG_RANGE_CELLS * s.dx
    out = _resample(ag, method, v, s, d, rm)
    ref = _oracle(orc, method, v, s, d, rm)
    _assert_close(out, ref, f"grid A {method} {points}")
    assert not np.isnan(out).any()


@pytest.fixture(scope="module")
def grid_b_small():
    base = grid_b_case(320, 0.0)
    return {f: grid_b_case(320, f, truth=base["truth"]) for f in (0.01, 0.05, 0.1)}


@pytest.mark.parametrize("frac", [0.01, 0.05, 0.1])
@pytest.mark.parametrize("method", ["bilinear", "bicubic", "kriging"])
def test_grid_b_resample_parity(ag, orc, grid_b_small, frac, method):
    c = grid_b_small[frac]
    cs, ts = c["coarse_spec"], c["truth_spec"]
    rm = KRIG_RANGE_CELLS * cs.dx
    out = _resample(ag, method, c["coarse"], cs, ts, rm)
    ref = _oracle(orc, method, c["coarse"], cs, ts, rm)
    _assert_close(out, ref, f"grid B {method} {frac}")
    mo = _assert_metrics_agree(out, ref, c["truth"], c["interp"])
    assert mo["holes"] > 0  # a removed corner leaves a hole (no further fallback)


@pytest.mark.parametrize("frac", [0.01, 0.1])
def test_grid_b_idw_parity(ag, orc, grid_b_small, frac):
    c = grid_b_small[frac]
    t = c["truth_spec"]
    radius = 3.0 * t.dx
    grid = ag.auv_grid_create(t)
    dev = [torch.from_numpy(c[k]).cuda() for k in ("x", "y", "z")]
    bins = ag.auv_bin_points(grid, *dev, radius, 0)
    res = ag.grid_idw(grid, bins, power=2.0, min_pts=1, max_pts=0, with_counts=True)
    torch.cuda.synchronize()
    gz = res["z"].cpu().numpy().astype(np.float64)
    gc = res["cnt"].cpu().numpy()
    oz, oc, _ = orc.idw(_og(orc, t), c["x"], c["y"], c["z"], radius)
    assert np.array_equal(gc, oc)
    _assert_close(gz, oz, f"grid B idw {frac}")
    # recorded nodes are hits and keep their value
    np.testing.assert_allclose(gz[::2, ::2][~c["removed"]], c["z"], rtol=REL, atol=0)
    _assert_metrics_agree(gz, oz, c["truth"], c["interp"])
