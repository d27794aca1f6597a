"""GPU parity of the empirical semivariogram (auv_variogram) against the
oracle, and kriging with the fitted range against the oracle's kriging with
its own fitted range.  Bar: pair counts exact; semivariogram values to 1e-9
relative (FP64 sums of up to ~1e6 positive terms in another order differ by
at most about n 2^-53 relative); fitted range and sill to 1e-6;
kriging values within 1e-5 relative with the NaN mask exact."""
import numpy as np
import pytest
import torch

from gen import GridSpec, dem_on_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ag():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22675_amd as ag
    ag.load_library()
    return ag


def _check_vario(ag, orc, z, g, nlags):
    src = torch.from_numpy(z.astype(np.float32)).cuda()
    gx, gy, px, py = ag.auv_variogram(src, g, nlags)
    og = orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    ox, oy, opx, opy = orc.variogram(og, z.astype(np.float32).astype(np.float64), nlags)
    assert np.array_equal(px, opx) and np.array_equal(py, opy)
    assert np.array_equal(np.isnan(gx), np.isnan(ox)) and np.array_equal(np.isnan(gy), np.isnan(oy))
    ok = ~np.isnan(ox)
    assert np.allclose(gx[ok], ox[ok], rtol=1e-9, atol=0)
    ok = ~np.isnan(oy)
    assert np.allclose(gy[ok], oy[ok], rtol=1e-9, atol=0)
    return src, og


@pytest.mark.parametrize("nx,ny,dx,dy,nlags,hole", [
    (1000, 700, 4.0, 4.0, 24, 0.05),    # bands of ragged row counts, holes
    (37, 300, 2.0, 3.0, 40, 0.3),       # lags beyond the row length, anisotropic spacing
    (1, 64, 1.0, 1.0, 8, 0.0),          # a single column: no horizontal pair
])
def test_variogram_parity(ag, orc, nx, ny, dx, dy, nlags, hole):
    g = GridSpec(100.0, -50.0, dx, dy, nx, ny)
    z = dem_on_grid(g, seed=5)
    rng = np.random.default_rng(nx)
    z[rng.random(z.shape) < hole] = np.nan
    _check_vario(ag, orc, z, g, nlags)


def test_fitted_range_kriging_parity(ag, orc):
    """Range fitted on the source grid (GPU semivariogram + library fit
    against oracle semivariogram + oracle fit), then a 2x kriging resample with
    it against the oracle's kriging with its own range."""
    g = GridSpec(0.0, 0.0, 8.0, 8.0, 300, 260)
    z = dem_on_grid(g, seed=9)
    z[np.random.default_rng(2).random(z.shape) < 0.02] = np.nan
    src, og = _check_vario(ag, orc, z, g, 64)
    a, c, rc = ag.fit_variogram_range(src, g, 64)
    oa, oc, orc_rc = orc.fit_grid_range(og, z.astype(np.float32).astype(np.float64), 64)
    assert rc == ag.AUV_OK and orc_rc == 0
    assert a == pytest.approx(oa, rel=1e-6) and c == pytest.approx(oc, rel=1e-6)
    d = GridSpec(g.x0, g.y0, g.dx / 2, g.dy / 2, 2 * g.nx, 2 * g.ny)
    dst = torch.empty((d.ny, d.nx), dtype=torch.float32, device="cuda")
    ag.auv_resample_kriging(src, g, dst, d, a)
    torch.cuda.synchronize()
    od = orc.kriging(og, z.astype(np.float32).astype(np.float64),
                     orc.Grid(d.x0, d.y0, d.dx, d.dy, d.nx, d.ny), oa)
    gz = dst.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(gz), np.isnan(od))
    ok = ~np.isnan(od)
    rel = np.abs(gz[ok] - od[ok]) / np.abs(od[ok])
    assert rel.max() <= 1e-5
