"""The allocation-free entry point (auv_grid_idw_noalloc) against the
allocating path (auv_bin_points + auv_interp_idw) through the C ABI.

Both run the same binning and IDW kernels, so every output must agree exactly:
values, counts, NaN masks, nearest indices and depths.  Two calls in a row
share the static scratch: the 2M-sounding swath first, then a smaller swath,
whose result must not depend on what the first call left behind.  The small
case is also held to the oracle (counts and nearest exact, values within
1e-5 relative).
"""
import numpy as np
import pytest
import torch

from gen import small_swath, workload_cfg2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ag():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22675_amd as ag
    ag.load_library()
    return ag


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _outputs(ag, grid, dev):
    shape = (grid.ny, grid.nx)
    return (torch.full(shape, 7.0, dtype=torch.float32, device=dev),
            torch.full(shape, -7, dtype=torch.int32, device=dev),
            torch.full(shape, -7, dtype=torch.int32, device=dev),
            torch.full(shape, 7.0, dtype=torch.float32, device=dev))


def _reference(ag, s, bin_log2, params):
    grid = ag.auv_grid_create(s.grid)
    x, y, z = _dev(s.x), _dev(s.y), _dev(s.z)
    bins = ag.auv_bin_points(grid, x, y, z, params.radius, bin_log2)
    out = _outputs(ag, grid, x.device)
    ag.auv_interp_idw(grid, bins, params, *out)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _noalloc(ag, s, bin_log2, params):
    grid = ag.auv_grid_create(s.grid)
    x, y, z = _dev(s.x), _dev(s.y), _dev(s.z)
    out = _outputs(ag, grid, x.device)
    print(f"noalloc call: n={s.n} grid={s.grid.nx}x{s.grid.ny} bin_log2={bin_log2}", flush=True)
    ag.auv_grid_idw_noalloc(grid, x, y, z, bin_log2, params, *out)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _assert_same(a, b, label):
    za, ca, na, nza = a
    zb, cb, nb, nzb = b
    assert np.array_equal(ca, cb), f"{label}: counts differ"
    assert np.array_equal(na, nb), f"{label}: nearest indices differ"
    assert np.array_equal(np.isnan(za), np.isnan(zb)), f"{label}: NaN masks differ"
    assert np.array_equal(za, zb, equal_nan=True), f"{label}: values differ"
    assert np.array_equal(nza, nzb, equal_nan=True), f"{label}: nearest depths differ"


def test_noalloc_matches_allocating_path_twice(ag, orc):
    big = workload_cfg2()
    p_big = ag.idw_params(power=big.power, radius=big.radius, min_pts=big.min_pts,
                          max_pts=big.max_pts)
    small = small_swath(nodes=200, pings=90, beams=120, n_lines=3, seed=41)
    p_small = ag.idw_params(power=3.0, radius=small.radius, min_pts=2, max_pts=8)

    got_big = _noalloc(ag, big, 0, p_big)
    got_small = _noalloc(ag, small, 18, p_small)
    _assert_same(got_big, _reference(ag, big, 0, p_big), "2M swath")
    _assert_same(got_small, _reference(ag, small, 18, p_small), "small swath after 2M")

    g = small.grid
    og = orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    oz, oc, on = orc.idw(og, small.x, small.y, small.z, small.radius, 3.0, 2, 8)
    z, c, nn, _ = got_small
    assert np.array_equal(c, oc)
    assert np.array_equal(nn, on)
    assert np.array_equal(np.isnan(z), np.isnan(oz))
    ok = ~np.isnan(oz)
    rel = np.abs(z[ok].astype(np.float64) - oz[ok]) / np.abs(oz[ok])
    assert rel.max() <= 1e-5


def test_noalloc_rejects_inputs_beyond_the_scratch(ag):
    big = workload_cfg2()
    grid = ag.auv_grid_create(big.grid)
    n = 3_000_000  # about 216 MB of bins on this grid: above the static limit
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = _outputs(ag, grid, x.device)
    p = ag.idw_params(radius=big.radius, max_pts=16)
    with pytest.raises(ag.AuvError) as e:
        ag.auv_grid_idw_noalloc(grid, x, x, x, 0, p, *out)
    assert e.value.status == ag.AUV_ERR_BUDGET
    assert int(torch.count_nonzero(out[1] != -7)) == 0  # nothing ran
