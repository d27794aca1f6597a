"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bar: bins, counts, NaN masks, nearest indices bit-exact; nearest depths equal
to the oracle depth rounded to float; IDW and bilinear values within 1e-5
relative of the oracle per node.
"""
import numpy as np
import pytest
import torch

from gen import small_swath, uniform_field, workload_cfg1, workload_cfg2

pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def ag():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22675_amd as ag
    ag.load_library()
    return ag


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _ogrid(orc, g):
    return orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def _assert_idw_equal(gz, gc, gn, gnz, oz, oc, on, z_src, label=""):
    gz = gz.astype(np.float64)
    assert np.array_equal(gc, oc), f"{label}: counts differ at {np.argwhere(gc != oc)[:5]}"
    nan_g, nan_o = np.isnan(gz), np.isnan(oz)
    assert np.array_equal(nan_g, nan_o), f"{label}: NaN masks differ"
    ok = ~nan_o
    err = np.abs(gz[ok] - oz[ok]) / np.maximum(np.abs(oz[ok]), 1e-30)
    assert err.size == 0 or err.max() <= REL, f"{label}: max rel err {err.max():.3e}"
    if gn is not None:
        assert np.array_equal(gn, on), f"{label}: nearest indices differ"
        have = on >= 0
        assert np.array_equal(gnz[have], z_src[on[have]].astype(np.float32))
        assert np.all(np.isnan(gnz[~have]))
    return err


def _run_idw(ag, s, bin_log2=0, max_pts=None, min_pts=None, power=None, radius=None,
             algo=0):
    grid = ag.auv_grid_create(s.grid)
    bins = ag.auv_bin_points(grid, _dev(s.x), _dev(s.y), _dev(s.z),
                             s.radius if radius is None else radius, bin_log2)
    out = ag.grid_idw(grid, bins, power=s.power if power is None else power,
                      min_pts=s.min_pts if min_pts is None else min_pts,
                      max_pts=s.max_pts if max_pts is None else max_pts,
                      with_counts=True, with_nearest=True, algo=algo)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, grid, bins


# ---------------------------------------------------------------- binning --

@pytest.mark.parametrize("bin_log2", [0, 16, 18, 20])
def test_binning_bit_exact(ag, orc, bin_log2):
    s = small_swath(nodes=200, pings=90, beams=80, n_lines=3, seed=51, x0=-300.0, y0=1200.0)
    x, y, z = s.x.copy(), s.y.copy(), s.z.copy()
    x[3], y[8], z[21] = np.nan, np.inf, -np.inf
    x[30] = 1e12
    grid = ag.auv_grid_create(s.grid)
    bins = ag.auv_bin_points(grid, _dev(x), _dev(y), _dev(z), s.radius, bin_log2)
    nbx, nby, halo, used = ag.auv_bins_info(bins)
    cs, perm, counts = ag.auv_bins_export(bins)
    og = _ogrid(orc, s.grid)
    ocs, operm, obad, oout = orc.bin_points(og, x, y, z, s.radius, used)
    assert (nbx, nby, halo) == orc.bin_dims(og, s.radius, used)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert counts == (operm.shape[0], obad, oout)


def test_binning_dense_bins_and_empty(ag, orc):
    # many soundings in few bins exercises the per-bin LDS ranking
    rng = np.random.default_rng(52)
    n = 60000
    x = rng.uniform(0, 20.0, n)
    y = rng.uniform(0, 20.0, n)
    z = -rng.uniform(100, 200, n)
    x[::7] = np.round(x[::7])                 # duplicates positions
    from gen import GridSpec
    g = GridSpec(0.0, 0.0, 1.0, 1.0, 20, 20)
    grid = ag.auv_grid_create(g)
    for b in (20, 22):
        bins = ag.auv_bin_points(grid, _dev(x), _dev(y), _dev(z), 2.0, b)
        cs, perm, counts = ag.auv_bins_export(bins)
        ocs, operm, _, _ = orc.bin_points(_ogrid(orc, g), x, y, z, 2.0, b)
        assert np.array_equal(cs.cpu().numpy(), ocs)
        assert np.array_equal(perm.cpu().numpy(), operm)
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    bins = ag.auv_bin_points(grid, empty, empty, empty, 2.0, 0)
    cs, perm, counts = ag.auv_bins_export(bins)
    assert counts == (0, 0, 0) and int(cs.abs().sum()) == 0
    out = ag.grid_idw(grid, bins, with_counts=True, with_nearest=True)
    torch.cuda.synchronize()
    assert torch.isnan(out["z"]).all() and int(out["cnt"].sum()) == 0
    assert bool((out["nn_idx"] == -1).all())


# -------------------------------------------------------------------- IDW --

def test_idw_cfg1_parity(ag, orc):
    s = workload_cfg1()
    res, grid, bins = _run_idw(ag, s)
    oz, oc, on = orc.idw(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, s.power,
                         s.min_pts, s.max_pts, bin_log2=20)
    err = _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on,
                            s.z, "cfg1")
    assert oc.mean() > 20 and err.size > 60000
    # nearest-neighbour grid through its own entry point
    idx = torch.empty((s.grid.ny, s.grid.nx), dtype=torch.int32, device="cuda")
    zz = torch.empty((s.grid.ny, s.grid.nx), dtype=torch.float32, device="cuda")
    ag.auv_interp_nearest(grid, bins, s.radius, idx, zz)
    oi, ozz = orc.nearest(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, bin_log2=20)
    assert np.array_equal(idx.cpu().numpy(), oi)
    have = oi >= 0
    assert np.array_equal(zz.cpu().numpy()[have], ozz[have].astype(np.float32))


@pytest.mark.parametrize("max_pts,min_pts,power,bin_log2", [
    (16, 1, 2.0, 0), (3, 2, 2.0, 18), (1, 1, 1.0, 19), (5, 0, 3.0, 17),
    (0, 4, 2.5, 0), (7, 1, 1.5, 20)])
def test_idw_swath_parity(ag, orc, max_pts, min_pts, power, bin_log2):
    s = small_swath(nodes=300, pings=140, beams=120, n_lines=4, seed=53, x0=5000.0, y0=-700.0)
    res, _, _ = _run_idw(ag, s, bin_log2=bin_log2, max_pts=max_pts, min_pts=min_pts,
                         power=power)
    oz, oc, on = orc.idw(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, power, min_pts,
                         max_pts, bin_log2=19)
    _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, s.z,
                      f"swath k={max_pts}")
    if max_pts:
        assert (oc == max_pts).sum() > 100  # the cap path was exercised


def test_idw_lattice_ties_and_caps(ag, orc):
    """Lattice-snapped soundings: equal distances, D^2 == R^2, coincident points
    and caps that cut through ties — the selection must match exactly."""
    from gen import GridSpec
    rng = np.random.default_rng(54)
    g = GridSpec(-3.0, 5.0, 0.5, 0.5, 61, 45)   # ragged tiles (61 x 45)
    n = 3000
    x = g.x0 + np.round(rng.uniform(-2, 33, n) * 4) / 4
    y = g.y0 + np.round(rng.uniform(-2, 25, n) * 4) / 4
    z = -np.round(rng.uniform(50, 80, n), 2)
    x[:300] = g.x0 + (rng.integers(0, 61, 300) + 0.5) * 0.5   # exactly on nodes
    y[:300] = g.y0 + (rng.integers(0, 45, 300) + 0.5) * 0.5
    for kcap, r in ((4, 1.0), (9, 1.25), (2, 0.75), (0, 1.0)):
        res, _, _ = _run_idw(ag, _with(g, x, y, z, r), max_pts=kcap, min_pts=2, power=2.0)
        oz, oc, on = orc.idw(_ogrid(orc, g), x, y, z, r, 2.0, 2, kcap, bin_log2=-1)
        _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, z,
                          f"ties k={kcap} r={r}")


def _with(g, x, y, z, r):
    from gen import Soundings
    return Soundings(x, y, z, g, radius=r)


def test_idw_general_power_and_far_origin(ag, orc):
    s = small_swath(nodes=160, pings=80, beams=64, n_lines=3, seed=55, x0=8000.0, y0=3000.0)
    for p in (0.5, 4.0, 7.25):
        res, _, _ = _run_idw(ag, s, power=p, max_pts=12)
        oz, oc, on = orc.idw(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, p, 1, 12,
                             bin_log2=19)
        _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on,
                          s.z, f"p={p}")


def test_idw_constant_field_and_hits(ag):
    x, y, z, g = uniform_field(n=5000, seed=56, extent=300.0, nodes=77)
    z = np.full_like(z, -3333.25)
    xs = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    x[:50] = xs[np.arange(50) % g.nx]
    y[:50] = g.y0 + 0.5 * g.dy
    from gen import Soundings
    res, _, _ = _run_idw(ag, Soundings(x, y, z, g, radius=8.0), min_pts=1, max_pts=0)
    ok = ~np.isnan(res["z"])
    assert ok.mean() > 0.9 and np.all(res["z"][ok] == np.float32(-3333.25))


def test_idw_deterministic(ag):
    s = small_swath(nodes=256, pings=120, beams=100, n_lines=3, seed=57)
    a, _, _ = _run_idw(ag, s)
    b, _, _ = _run_idw(ag, s)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True)


@pytest.fixture(scope="module")
def cfg2_run(ag):
    s = workload_cfg2()
    res, grid, bins = _run_idw(ag, s)
    return s, res, grid, bins


def _assert_within_bounds(z, lo, hi, label=""):
    """Every non-NaN output lies within [min, max] of its selected set's depths
    rounded to FP32 (the GPU clamps to the FP32 depths it holds); a node is
    NaN exactly where the oracle's set is empty or below min_pts."""
    z = z.astype(np.float32)
    ok = ~np.isnan(z)
    assert not np.isnan(lo[ok]).any(), f"{label}: value where the selected set is empty"
    flo, fhi = lo[ok].astype(np.float32), hi[ok].astype(np.float32)
    below = np.flatnonzero(z[ok] < flo)
    above = np.flatnonzero(z[ok] > fhi)
    assert below.size == 0 and above.size == 0, (
        f"{label}: {below.size} below / {above.size} above the selected depths")
    return int(ok.sum())


def test_cfg2_full_grid_parity(ag, orc, cfg2_run):
    """The headline workload at full size (2M soundings -> 4096^2, r=6, k=16),
    in the launch configuration the benchmark times, on every node: counts,
    NaN mask, nearest index and depth exact, IDW within 1e-5, and every value
    within its selected depths."""
    s, res, grid, bins = cfg2_run
    og = _ogrid(orc, s.grid)
    oz, oc, on = orc.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts,
                         bin_log2=19)
    _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, s.z,
                      "cfg2 full grid")
    lo, hi = orc.idw_bounds(og, s.x, s.y, s.z, s.radius, s.max_pts, bin_log2=19)
    assert _assert_within_bounds(res["z"], lo, hi, "cfg2") > 0.75 * oz.size
    assert np.all(res["cnt"] <= 16)


def test_idw_span_form_parity(ag, orc, cfg2_run):
    """The span form (AUV_ALGO_SPAN) against the oracle: cfg1 (no cap, about 25
    members per node), swaths with caps that bind and integer powers 1..3,
    lattice-snapped ties and hits on a ragged grid, and every node of cfg2."""
    from gen import GridSpec
    span = ag.AUV_ALGO_SPAN
    s = workload_cfg1()
    res, _, _ = _run_idw(ag, s, algo=span)
    oz, oc, on = orc.idw(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, s.power, s.min_pts,
                         s.max_pts, bin_log2=20)
    _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, s.z,
                      "span cfg1")
    s = small_swath(nodes=300, pings=140, beams=120, n_lines=4, seed=53, x0=5000.0, y0=-700.0)
    for kcap, power in ((16, 2.0), (3, 1.0), (0, 3.0)):
        res, _, _ = _run_idw(ag, s, max_pts=kcap, power=power, algo=span)
        oz, oc, on = orc.idw(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, power, 1, kcap,
                             bin_log2=19)
        _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, s.z,
                          f"span swath k={kcap} p={power}")
    rng = np.random.default_rng(54)
    g = GridSpec(-3.0, 5.0, 0.5, 0.5, 61, 45)
    n = 3000
    x = g.x0 + np.round(rng.uniform(-2, 33, n) * 4) / 4
    y = g.y0 + np.round(rng.uniform(-2, 25, n) * 4) / 4
    z = -np.round(rng.uniform(50, 80, n), 2)
    x[:300] = g.x0 + (rng.integers(0, 61, 300) + 0.5) * 0.5
    y[:300] = g.y0 + (rng.integers(0, 45, 300) + 0.5) * 0.5
    for kcap, r in ((4, 1.0), (0, 1.25)):
        res, _, _ = _run_idw(ag, _with(g, x, y, z, r), max_pts=kcap, min_pts=2, power=2.0,
                             algo=span)
        oz, oc, on = orc.idw(_ogrid(orc, g), x, y, z, r, 2.0, 2, kcap, bin_log2=-1)
        _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, z,
                          f"span ties k={kcap} r={r}")
    s, _, grid, bins = cfg2_run
    out = ag.grid_idw(grid, bins, power=s.power, min_pts=s.min_pts, max_pts=s.max_pts,
                      with_counts=True, with_nearest=True, algo=span)
    torch.cuda.synchronize()
    og = _ogrid(orc, s.grid)
    oz, oc, on = orc.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts,
                         bin_log2=19)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, s.z,
                      "span cfg2 full grid")
    lo, hi = orc.idw_bounds(og, s.x, s.y, s.z, s.radius, s.max_pts, bin_log2=19)
    _assert_within_bounds(res["z"], lo, hi, "span cfg2")


def test_cfg4_exact_path_full_size(ag, orc):
    """cfg2's soundings at UTM-scale coordinates (easting 5e5, northing 4e6,
    float64 input): the FP64-rebase path keeps the exact contract on every node
    (counts, NaN mask, nearest picks exact; values within 1e-5 relative)."""
    from gen import workload_cfg4
    s = workload_cfg4()
    res, grid, bins = _run_idw(ag, s)
    og = _ogrid(orc, s.grid)
    oz, oc, on = orc.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts,
                         bin_log2=19)
    err = _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, s.z,
                            "cfg4 exact path")
    assert err.size > 0.75 * oz.size
    lo, hi = orc.idw_bounds(og, s.x, s.y, s.z, s.radius, s.max_pts, bin_log2=19)
    _assert_within_bounds(res["z"], lo, hi, "cfg4")


@pytest.mark.parametrize("case", ["cfg1", "capped", "dense", "hits"])
def test_idw_values_within_selected_depths(ag, orc, case):
    """The clamp of the definition (every value within [min, max] of its
    selected set), on the window form with no cap (cfg1), with a cap that binds
    (the exact per-node path), on the dense form, and with lattice-snapped
    soundings that sit on nodes (hits)."""
    from gen import GridSpec, Soundings
    if case == "cfg1":
        s = workload_cfg1()
        algo = ag.AUV_ALGO_AUTO
    else:
        rng = np.random.default_rng({"capped": 81, "dense": 82, "hits": 83}[case])
        g = GridSpec(250.0, -40.0, 2.0, 2.0, 90, 75)
        n = {"capped": 30000, "dense": 30000, "hits": 6000}[case]
        x = g.x0 + rng.uniform(-6, 186, n)
        y = g.y0 + rng.uniform(-6, 156, n)
        if case == "hits":
            x = g.x0 + np.round((x - g.x0) / 0.5) * 0.5 + 0.0
            y = g.y0 + np.round((y - g.y0) / 0.5) * 0.5 + 0.0
        # a rough field: neighbouring depths differ a lot, so the weighted
        # mean is often close to one of them
        z = -4000.0 + 300.0 * rng.standard_normal(n) * (rng.random(n) < 0.3)
        s = Soundings(x, y, z, g, radius=6.0, power=2.0, min_pts=1,
                      max_pts=0 if case == "hits" else 12)
        algo = ag.AUV_ALGO_DENSE if case == "dense" else ag.AUV_ALGO_SPARSE
    grid = ag.auv_grid_create(s.grid)
    bins = ag.auv_bin_points(grid, _dev(s.x), _dev(s.y), _dev(s.z), s.radius, 0)
    out = ag.grid_idw(grid, bins, power=s.power, min_pts=s.min_pts, max_pts=s.max_pts,
                      with_counts=True, with_nearest=True, algo=algo)
    torch.cuda.synchronize()
    og = _ogrid(orc, s.grid)
    oz, oc, on = orc.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts,
                         bin_log2=17)
    _assert_idw_equal(out["z"].cpu().numpy(), out["cnt"].cpu().numpy(),
                      out["nn_idx"].cpu().numpy(), out["nn_z"].cpu().numpy(), oz, oc, on, s.z,
                      case)
    lo, hi = orc.idw_bounds(og, s.x, s.y, s.z, s.radius, s.max_pts, bin_log2=17)
    gz = out["z"].cpu().numpy()
    # min_pts = 1 here, so the value is NaN exactly where the selected set is empty
    assert np.array_equal(np.isnan(gz), np.isnan(lo))
    assert _assert_within_bounds(gz, lo, hi, case) > 0


def test_cfg2_binning_counts(ag, orc, cfg2_run):
    s, res, grid, bins = cfg2_run
    cs, perm, counts = ag.auv_bins_export(bins)
    ocs, operm, obad, oout = orc.bin_points(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius,
                                            ag.auv_bins_info(bins)[3])
    assert counts == (operm.shape[0], obad, oout)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    assert np.array_equal(perm.cpu().numpy(), operm)


# --------------------------------------------------------------- bilinear --

@pytest.mark.parametrize("src_shape,dst_shape,nan_frac", [
    ((64, 64), (128, 128), 0.0), ((97, 45), (194, 90), 0.02),
    ((50, 70), (33, 101), 0.05), ((1, 7), (3, 15), 0.0), ((33, 33), (33, 33), 0.1),
    # strong downsampling: a patch's source rectangle exceeds the LDS stage
    # and corners are read from global memory
    ((120, 4000), (30, 1100), 0.02),
    # large enough for several row groups per block (four here): 875 row
    # groups of 8 do not divide into fours and the last group has 7 rows
    ((3500, 2500), (6999, 5000), 0.01)])
def test_bilinear_parity(ag, orc, src_shape, dst_shape, nan_frac):
    sh, sw = src_shape
    dh, dw = dst_shape
    rng = np.random.default_rng(sh * 1000 + dw)
    v = (-5000.0 + rng.normal(0, 400.0, (sh, sw))).astype(np.float32)
    if nan_frac:
        v[rng.random((sh, sw)) < nan_frac] = np.nan
    from gen import GridSpec
    sg = GridSpec(1000.0, 2000.0, 2.0, 3.0, sw, sh)
    dg = GridSpec(1000.0, 2000.0, 2.0 * sw / dw, 3.0 * sh / dh, dw, dh)
    src = torch.from_numpy(v).cuda()
    dst = torch.empty((dh, dw), dtype=torch.float32, device="cuda")
    ag.auv_resample_bilinear(src, sg, dst, dg)
    torch.cuda.synchronize()
    ref = orc.bilinear(_ogrid(orc, sg), v.astype(np.float64), _ogrid(orc, dg))
    out = dst.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(out), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.max(np.abs(out[ok] - ref[ok]) / np.abs(ref[ok])) <= REL


def _full_resample_check(out, ref, label):
    assert np.array_equal(np.isnan(out), np.isnan(ref)), f"{label}: NaN masks differ"
    ok = ~np.isnan(ref)
    o = out[ok].astype(np.float64)
    r = ref[ok]
    err = np.abs(o - r) / np.abs(r)
    assert err.max() <= REL, f"{label}: max rel err {err.max():.3e}"
    return int(ok.sum())


def test_bilinear_cfg2_upsample(ag, orc, cfg2_run):
    """2x resample of the full cfg2 IDW grid to 8192^2 at 1 m, every one of the
    67.1M destination nodes against the oracle (holes included)."""
    s, res, grid, bins = cfg2_run
    from gen import GridSpec
    sg = s.grid
    dg = GridSpec(0.0, 0.0, 1.0, 1.0, 8192, 8192)
    src = torch.from_numpy(res["z"]).cuda()
    dst = torch.empty((8192, 8192), dtype=torch.float32, device="cuda")
    ag.auv_resample_bilinear(src, sg, dst, dg)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    del dst
    ref = orc.bilinear(_ogrid(orc, sg), res["z"].astype(np.float64), _ogrid(orc, dg))
    n = _full_resample_check(out, ref, "bilinear cfg2 2x")
    assert 0.5 * out.size < n < out.size


# ---------------------------------------------------------------- bicubic --

@pytest.mark.parametrize("src_shape,dst_shape,nan_frac", [
    ((64, 64), (128, 128), 0.0), ((97, 45), (194, 90), 0.02),
    ((50, 70), (33, 101), 0.05), ((1, 7), (3, 15), 0.0), ((2, 3), (5, 9), 0.0),
    ((33, 33), (33, 33), 0.1), ((300, 1100), (600, 2200), 0.01),
    ((120, 4000), (30, 1100), 0.02)])   # taps from global memory (no LDS stage)
def test_bicubic_parity(ag, orc, src_shape, dst_shape, nan_frac):
    sh, sw = src_shape
    dh, dw = dst_shape
    rng = np.random.default_rng(sh * 1000 + dw + 7)
    v = (-5000.0 + rng.normal(0, 400.0, (sh, sw))).astype(np.float32)
    if nan_frac:
        v[rng.random((sh, sw)) < nan_frac] = np.nan
    from gen import GridSpec
    sg = GridSpec(1000.0, 2000.0, 2.0, 3.0, sw, sh)
    dg = GridSpec(1000.0, 2000.0, 2.0 * sw / dw, 3.0 * sh / dh, dw, dh)
    src = torch.from_numpy(v).cuda()
    dst = torch.empty((dh, dw), dtype=torch.float32, device="cuda")
    ag.auv_resample_bicubic(src, sg, dst, dg)
    torch.cuda.synchronize()
    ref = orc.bicubic(_ogrid(orc, sg), v.astype(np.float64), _ogrid(orc, dg))
    out = dst.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(out), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.max(np.abs(out[ok] - ref[ok]) / np.abs(ref[ok])) <= REL


def test_bicubic_cfg2_upsample(ag, orc, cfg2_run):
    """2x Catmull-Rom resample of the full cfg2 IDW grid (holes included) to
    8192^2 at 1 m, every destination node against the oracle."""
    s, res, grid, bins = cfg2_run
    from gen import GridSpec
    sg = s.grid
    dg = GridSpec(0.0, 0.0, 1.0, 1.0, 8192, 8192)
    src = torch.from_numpy(res["z"]).cuda()
    dst = torch.empty((8192, 8192), dtype=torch.float32, device="cuda")
    ag.auv_resample_bicubic(src, sg, dst, dg)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    del dst
    ref = orc.bicubic(_ogrid(orc, sg), res["z"].astype(np.float64), _ogrid(orc, dg))
    n = _full_resample_check(out, ref, "Catmull-Rom cfg2 2x")
    # the fallback to bilinear next to holes happens (more NaN-free nodes than
    # a strict 16-tap rule would leave)
    bil = orc.bilinear(_ogrid(orc, sg), res["z"].astype(np.float64), _ogrid(orc, dg))
    assert np.array_equal(np.isnan(ref), np.isnan(bil)) and n < out.size


# ------------------------------------------------------- dispatch branches --

@pytest.mark.parametrize("dx,radius,kcap", [
    (1000.0 / 255.0, 9.0, 0),    # node lattice not linear -> tile kernel
    (0.5, 3.9, 6),               # 16 x 16 window, four lane chunks
    (0.25, 6.0, 9),              # window too wide -> tile kernel
    (3.90625, 20.0, 0),          # 11 x 11 window, two lane chunks
])
def test_idw_dispatch_branches(ag, orc, dx, radius, kcap):
    from gen import GridSpec, Soundings
    nodes = int(min(300, 160.0 / dx))
    rng = np.random.default_rng(int(dx * 1000) + int(radius))
    ext = nodes * dx
    n = int(ext * ext * 0.08) + 500
    x = rng.uniform(-radius, ext + radius, n) + 123.0
    y = rng.uniform(-radius, ext + radius, n) - 45.0
    z = -4000.0 - 50.0 * np.sin(x / 37.0) + rng.normal(0, 2.0, n)
    g = GridSpec(123.0, -45.0, dx, dx, nodes, nodes - 3)
    s = Soundings(x, y, z, g, radius=radius, power=2.0, min_pts=2, max_pts=kcap)
    res, _, _ = _run_idw(ag, s)
    oz, oc, on = orc.idw(_ogrid(orc, g), x, y, z, radius, 2.0, 2, kcap,
                         bin_log2=18 if radius < 10 else 20)
    _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, z,
                      f"dx={dx} r={radius}")


def test_binning_many_rows_fallback(ag, orc):
    """More than 8192 bin rows takes the per-sounding atomic counting sort."""
    x, y, z, g = uniform_field(n=30000, seed=59, extent=700.0, nodes=175)
    grid = ag.auv_grid_create(g)
    bins = ag.auv_bin_points(grid, _dev(x), _dev(y), _dev(z), 1.0, 12)
    nbx, nby, halo, used = ag.auv_bins_info(bins)
    assert nby > 8192
    cs, perm, counts = ag.auv_bins_export(bins)
    ocs, operm, _, _ = orc.bin_points(_ogrid(orc, g), x, y, z, 1.0, 12)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    assert np.array_equal(perm.cpu().numpy(), operm)
    out = ag.grid_idw(grid, bins, power=2.0, radius=1.0, with_counts=True, with_nearest=True)
    torch.cuda.synchronize()
    oz, oc, on = orc.idw(_ogrid(orc, g), x, y, z, 1.0, 2.0, 1, 0, bin_log2=16)
    _assert_idw_equal(out["z"].cpu().numpy(), out["cnt"].cpu().numpy(),
                      out["nn_idx"].cpu().numpy(), out["nn_z"].cpu().numpy(), oz, oc, on, z,
                      "fallback bins")


# ----------------------------------------------------- precision variants --

def _variant_errors(ag, orc, s, precision):
    grid = ag.auv_grid_create(s.grid)
    bins = ag.auv_bin_points(grid, _dev(s.x), _dev(s.y), _dev(s.z), s.radius, 0)
    out = ag.grid_idw(grid, bins, power=s.power, min_pts=s.min_pts, max_pts=s.max_pts,
                      with_counts=True, precision=precision)
    torch.cuda.synchronize()
    gz = out["z"].cpu().numpy().astype(np.float64)
    oz, oc, on = orc.idw(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, s.power, s.min_pts,
                         s.max_pts, bin_log2=19)
    both = ~np.isnan(gz) & ~np.isnan(oz)
    err = np.abs(gz[both] - oz[both])
    return {"max_abs": float(err.max()), "max_rel": float((err / np.abs(oz[both])).max()),
            "nan_mismatch": int((np.isnan(gz) != np.isnan(oz)).sum()),
            "count_mismatch": int((out["cnt"].cpu().numpy() != oc).sum()), "n": int(both.sum())}


def test_precision_variants_at_utm_scale(ag, orc):
    """cfg4-style input: absolute UTM-like coordinates (easting ~5e5, northing
    ~4e6).  The FP64-rebase path keeps the exact contract; the FP16-offset and
    FP32-absolute variants are measured against the oracle."""
    s = small_swath(nodes=256, pings=120, beams=100, n_lines=3, seed=60,
                    x0=500000.0, y0=4000000.0, max_pts=16)
    exact = _variant_errors(ag, orc, s, ag.AUV_P_FP32_REBASE)
    assert exact["max_rel"] <= 1e-5 and exact["nan_mismatch"] == 0
    assert exact["count_mismatch"] == 0
    fp16 = _variant_errors(ag, orc, s, ag.AUV_P_FP16_OFFSETS)
    fp32abs = _variant_errors(ag, orc, s, ag.AUV_P_FP32_ABSOLUTE)
    print("precision errors", exact, fp16, fp32abs)
    # FP16 offsets (tiles of 32 m): ~1 cm position error, close to the oracle
    assert fp16["max_abs"] < 5.0 and fp16["n"] > 0.9 * exact["n"]
    # FP32 absolute: 0.25-0.5 m coordinate ulps, gross but bounded errors
    assert fp32abs["n"] > 0.8 * exact["n"]
    assert fp32abs["count_mismatch"] > fp16["count_mismatch"]


# ------------------------------------------------------------- dense form --

@pytest.mark.parametrize("kcap,power,min_pts,snap,bin_log2", [
    (16, 2.0, 1, 0.0, 15), (16, 1.0, 3, 0.0, 0), (32, 3.0, 1, 0.0, 15),
    (5, 2.5, 2, 0.25, 14), (1, 2.0, 1, 0.125, 15)])
def test_idw_dense_form_parity(ag, orc, kcap, power, min_pts, snap, bin_log2):
    """Dense soundings (hundreds per disk) with a small cap: the ring-search
    top-k form must select exactly the oracle's k nearest (ties included)."""
    from gen import GridSpec, Soundings
    rng = np.random.default_rng(61 + kcap)
    g = GridSpec(3000.0, -2000.0, 2.0, 2.0, 70, 45)     # ragged 8x8 tiles
    n = 40000
    x = g.x0 + rng.uniform(-6, 146, n)
    y = g.y0 + rng.uniform(-6, 96, n)
    if snap:
        x = g.x0 + np.round((x - g.x0) / snap) * snap
        y = g.y0 + np.round((y - g.y0) / snap) * snap
    z = -4500.0 + 30.0 * np.sin((x - g.x0) / 17.0) + rng.normal(0, 5.0, n)
    s = Soundings(x, y, z, g, radius=6.0, power=power, min_pts=min_pts, max_pts=kcap)
    grid = ag.auv_grid_create(g)
    bins = ag.auv_bin_points(grid, _dev(x), _dev(y), _dev(z), 6.0, bin_log2)
    out = ag.grid_idw(grid, bins, power=power, min_pts=min_pts, max_pts=kcap,
                      with_counts=True, with_nearest=True, algo=ag.AUV_ALGO_DENSE)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    oz, oc, on = orc.idw(_ogrid(orc, g), x, y, z, 6.0, power, min_pts, kcap, bin_log2=18)
    _assert_idw_equal(res["z"], res["cnt"], res["nn_idx"], res["nn_z"], oz, oc, on, z,
                      f"dense k={kcap}")
    assert (oc == kcap).mean() > 0.95
    # the sparse form (window + exact per-node selection) gives the same result
    out2 = ag.grid_idw(grid, bins, power=power, min_pts=min_pts, max_pts=kcap,
                       with_counts=True, with_nearest=True, algo=ag.AUV_ALGO_SPARSE)
    torch.cuda.synchronize()
    _assert_idw_equal(out2["z"].cpu().numpy(), out2["cnt"].cpu().numpy(),
                      out2["nn_idx"].cpu().numpy(), out2["nn_z"].cpu().numpy(), oz, oc, on, z,
                      f"sparse on dense k={kcap}")


# ------------------------------------------------------------------ kriging --

@pytest.mark.parametrize("src_shape,dst_shape,range_cells,nan_frac", [
    ((37, 53), (74, 106), 3.0, 0.0),     # 2x upsample, several blocks and a ragged tail
    ((64, 300), (21, 97), 0.5, 0.0),     # downsample: source patch not staged
    ((40, 40), (160, 160), 10.0, 0.02),  # holes: windows with NaN fall back to bilinear
    ((5, 5), (13, 11), 2.0, 0.0),        # the smallest grid with a 5 x 5 window
    ((9, 600), (9, 1300), 1.0, 0.0),     # wide and flat: many column blocks
    ((30, 40), (90, 70), 20.0, 0.0),     # longest range of the exp form
    ((30, 40), (90, 70), 60.0, 0.0),     # series form of 1 - exp(-t)
    ((24, 24), (61, 47), 1000.0, 0.01),  # very long range, holes
    ((12, 12), (20, 20), 9000.0, 0.0),   # near the range limit
    ((5, 40), (11, 90), 2.0, 0.0),       # exactly five rows: every window the same rows
    ((40, 5), (70, 9), 2.0, 0.05),       # exactly five columns, holes
])
def test_kriging_parity(ag, orc, src_shape, dst_shape, range_cells, nan_frac):
    sh, sw = src_shape
    dh, dw = dst_shape
    rng = np.random.default_rng(sh * 7919 + dw * 31 + int(range_cells * 10))
    v = (-5000.0 + rng.normal(0, 400.0, (sh, sw))).astype(np.float32)
    if nan_frac:
        v[rng.random((sh, sw)) < nan_frac] = np.nan
    from gen import GridSpec
    sg = GridSpec(1000.0, 2000.0, 2.0, 3.0, sw, sh)
    dg = GridSpec(1000.0, 2000.0, 2.0 * sw / dw, 3.0 * sh / dh, dw, dh)
    rng_m = range_cells * 2.0
    src = torch.from_numpy(v).cuda()
    dst = torch.empty((dh, dw), dtype=torch.float32, device="cuda")
    ag.auv_resample_kriging(src, sg, dst, dg, rng_m)
    torch.cuda.synchronize()
    ref = orc.kriging(_ogrid(orc, sg), v.astype(np.float64), _ogrid(orc, dg), rng_m)
    out = dst.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(out), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.max(np.abs(out[ok] - ref[ok]) / np.abs(ref[ok])) <= REL


def test_kriging_small_grid_is_bilinear(ag):
    """A source grid under 5 x 5 has no kriging window: the entry point gives
    exactly the bilinear resample."""
    from gen import GridSpec
    rng = np.random.default_rng(5)
    v = (-100.0 + rng.normal(0, 5.0, (4, 9))).astype(np.float32)
    sg = GridSpec(0.0, 0.0, 1.0, 1.0, 9, 4)
    dg = GridSpec(0.0, 0.0, 0.5, 0.5, 18, 8)
    src = torch.from_numpy(v).cuda()
    a = torch.empty((8, 18), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ag.auv_resample_kriging(src, sg, a, dg, 3.0)
    ag.auv_resample_bilinear(src, sg, b, dg)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_kriging_rejects_bad_range(ag):
    from gen import GridSpec
    g = GridSpec(0.0, 0.0, 1.0, 1.0, 8, 8)
    src = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for r in (0.0, -1.0, float("nan"), float("inf"), 2e4):
        with pytest.raises(ag.AuvError):
            ag.auv_resample_kriging(src, g, dst, g, r)


@pytest.mark.parametrize("range_cells", [3.0, 1000.0])
def test_kriging_ragged_tall_blocks(ag, orc, range_cells):
    """2x kriging of a 2048 x 1100 grid to 4096 x 2200: enough blocks for 32
    rows per block, so the last block holds 24 rows; sampled rows (the last
    26, the first 4, a few inside) against the oracle on a band of source rows
    that holds each row's windows without moving them.  The long range takes
    the series form of the covariance terms."""
    from gen import GridSpec
    sh, sw = 1100, 2048
    rng = np.random.default_rng(int(range_cells))
    v = (-5000.0 + rng.normal(0, 400.0, (sh, sw))).astype(np.float32)
    v[rng.random((sh, sw)) < 0.002] = np.nan
    sg = GridSpec(1000.0, 2000.0, 2.0, 2.0, sw, sh)
    dg = GridSpec(1000.0, 2000.0, 1.0, 1.0, 2 * sw, 2 * sh)
    rng_m = range_cells * sg.dx
    src = torch.from_numpy(v).cuda()
    dst = torch.empty((dg.ny, dg.nx), dtype=torch.float32, device="cuda")
    ag.auv_resample_kriging(src, sg, dst, dg, rng_m)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    rows = list(range(dg.ny - 26, dg.ny)) + [0, 1, 2, 3, 31, 32, 33, 1000, 1601]
    for r in rows:
        band_lo = max(0, r // 2 - 4)
        band_hi = min(sh, r // 2 + 5)
        sub = GridSpec(sg.x0, sg.y0 + band_lo * sg.dy, sg.dx, sg.dy, sw, band_hi - band_lo)
        drow = GridSpec(dg.x0, dg.y0 + float(r), 1.0, 1.0, dg.nx, 1)
        ref = orc.kriging(_ogrid(orc, sub), v[band_lo:band_hi].astype(np.float64),
                          _ogrid(orc, drow), rng_m)[0]
        o = out[r].astype(np.float64)
        assert np.array_equal(np.isnan(o), np.isnan(ref)), f"row {r}"
        ok = ~np.isnan(ref)
        assert np.max(np.abs(o[ok] - ref[ok]) / np.abs(ref[ok])) <= REL, f"row {r}"


def test_kriging_cfg2_upsample(ag, orc, cfg2_run):
    """2x kriging resample of the full cfg2 IDW grid (holes included) to
    8192^2 at 1 m, checked on 320 whole destination rows (ten blocks of 32,
    the first and last rows of the grid included) against the oracle on a band
    of source rows that holds every window of the block without moving it."""
    s, res, grid, bins = cfg2_run
    from gen import GridSpec
    sg = s.grid
    dg = GridSpec(0.0, 0.0, 1.0, 1.0, 8192, 8192)
    rng_m = 3.0 * sg.dx
    src = torch.from_numpy(res["z"]).cuda()
    dst = torch.empty((8192, 8192), dtype=torch.float32, device="cuda")
    ag.auv_resample_kriging(src, sg, dst, dg, rng_m)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    del dst
    fallbacks = 0
    rows = 0
    for r0 in [0, 819, 1650, 2477, 3290, 4080, 4919, 5731, 6555, 8160]:
        r1 = min(8192, r0 + 32)
        band_lo = max(0, r0 // 2 - 4)
        band_hi = min(4096, (r1 - 1) // 2 + 5)
        sub = GridSpec(sg.x0, sg.y0 + band_lo * sg.dy, sg.dx, sg.dy, sg.nx, band_hi - band_lo)
        blk = GridSpec(0.0, float(r0), 1.0, 1.0, 8192, r1 - r0)
        ref = orc.kriging(_ogrid(orc, sub), res["z"][band_lo:band_hi].astype(np.float64),
                          _ogrid(orc, blk), rng_m)
        _full_resample_check(out[r0:r1], ref, f"kriging rows {r0}..{r1}")
        fallbacks += int(np.isnan(res["z"][band_lo:band_hi]).any())
        rows += r1 - r0
    assert fallbacks > 0 and rows >= 256
