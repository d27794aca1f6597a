"""GPU tests of the serving path: resident per-vehicle IDW sums updated by
request streams, through the C ABI.

Bar: after any set of requests a vehicle's read-out equals the oracle's IDW
(no cap) on the union of that vehicle's soundings -- counts and NaN masks
exact, depths within 1e-5 relative; a vehicle's grid is bit-identical whether
its requests ran FIFO, continuously batched with other vehicles, or alone.
"""
import numpy as np
import pytest
import torch

from gen import GridSpec, serving_schedule

pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def ag():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22675_amd as ag
    ag.load_library()
    return ag


def _small_schedule():
    grids, reqs = serving_schedule(n_vehicles=3, duration=1.5, rate_hz=12.0, n_lo=300,
                                   n_hi=4000, seed=55, nodes=256, dx=2.0, beams=100,
                                   altitude=60.0, line_spacing=128.0, ping_spacing=2.0)
    reqs = list(reqs)
    # edge cases: an empty request, invalid soundings, soundings off the grid,
    # soundings exactly on nodes (hits) in two different requests
    v = reqs[0].vehicle
    g = grids[v]
    reqs.append(type(reqs[0])(v, 0.0, np.zeros(0), np.zeros(0), np.zeros(0)))
    bad = reqs[1]
    x, y, z = bad.x.copy(), bad.y.copy(), bad.z.copy()
    x[::97] = np.nan
    z[5::89] = np.inf
    x[3::50] = g.x0 - 3.0            # left of the grid, within the radius
    y[7::50] = g.y0 + g.ny * g.dy + 50.0   # far above the grid: dropped
    reqs.append(type(reqs[0])(bad.vehicle, 0.0, x, y, z))
    for k in range(2):
        nx = g.x0 + (np.array([10, 11, 40]) + 0.5) * g.dx
        ny = g.y0 + (np.array([20, 20, 33]) + 0.5) * g.dy
        reqs.append(type(reqs[0])(v, 0.0, nx, ny, np.array([-100.0 - k, -50.0, -75.0 + k])))
    return grids, reqs


def _ogrid(orc, g):
    return orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def _run(ag, grids, reqs, mode, max_batch=0, vehicles=None, arena_extra=0, min_pts=1,
         max_request=None):
    mr = max_request or max(1, max(len(r.x) for r in reqs))
    desc = ag.session_desc(grids, power=2.0, radius=6.0, min_pts=min_pts, max_request=mr,
                           slots=8, mode=mode, max_batch=max_batch,
                           z_ref=[-3000.0] * len(grids))
    fixed, per_v = ag.auv_session_budget(desc)
    arena = torch.empty(fixed + len(grids) * per_v + arena_extra, dtype=torch.uint8,
                        device="cuda")
    s = ag.Session(desc, arena)
    tickets = []
    for r in reqs:
        if vehicles is not None and r.vehicle not in vehicles:
            continue
        tickets.append(s.submit(r.vehicle, r.x, r.y, r.z))
    s.drain()
    out = {}
    for v in range(len(grids)):
        if vehicles is not None and v not in vehicles:
            continue
        z, c = s.read_grid(v)
        torch.cuda.synchronize()
        out[v] = (z.cpu().numpy(), c.cpu().numpy())
    infos = [s.poll(t) for t in tickets]
    s.close()
    return out, infos


def _union(reqs, v):
    xs = [r.x for r in reqs if r.vehicle == v]
    if not xs:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    return (np.concatenate(xs), np.concatenate([r.y for r in reqs if r.vehicle == v]),
            np.concatenate([r.z for r in reqs if r.vehicle == v]))


def _check(orc, g, reqs, v, z, c, min_pts=1, label=""):
    x, y, zz = _union(reqs, v)
    oz, oc, _ = orc.idw(_ogrid(orc, g), x, y, zz, 6.0, 2.0, min_pts, 0, bin_log2=16)
    bad = np.argwhere(c != oc)
    assert bad.size == 0, f"{label}: counts differ at {bad[:5]}"
    gz = z.astype(np.float64)
    assert np.array_equal(np.isnan(gz), np.isnan(oz)), f"{label}: NaN masks differ"
    ok = ~np.isnan(oz)
    err = np.abs(gz[ok] - oz[ok]) / np.abs(oz[ok])
    assert err.size == 0 or err.max() <= REL, f"{label}: max rel err {err.max():.3e}"
    return int(ok.sum())


@pytest.mark.parametrize("mode", [0, 1])
def test_serving_matches_oracle_on_union(ag, orc, mode):
    grids, reqs = _small_schedule()
    out, infos = _run(ag, grids, reqs, mode)
    assert all(i.state == ag.AUV_T_DONE for i in infos)
    assert all(i.t_done >= i.t_launch >= i.t_arrival - 1e-3 for i in infos if i.n > 0)
    filled = 0
    for v, g in enumerate(grids):
        filled += _check(orc, g, reqs, v, *out[v], label=f"mode {mode} vehicle {v}")
    assert filled > 1000
    for v, g in enumerate(grids):
        x, y, zz = _union(reqs, v)
        lo, hi = orc.idw_bounds(_ogrid(orc, g), x, y, zz, 6.0, 0, bin_log2=16)
        z = out[v][0]
        ok = ~np.isnan(z)
        assert np.all(z[ok] >= lo[ok].astype(np.float32))
        assert np.all(z[ok] <= hi[ok].astype(np.float32))
    # the planted hits read out as the mean of the coincident soundings
    g, v = grids[reqs[0].vehicle], reqs[0].vehicle
    z = out[v][0]
    assert abs(z[20, 10] - np.mean([-100.0, -101.0])) <= REL * 100.5
    assert abs(z[33, 40] - np.mean([-75.0, -74.0])) <= REL * 74.5


def test_serving_fifo_batched_alone_bit_identical(ag):
    grids, reqs = _small_schedule()
    fifo, _ = _run(ag, grids, reqs, ag.AUV_SERVE_FIFO)
    batched, _ = _run(ag, grids, reqs, ag.AUV_SERVE_BATCHED)
    small_batches, _ = _run(ag, grids, reqs, ag.AUV_SERVE_BATCHED, max_batch=2)
    for v in range(len(grids)):
        alone, _ = _run(ag, grids, reqs, ag.AUV_SERVE_BATCHED, vehicles={v})
        for other in (batched, small_batches, alone):
            assert np.array_equal(fifo[v][0], other[v][0], equal_nan=True), f"vehicle {v} z"
            assert np.array_equal(fifo[v][1], other[v][1]), f"vehicle {v} counts"


def test_serving_min_pts_holes(ag, orc):
    grids, reqs = _small_schedule()
    out, _ = _run(ag, grids, reqs, ag.AUV_SERVE_BATCHED, min_pts=4)
    for v, g in enumerate(grids):
        _check(orc, g, reqs, v, *out[v], min_pts=4, label=f"min_pts 4 vehicle {v}")


def test_serving_admission_and_retire(ag, orc):
    grids, reqs = _small_schedule()
    desc = ag.session_desc(grids, max_request=5000, slots=4, mode=ag.AUV_SERVE_BATCHED)
    fixed, per_v = ag.auv_session_budget(desc)
    # room for the fixed part and two vehicles only
    arena = torch.empty(fixed + 2 * per_v + 100, dtype=torch.uint8, device="cuda")
    with pytest.raises(ag.AuvError) as e:
        ag.Session(desc, arena[: fixed - 256])
    assert e.value.status == ag.AUV_ERR_BUDGET
    s = ag.Session(desc, arena)
    by_v = {v: [r for r in reqs if r.vehicle == v and len(r.x) > 0] for v in range(3)}
    s.submit(0, by_v[0][0].x, by_v[0][0].y, by_v[0][0].z)
    s.submit(1, by_v[1][0].x, by_v[1][0].y, by_v[1][0].z)
    with pytest.raises(ag.AuvError) as e:
        s.submit(2, by_v[2][0].x, by_v[2][0].y, by_v[2][0].z)
    assert e.value.status == ag.AUV_ERR_BUDGET
    with pytest.raises(ag.AuvError) as e:
        s.submit(0, np.zeros(5001), np.zeros(5001), np.zeros(5001))
    assert e.value.status == ag.AUV_ERR_INVALID
    s.retire(0)
    with pytest.raises(ag.AuvError) as e:
        s.read_grid(0)
    assert e.value.status == ag.AUV_ERR_STATE
    # vehicle 2 takes vehicle 0's place and starts empty
    r2 = by_v[2][0]
    s.submit(2, r2.x, r2.y, r2.z)
    s.drain()
    z, c = s.read_grid(2)
    torch.cuda.synchronize()
    one = [r2]
    _check(orc, grids[2], one, 2, z.cpu().numpy(), c.cpu().numpy(), label="admitted after retire")
    # vehicle 0 comes back empty after vehicle 1 leaves
    s.retire(1)
    r0 = by_v[0][1]
    s.submit(0, r0.x, r0.y, r0.z)
    s.drain()
    z, c = s.read_grid(0)
    torch.cuda.synchronize()
    _check(orc, grids[0], [r0], 0, z.cpu().numpy(), c.cpu().numpy(), label="re-admitted")
    with pytest.raises(ag.AuvError):
        s.poll(10_000)
    s.close()


def test_serving_full_size(ag, orc):
    """16 vehicles with 2048^2 grids at 2 m and cfg-size requests
    (2k..50k soundings of a +-60 deg fan at 150 m altitude), batched as
    served: every node of every vehicle's grid against the oracle on the union
    of its soundings -- counts and NaN masks exact (nodes left empty by either
    side included), depths within 1e-5, every value within the depth range of
    its soundings."""
    grids, reqs = serving_schedule(duration=0.4)
    out, infos = _run(ag, grids, reqs, ag.AUV_SERVE_BATCHED, max_request=50000)
    assert all(i.state == ag.AUV_T_DONE for i in infos)
    filled = empty = 0
    for v, g in enumerate(grids):
        z, c = out[v]
        n = _check(orc, g, reqs, v, z, c, label=f"vehicle {v}")
        x, y, zz = _union(reqs, v)
        lo, hi = orc.idw_bounds(_ogrid(orc, g), x, y, zz, 6.0, 0, bin_log2=16)
        ok = ~np.isnan(z)
        assert np.all(z[ok] >= lo[ok].astype(np.float32)), f"vehicle {v}: below range"
        assert np.all(z[ok] <= hi[ok].astype(np.float32)), f"vehicle {v}: above range"
        filled += n
        empty += int((c == 0).sum())
    assert filled > 100000 and empty > 100000
