"""GPU parity of the batched path (many independent, uneven items: batched
binning, persistent per-XCD-queue IDW kernels, one captured HIP graph)
against the FP64 oracle, through the C ABI.

Each item's result has the definition and bar of a single auv_interp_idw
call: counts, NaN masks and nearest indices bit-exact, depths within 1e-5
relative of the oracle.  The batch only changes the schedule.
"""
import numpy as np
import pytest
import torch

from gen import GridSpec, Soundings, uniform_field, workload_cfg3_tiles

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


class _Item:
    """Device inputs and outputs of one batch item (kept alive by the test)."""

    def __init__(self, ag, s: Soundings, with_nearest=True, with_counts=True, algo=0,
                 max_pts=None, min_pts=None, power=None):
        self.s = s
        self.power = s.power if power is None else power
        self.max_pts = s.max_pts if max_pts is None else max_pts
        self.min_pts = s.min_pts if min_pts is None else min_pts
        g = s.grid
        self.desc = ag.make_desc(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
        self.x, self.y, self.z = _dev(s.x), _dev(s.y), _dev(s.z)
        shape = (g.ny, g.nx)
        self.zo = torch.full(shape, -1.0, dtype=torch.float32, device="cuda")
        self.co = torch.full(shape, -7, dtype=torch.int32, device="cuda") if with_counts else None
        self.no = torch.full(shape, -7, dtype=torch.int32, device="cuda") if with_nearest else None
        self.nz = torch.full(shape, -1.0, dtype=torch.float32, device="cuda") if with_nearest else None
        p = ag.idw_params(self.power, s.radius, self.min_pts, self.max_pts, algo=algo)
        self.item = ag.batch_item(self.desc, self.x, self.y, self.z, p, self.zo, self.co,
                                  self.no, self.nz)

    def clear(self):
        self.zo.fill_(-1.0)
        for t in (self.co, self.no):
            if t is not None:
                t.fill_(-7)
        if self.nz is not None:
            self.nz.fill_(-1.0)

    def host(self):
        out = {"z": self.zo.cpu().numpy()}
        if self.co is not None:
            out["cnt"] = self.co.cpu().numpy()
        if self.no is not None:
            out["nn"] = self.no.cpu().numpy()
            out["nz"] = self.nz.cpu().numpy()
        return out


def _ogrid(orc, g):
    return orc.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def _check_item(orc, it: _Item, out, label):
    s = it.s
    oz, oc, on = orc.idw(_ogrid(orc, s.grid), s.x, s.y, s.z, s.radius, it.power, it.min_pts,
                         it.max_pts, bin_log2=16)
    gz = out["z"].astype(np.float64)
    if "cnt" in out:
        bad = np.argwhere(out["cnt"] != oc)
        assert bad.size == 0, f"{label}: counts differ at {bad[:5]}"
    assert np.array_equal(np.isnan(gz), np.isnan(oz)), f"{label}: NaN masks differ"
    ok = ~np.isnan(oz)
    err = np.abs(gz[ok] - oz[ok]) / np.maximum(np.abs(oz[ok]), 1e-30)
    assert err.size == 0 or err.max() <= REL, f"{label}: max rel err {err.max():.3e}"
    if "nn" in out:
        assert np.array_equal(out["nn"], on), f"{label}: nearest indices differ"
        have = on >= 0
        assert np.array_equal(out["nz"][have], s.z[on[have]].astype(np.float32))
        assert np.all(np.isnan(out["nz"][~have]))


def _mixed_items(ag):
    """Uneven tiles of the batched workload (scaled down) plus items that
    exercise every schedule branch: general power, no cap, min_pts, empty,
    a non-linear node lattice, a wide window, a forced dense form with a cap
    above the persistent dense limit, outputs without counts / nearest."""
    tiles = workload_cfg3_tiles(n_tiles=14, seed=3, scale=0.08, sides=(64, 128, 256))
    items = [_Item(ag, s) for s in tiles]
    fx, fy, fz, fg = uniform_field(n=6000, seed=11, extent=500.0, nodes=128)
    f = Soundings(fx, fy, fz, fg, radius=6.0, power=2.0, min_pts=1, max_pts=16, name="field")
    items.append(_Item(ag, f, power=1.5, max_pts=16))               # general power
    items.append(_Item(ag, f, power=2.0, max_pts=0, min_pts=3))     # no cap, min 3
    e = Soundings(np.zeros(0), np.zeros(0), np.zeros(0), GridSpec(0.0, 0.0, 2.0, 2.0, 40, 24),
                  radius=6.0, power=2.0, min_pts=1, max_pts=16, name="empty")
    items.append(_Item(ag, e))                                       # empty item
    nl = Soundings(f.x, f.y, f.z, GridSpec(0.0, 0.0, 1000.0 / 255.0, 1000.0 / 255.0, 128, 128),
                   radius=6.0, power=2.0, min_pts=1, max_pts=8, name="nonlinear")
    items.append(_Item(ag, nl))                                      # generic tile kernel
    w = Soundings(f.x, f.y, f.z, GridSpec(0.0, 0.0, 2.0, 2.0, 200, 200), radius=10.0,
                  power=3.0, min_pts=1, max_pts=16, name="two-chunk")
    items.append(_Item(ag, w))                                       # 11 x 11 node window
    w = Soundings(f.x, f.y, f.z, GridSpec(0.0, 0.0, 2.0, 2.0, 200, 200), radius=20.0,
                  power=2.0, min_pts=1, max_pts=16, name="too-wide")
    items.append(_Item(ag, w))                                       # generic tile kernel
    d = tiles[int(np.argmax([len(t.x) for t in tiles]))]
    items.append(_Item(ag, d, max_pts=24, algo=ag.AUV_ALGO_DENSE))  # dense, k > 16
    items.append(_Item(ag, tiles[0], with_nearest=False, with_counts=False))
    items.append(_Item(ag, tiles[1], algo=ag.AUV_ALGO_SPAN))          # span form
    items.append(_Item(ag, f, power=3.0, max_pts=0, algo=ag.AUV_ALGO_SPAN))
    return items


def test_batch_mixed_parity_and_replay(ag, orc):
    items = _mixed_items(ag)
    b = ag.Batch([it.item for it in items])
    plans = [b.item_plan(i) for i in range(len(items))]
    assert any(a == ag.AUV_ALGO_DENSE for _, a in plans)
    assert any(a == ag.AUV_ALGO_SPARSE for _, a in plans)
    b.launch()
    torch.cuda.synchronize()
    first = [it.host() for it in items]
    for k, (it, out) in enumerate(zip(items, first)):
        _check_item(orc, it, out, f"item {k} ({it.s.name}, plan {plans[k]})")
    # replays: outputs cleared and unrelated eager work in between; every
    # replay must reproduce the first launch bit for bit
    for rep in range(3):
        for it in items:
            it.clear()
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2.0).sum().item()
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for k, (it, ref) in enumerate(zip(items, first)):
            out = it.host()
            for key in ref:
                assert np.array_equal(out[key], ref[key], equal_nan=True), \
                    f"replay {rep}: item {k} output {key} differs"
    b.close()


def test_batch_overcap_nodes(ag, orc):
    """Window-form items whose clustered soundings put most nodes above the
    cap: those nodes are finished after the persistent kernels, one lane per
    node (caps up to 16), or inside their tile (cap above 16).  Every node
    against the oracle, on the first launch and on replays."""
    rng = np.random.default_rng(97)
    g = GridSpec(500.0, 800.0, 2.0, 2.0, 120, 88)
    centres = rng.uniform([0, 0], [240, 176], size=(12, 2))
    pts = np.concatenate([c + rng.normal(0, 8.0, size=(3000, 2)) for c in centres])
    pts = np.concatenate([pts, rng.uniform([-6, -6], [246, 182], size=(3000, 2))])
    x, y = g.x0 + pts[:, 0], g.y0 + pts[:, 1]
    snap = np.arange(len(x)) % 3 == 0                      # lattice ties on a third
    x[snap] = g.x0 + np.round((x[snap] - g.x0) / 0.25) * 0.25
    y[snap] = g.y0 + np.round((y[snap] - g.y0) / 0.25) * 0.25
    z = -3000.0 + 20.0 * np.cos((x - g.x0) / 23.0) + rng.normal(0, 2.0, len(x))
    items = []
    for k, p in ((4, 2.0), (16, 1.0), (9, 1.5), (20, 3.0)):
        s = Soundings(x, y, z, g, radius=6.0, power=p, min_pts=1, max_pts=k, name=f"k{k}")
        items.append(_Item(ag, s, algo=ag.AUV_ALGO_SPARSE))
    b = ag.Batch([it.item for it in items])
    assert all(b.item_plan(i)[1] == ag.AUV_ALGO_SPARSE for i in range(len(items)))
    b.launch()
    torch.cuda.synchronize()
    first = [it.host() for it in items]
    for it, out in zip(items, first):
        assert (out["cnt"] == it.max_pts).mean() > 0.3, "too few nodes at the cap"
        _check_item(orc, it, out, f"over-cap item {it.s.name}")
    for rep in range(2):
        for it in items:
            it.clear()
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for k, (it, ref) in enumerate(zip(items, first)):
            out = it.host()
            for key in ref:
                assert np.array_equal(out[key], ref[key], equal_nan=True), \
                    f"replay {rep}: item {k} output {key} differs"
    b.close()


def test_batch_plain_form_parity(ag, orc):
    items = _mixed_items(ag)
    b = ag.Batch([it.item for it in items])
    b.launch_plain()
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        _check_item(orc, it, it.host(), f"plain item {k} ({it.s.name})")
    b.close()


def test_batch_autotune_round_trip(ag, orc, tmp_path):
    tiles = workload_cfg3_tiles(n_tiles=10, seed=3, scale=0.08, sides=(64, 128))
    items = [_Item(ag, s) for s in tiles]
    b0 = ag.Batch([it.item for it in items])
    path = str(tmp_path / "tune.txt")
    ag.auv_batch_autotune([it.item for it in items], b0.ws, path)
    torch.cuda.synchronize()
    rows = [ln.split() for ln in open(path) if ln.startswith("class ")]
    assert rows, "autotune wrote no class"
    table = {}
    for r in rows:
        assert r[3] == "bin_log2" and r[5] == "algo" and r[7] == "tile" and r[10] == "ms"
        assert 12 <= int(r[4]) <= 26 and int(r[6]) in (ag.AUV_ALGO_SPARSE, ag.AUV_ALGO_DENSE)
        tw, th = int(r[8]), int(r[9])
        if int(r[6]) == ag.AUV_ALGO_DENSE:
            assert tw * th == 64 and tw in (4, 8, 16)
        else:
            assert tw == 16 and th in (8, 16)
        assert float(r[11]) > 0.0
        table[(int(r[1]), int(r[2]))] = (int(r[4]), int(r[6]), tw, th)
    b0.close()
    b = ag.Batch([it.item for it in items], tune_path=path)
    chosen = {b.item_plan_full(i) for i in range(len(items))}
    assert chosen <= set(table.values())
    for it in items:
        it.clear()
    b.launch()
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        _check_item(orc, it, it.host(), f"tuned item {k} (plan {b.item_plan(k)})")
    b.close()


def _class_of(s):
    """The batch's item class: floor(log2(expected soundings per disk + 1)),
    round(log2(largest grid side))."""
    g, r = s.grid, s.radius
    area = (g.nx * g.dx + 2 * r) * (g.ny * g.dy + 2 * r)
    pop = len(s.x) / area * np.pi * r * r
    return int(np.floor(np.log2(pop + 1.0))), int(round(np.log2(max(g.nx, g.ny))))


def test_batch_non_default_tiles(ag, orc, tmp_path):
    """Every item planned with a node tile other than its form's default (from
    a written tune table: window form 16 x 8, dense form 16 x 4 or 4 x 16),
    run by the persistent kernels, against the oracle node by node."""
    tiles = workload_cfg3_tiles(n_tiles=12, seed=5, scale=0.08, sides=(64, 128, 256))
    items = [_Item(ag, s) for s in tiles]
    b0 = ag.Batch([it.item for it in items])
    lines, seen, dense_w = [], set(), 16
    for k, it in enumerate(items):
        key = _class_of(it.s)
        if key in seen:
            continue
        seen.add(key)
        s_log2, algo = b0.item_plan(k)
        if algo == ag.AUV_ALGO_DENSE:
            tw, th = dense_w, 64 // dense_w
            dense_w = 4 if dense_w == 16 else 16
        else:
            tw, th = 16, 8
        lines.append(f"class {key[0]} {key[1]} bin_log2 {s_log2} algo {algo} tile {tw} {th} ms 1")
    b0.close()
    path = tmp_path / "tune.txt"
    path.write_text("\n".join(lines) + "\n")
    b = ag.Batch([it.item for it in items], tune_path=str(path))
    plans = [b.item_plan_full(i) for i in range(len(items))]
    assert all((p[2], p[3]) in ((16, 8), (16, 4), (4, 16)) for p in plans), plans
    assert {(p[2], p[3]) for p in plans} >= {(16, 8)}
    b.launch()
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        _check_item(orc, it, it.host(), f"item {k} (plan {plans[k]})")
    b.close()


def test_batch_full_size(ag, orc, tmp_path):
    """The 256-tile batch at full size, autotuned as timed (two replays of the
    graph): every node of every tile against the oracle.  A tile whose oracle
    search would visit more than 6e7 candidates would be checked on 8192 nodes
    (edges included) instead; at this workload none does."""
    tiles = workload_cfg3_tiles()
    items = [_Item(ag, s) for s in tiles]
    b0 = ag.Batch([it.item for it in items])
    path = str(tmp_path / "tune.txt")
    ag.auv_batch_autotune([it.item for it in items], b0.ws, path)
    b0.close()
    b = ag.Batch([it.item for it in items], tune_path=path)
    for it in items:
        it.clear()
    b.launch()
    b.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(31)
    full = 0
    for k, it in enumerate(items):
        g = it.s.grid
        m = g.nx * g.ny
        density = len(it.s.x) / (g.nx * g.dx * g.ny * g.dy)
        label = f"tile {k} (n={len(it.s.x)}, side={g.nx}, plan {b.item_plan(k)})"
        if m * density * 169.0 <= 6e7:
            nodes = None
            full += 1
            gz = it.zo.cpu().numpy().astype(np.float64)
            gc, gn = it.co.cpu().numpy(), it.no.cpu().numpy()
        else:
            edges = np.concatenate([np.arange(g.nx), np.arange(m - g.nx, m),
                                    np.arange(0, m, g.nx), np.arange(g.nx - 1, m, g.nx)])
            nodes = np.unique(np.concatenate([edges, rng.integers(0, m, 8192)]))[:8192]
            nodes = nodes.astype(np.int64)
            sel = torch.from_numpy(nodes).cuda()
            gz = it.zo.view(-1)[sel].cpu().numpy().astype(np.float64)
            gc = it.co.view(-1)[sel].cpu().numpy()
            gn = it.no.view(-1)[sel].cpu().numpy()
        oz, oc, on = orc.idw(_ogrid(orc, g), it.s.x, it.s.y, it.s.z, it.s.radius, it.s.power,
                             it.s.min_pts, it.s.max_pts, bin_log2=16, nodes=nodes)
        assert np.array_equal(gc, oc), f"{label}: counts differ"
        assert np.array_equal(gn, on), f"{label}: nearest differ"
        assert np.array_equal(np.isnan(gz), np.isnan(oz)), f"{label}: NaN masks differ"
        ok = ~np.isnan(oz)
        err = np.abs(gz[ok] - oz[ok]) / np.maximum(np.abs(oz[ok]), 1e-30)
        assert err.size == 0 or err.max() <= REL, f"{label}: max rel err {err.max():.3e}"
    assert full == len(items), f"only {full} tiles checked in full"
    b.close()
