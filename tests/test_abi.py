"""CPU-only checks of the C ABI: the library loads, exports every declared
entry point, and validates arguments on the host (no device work)."""
import ctypes
import os
import re

import pytest

import paper_2505_22675_amd as ag

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(auv_\w+)\s*\(", text, re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = ag.load_library()
    names = _declared()
    assert {"auv_grid_create", "auv_bin_points", "auv_interp_idw",
            "auv_interp_nearest", "auv_resample_bilinear"} <= names
    raw = ctypes.CDLL(ag.LIB_PATH)
    for n in sorted(names):
        assert hasattr(raw, n), n
    assert "gfx950" in ag.auv_version()
    del lib


def test_grid_validation_on_host():
    g = ag.auv_grid_create(ag.make_desc(0, 0, 2.0, 2.0, 4096, 4096))
    assert g.nx == 4096
    with pytest.raises(ag.AuvError) as e:
        ag.auv_grid_create(ag.make_desc(0, 0, 0.0, 2.0, 10, 10))
    assert e.value.status == ag.AUV_ERR_INVALID
    with pytest.raises(ag.AuvError) as e:
        ag.auv_grid_create(ag.make_desc(0, 0, 2.0, 2.0, 9000, 10))
    assert e.value.status == ag.AUV_ERR_RANGE
    with pytest.raises(ag.AuvError):
        ag.auv_grid_create(ag.make_desc(float("nan"), 0, 1.0, 1.0, 10, 10))


def test_workspace_query_on_host():
    g = ag.auv_grid_create(ag.make_desc(0, 0, 2.0, 2.0, 4096, 4096))
    b = ag.auv_bin_workspace_size(g, 2_000_000, 6.0, 19)
    assert 2_000_000 * 40 < b < 2_000_000 * 64 + 64 * 1026 * 1026
    assert ag.auv_bin_workspace_size(g, 0, 6.0, 0) > 0
    with pytest.raises(ag.AuvError) as e:
        ag.auv_bin_workspace_size(g, 10, 6.0, 40)
    assert e.value.status == ag.AUV_ERR_INVALID
    with pytest.raises(ag.AuvError):
        ag.auv_bin_workspace_size(g, 10, -1.0, 0)
    with pytest.raises(ag.AuvError):
        ag.auv_bin_workspace_size(g, -5, 6.0, 0)
    assert "radius" in ag.auv_last_error() or "n must" in ag.auv_last_error()


def _host_item(n=1000, side=64, power=2.0, precision=ag.AUV_P_FP32_REBASE, max_pts=16):
    # placeholder addresses: planning validates and sizes, it never dereferences
    it = ag.auv_batch_item()
    it.grid = ag.make_desc(0, 0, 2.0, 2.0, side, side)
    it.x, it.y, it.z = 0x10000, 0x20000, 0x30000
    it.n = n
    it.params = ag.idw_params(power, 6.0, 1, max_pts, precision)
    it.z_out = 0x40000
    return it


def test_batch_plan_on_host():
    lib = ag.load_library()
    items = [_host_item(200_000, 64), _host_item(1_000, 1024, power=1.5),
             _host_item(0, 128, max_pts=0)]
    arr = (ag.auv_batch_item * 3)(*items)
    h = ctypes.c_void_p()
    assert lib.auv_batch_plan(arr, 3, None, ctypes.byref(h)) == ag.AUV_OK
    nbytes = ctypes.c_size_t()
    assert lib.auv_batch_workspace_size(h, ctypes.byref(nbytes)) == ag.AUV_OK
    # at least the binned records of every item
    assert nbytes.value > 201_000 * 40
    s, a = ctypes.c_int32(), ctypes.c_int32()
    assert lib.auv_batch_item_plan(h, 0, ctypes.byref(s), ctypes.byref(a), None, None) == ag.AUV_OK
    # ~1150 soundings per disk with k = 16: the dense form by default
    assert (s.value, a.value) == (19, ag.AUV_ALGO_DENSE)
    assert lib.auv_batch_item_plan(h, 1, ctypes.byref(s), ctypes.byref(a), None, None) == ag.AUV_OK
    assert (s.value, a.value) == (19, ag.AUV_ALGO_SPARSE)
    assert lib.auv_batch_item_plan(h, 3, ctypes.byref(s), ctypes.byref(a), None, None) == ag.AUV_ERR_INVALID
    lib.auv_batch_destroy(h)


def test_batch_plan_reads_tune_table(tmp_path):
    lib = ag.load_library()
    items = [_host_item(200_000, 64)]
    # class of the item: floor(log2(disk population + 1)), round(log2(side))
    pop = 200_000 / (128.0 + 12.0) ** 2 * 3.141592653589793 * 36.0
    dens = int(__import__("math").floor(__import__("math").log2(pop + 1.0)))
    table = tmp_path / "tune.txt"
    table.write_text("# comment line\n"
                     f"class {dens} 6 bin_log2 17 algo {ag.AUV_ALGO_SPARSE} ms 0.1\n")
    arr = (ag.auv_batch_item * 1)(*items)
    h = ctypes.c_void_p()
    assert lib.auv_batch_plan(arr, 1, str(table).encode(), ctypes.byref(h)) == ag.AUV_OK
    s, a = ctypes.c_int32(), ctypes.c_int32()
    assert lib.auv_batch_item_plan(h, 0, ctypes.byref(s), ctypes.byref(a), None, None) == ag.AUV_OK
    assert (s.value, a.value) == (17, ag.AUV_ALGO_SPARSE)
    tw, th = ctypes.c_int32(), ctypes.c_int32()
    assert lib.auv_batch_item_plan(h, 0, None, None, ctypes.byref(tw),
                                   ctypes.byref(th)) == ag.AUV_OK
    assert (tw.value, th.value) == (16, 16)  # no tile fields: the form's default
    lib.auv_batch_destroy(h)
    # a table with a node tile
    table.write_text(f"class {dens} 6 bin_log2 16 algo {ag.AUV_ALGO_DENSE} tile 16 4 ms 0.1\n")
    assert lib.auv_batch_plan(arr, 1, str(table).encode(), ctypes.byref(h)) == ag.AUV_OK
    assert lib.auv_batch_item_plan(h, 0, ctypes.byref(s), ctypes.byref(a), ctypes.byref(tw),
                                   ctypes.byref(th)) == ag.AUV_OK
    assert (s.value, a.value, tw.value, th.value) == (16, ag.AUV_ALGO_DENSE, 16, 4)
    lib.auv_batch_destroy(h)


def test_batch_plan_rejects_bad_items():
    lib = ag.load_library()
    bad = [_host_item(), _host_item(precision=ag.AUV_P_FP16_OFFSETS)]
    arr = (ag.auv_batch_item * 2)(*bad)
    h = ctypes.c_void_p()
    assert lib.auv_batch_plan(arr, 2, None, ctypes.byref(h)) == ag.AUV_ERR_INVALID
    assert "item 1" in ag.auv_last_error()
    assert not h.value
    bad = [_host_item(power=-1.0)]
    arr = (ag.auv_batch_item * 1)(*bad)
    assert lib.auv_batch_plan(arr, 1, None, ctypes.byref(h)) == ag.AUV_ERR_INVALID
    assert "item 0" in ag.auv_last_error()
    assert lib.auv_batch_plan(arr, 0, None, ctypes.byref(h)) == ag.AUV_ERR_INVALID
    it = _host_item()
    it.z_out = None
    arr = (ag.auv_batch_item * 1)(it)
    assert lib.auv_batch_plan(arr, 1, None, ctypes.byref(h)) == ag.AUV_ERR_INVALID


def _serve_desc(**kw):
    grids = [ag.make_desc(v * 8192.0, 0.0, 2.0, 2.0, 2048, 2048) for v in range(4)]
    return ag.session_desc(grids, **kw)


def test_session_budget_on_host():
    fixed, per_vehicle = ag.auv_session_budget(_serve_desc(max_request=50000, slots=8))
    # five 4-byte planes per node of a 2048^2 grid: weighted depth, weight,
    # count, smallest and largest depth
    assert per_vehicle == 5 * 2048 * 2048 * 4
    # per slot: 24 B per sounding staged plus the binning workspace of 514^2 bins
    assert 8 * (50000 * 24 + 514 * 514 * 8) < fixed < 8 * (50000 * 200 + 514 * 514 * 20) + 2 ** 22
    f2, _ = ag.auv_session_budget(_serve_desc(max_request=50000, slots=16))
    assert f2 > fixed


@pytest.mark.parametrize("kw, needle", [
    ({"power": 2.5}, "power"),
    ({"max_request": 0}, "max_request"),
    ({"slots": 0}, "slots"),
    ({"mode": 7}, "mode"),
    ({"max_batch": 65}, "max_batch"),
    ({"radius": 300.0}, "radius"),
    ({"radius": 20.0}, "window"),
])
def test_session_desc_validation_on_host(kw, needle):
    with pytest.raises(ag.AuvError) as e:
        ag.auv_session_budget(_serve_desc(**kw))
    assert needle in str(e.value)


def test_session_rejects_capped_idw_on_host():
    d = _serve_desc()
    d.params.max_pts = 16
    with pytest.raises(ag.AuvError) as e:
        ag.auv_session_budget(d)
    assert "max_pts" in str(e.value)
