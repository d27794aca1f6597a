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
