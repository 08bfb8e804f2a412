"""The C ABI library: it loads, exports every function include/ged.h declares,
and rejects invalid input on the host before touching the device (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_00830_amd import ged

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ged.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ged_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = ged.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ged.EXPORTS)


def test_abi_version_and_status_names():
    lib = ged.load()
    assert lib.ged_abi_version() == 6
    assert ged.status_name(ged.GED_OK) == "GED_OK"
    assert ged.status_name(ged.GED_EUNSUPPORTED) == "GED_EUNSUPPORTED"
    assert ged.status_name(99) == "GED_UNKNOWN"


def _db_create(graph_tuples, flags=None):
    """Call ged_db_create (ged_db_create_ex with flags) on host graphs; returns (status, message)."""
    lib = ged.load()
    keep = []
    recs = np.zeros(max(len(graph_tuples), 1), dtype=ged.GRAPH_DTYPE)
    for k, (n, vl, eu, ev, el) in enumerate(graph_tuples):
        arrs = [np.ascontiguousarray(x, dtype=np.int32) if x is not None else None for x in (vl, eu, ev, el)]
        keep.append(arrs)
        recs[k]["n"] = n
        recs[k]["m"] = len(eu)
        for name, a in zip(("vlabel", "eu", "ev", "elabel"), arrs):
            recs[k][name] = 0 if a is None else a.ctypes.data
    h = ctypes.c_void_p()
    if flags is None:
        st = lib.ged_db_create(recs.ctypes.data, len(graph_tuples), ctypes.byref(h))
    else:
        st = lib.ged_db_create_ex(recs.ctypes.data, len(graph_tuples), flags, ctypes.byref(h))
    assert h.value is None  # nothing is returned on failure
    return st, lib.ged_last_error().decode()


@pytest.mark.parametrize("case,status,text", [
    ((2, [0, 0], [0], [0], None), ged.GED_EINVAL, "self-loop"),
    ((3, [0, 0, 0], [0, 1], [1, 0], None), ged.GED_EINVAL, "repeats"),
    ((3, [0, 0, 0], [0], [3], None), ged.GED_EINVAL, "out of range"),
    ((-1, [], [], [], None), ged.GED_EINVAL, "negative"),
    ((1025, [0] * 1025, [], [], None), ged.GED_EUNSUPPORTED, "exceeds"),
    ((6, [0] * 6, [0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 3, 3, 4, 1, 2],
      [1, 2, 3, 4, 5, 2, 3, 4, 5, 3, 4, 5, 4, 5, 5, 2, 3], None), ged.GED_EINVAL, "more edges"),
])
def test_db_create_rejects_invalid_graphs(case, status, text):
    st, msg = _db_create([case])
    assert st == status and text in msg


@pytest.mark.parametrize("case,status,text", [
    ((2, [0, 0], [0], [0], None), ged.GED_EINVAL, "self-loop"),
    ((3, [0, 0, 0], [0, 1, 0], [1, 0, 1], None), ged.GED_EINVAL, "repeats"),
    ((3, [0, 0, 0], [2], [3], None), ged.GED_EINVAL, "out of range"),
    ((3, [0] * 3, [0, 0, 1, 1, 2, 2, 0], [1, 2, 0, 2, 0, 1, 1], None), ged.GED_EINVAL, "more edges"),
])
def test_directed_db_create_rejects_invalid_graphs(case, status, text):
    """Directed: arcs a -> b and b -> a are distinct, a repeated arc is not."""
    st, msg = _db_create([case], flags=ged.DB_DIRECTED)
    assert st == status and text in msg


def test_db_create_ex_rejects_unknown_flags():
    st, msg = _db_create([(2, [0, 0], [0], [1], None)], flags=2)
    assert st == ged.GED_EINVAL and "flags" in msg


def test_db_create_rejects_too_many_edge_labels():
    n = 8
    eu, ev = np.triu_indices(n, 1)
    eu, ev = eu[:17], ev[:17]
    st, msg = _db_create([(n, [0] * n, eu, ev, np.arange(17))])
    assert st == ged.GED_EUNSUPPORTED and "edge labels" in msg


def test_db_create_null_arguments():
    lib = ged.load()
    assert lib.ged_db_create(None, 1, ctypes.byref(ctypes.c_void_p())) == ged.GED_EINVAL
    assert lib.ged_db_create(None, 0, None) == ged.GED_EINVAL
    assert lib.ged_db_create(None, -1, ctypes.byref(ctypes.c_void_p())) == ged.GED_EINVAL


def test_null_handles_are_rejected():
    lib = ged.load()
    out = ctypes.c_int64()
    assert lib.ged_db_count(None, ctypes.byref(out)) == ged.GED_EINVAL
    flags = ctypes.c_uint32()
    assert lib.ged_db_flags(None, ctypes.byref(flags)) == ged.GED_EINVAL
    assert lib.ged_db_create_ex(None, 1, 0, ctypes.byref(ctypes.c_void_p())) == ged.GED_EINVAL
    assert lib.ged_db_create_ex(None, 0, 0, None) == ged.GED_EINVAL
    assert lib.ged_plan_map_size(None, ctypes.byref(out)) == ged.GED_EINVAL
    assert lib.ged_plan_create(None, None, 0, 4, ctypes.byref(ctypes.c_void_p())) == ged.GED_EINVAL
    assert lib.ged_plan_run(None, ged.Costs(1, 1, 1, 1, 1, 1), None, None, None, None) == ged.GED_EINVAL
    assert lib.ged_db_destroy(None) == ged.GED_OK
    assert lib.ged_plan_destroy(None) == ged.GED_OK


def test_new_boundary_calls_reject_null_arguments():
    """ged_plan_run_ex, ged_kbest_ex, ged_map_offsets, ged_kbest_noalloc and
    ged_server_submit_id check their arguments on the host first."""
    lib = ged.load()
    c = ged.Costs(1, 1, 1, 1, 1, 1)
    h = ctypes.c_void_p()
    t = ctypes.c_uint64()
    assert lib.ged_plan_run_ex(None, c, None, None, None, None, None) == ged.GED_EINVAL
    assert lib.ged_kbest_ex(None, None, 0, c, 4, None, None, None, None, None, None) == ged.GED_EINVAL
    bad = ged.PlanOptions(0, 0, 0, 0, 0x10)
    assert lib.ged_kbest_ex(None, None, 0, c, 4, ctypes.byref(bad), None, None, None, None, None) == ged.GED_EINVAL
    assert "flags" in lib.ged_last_error().decode()
    assert lib.ged_map_offsets(None, None, 0, None, None) == ged.GED_EINVAL
    assert lib.ged_kbest_noalloc(None, None, 0, c, 4, None, None, None) == ged.GED_EINVAL
    assert lib.ged_kbest_noalloc(None, None, 0, ged.Costs(1, -1, 1, 1, 1, 1), 4, None, None, None) == ged.GED_EINVAL
    assert lib.ged_server_submit_id(None, 0, 0, ctypes.byref(t)) == ged.GED_EINVAL
    assert h.value is None
