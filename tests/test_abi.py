"""The C-ABI library loads and exports every function that include/trimap.h
declares; plan validation and error codes work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trimap.h")
LIB = os.path.join(ROOT, "paper_1609_01490_amd", "libtrimap.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tri_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("tri_map_plan", "tri_launch_elementwise", "tri_launch_stencil", "tri_edm",
                 "tri_plan_destroy", "tri_plan_query", "tri_status_str"):
        assert need in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtrimap.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtrimap.so not built")
def test_plan_validation_on_host():
    from paper_1609_01490_amd import trimap as tm
    p = tm.Plan(2048, 16, "lambda")
    assert (p.info.m, p.info.tiles, p.info.grid_blocks, p.info.wasted_blocks) == (128, 8256, 8256, 0)
    q = tm.Plan(2048, 16, "bb")
    assert (q.info.grid_x, q.info.grid_y, q.info.wasted_blocks) == (128, 128, 128 * 127 // 2)
    r = tm.Plan(65536, 16, "lambda", include_diag=False)
    assert r.info.m == 4096 and r.info.elements == 65536 * 65535 // 2
    u = tm.Plan(100, 16, "utm")
    assert u.info.dump_entries == 5050 and u.info.grid_blocks == -(-5050 // 256)
    rb = tm.Plan(100, 16, "rb")     # m = 7: 7 x 4 grid
    assert (rb.info.grid_x, rb.info.grid_y) == (7, 4)
    rec = tm.Plan(2048, 16, "rec")  # m = 128: 64 x 129 grid
    assert (rec.info.grid_x, rec.info.grid_y, rec.info.wasted_blocks) == (64, 129, 0)
    e = tm.Plan(0, 16, "lambda")
    assert e.info.tiles == 0 and e.info.grid_blocks == 0
    for bad, code in [((-1, 16, "lambda"), tm.E_INVAL), ((10, 12, "lambda"), tm.E_INVAL),
                      ((2**31, 16, "lambda"), tm.E_RANGE), ((100, 32, "rec"), None),
                      ((300, 32, "rec"), tm.E_UNSUPPORTED)]:
        if code is None:
            tm.Plan(*bad)
            continue
        with pytest.raises(tm.TrimapError) as ei:
            tm.Plan(*bad)
        assert ei.value.status == code
    with pytest.raises(tm.TrimapError) as ei:
        tm.Plan(100, 16, "lambda", flags=1 << 17)
    assert ei.value.status == tm.E_INVAL
    assert tm.status_str(tm.E_RANGE) == "TRI_E_RANGE"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtrimap.so not built")
def test_edm_argument_checks_on_host():
    from paper_1609_01490_amd import trimap as tm
    p = tm.Plan(100, 16, "lambda")
    with pytest.raises(tm.TrimapError) as ei:
        p.edm_workspace_size(8, tm.EDM_FP32)
    assert ei.value.status == tm.E_INVAL   # diagonal included
    q = tm.Plan(100, 16, "lambda", include_diag=False)
    assert q.edm_workspace_size(8, tm.EDM_FP32) == 0
    with pytest.raises(tm.TrimapError) as ei:
        q.edm_workspace_size(0, tm.EDM_FP32)
    assert ei.value.status == tm.E_RANGE


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtrimap.so not built")
def test_tune_cache_file_round_trip(tmp_path):
    """The tuning cache parser reads back exactly what its writer writes
    (host-only: no GPU is needed to save or load)."""
    from paper_1609_01490_amd import trimap as tm
    src = tmp_path / "in.json"
    src.write_text(
        '{\n  "entries": [\n'
        '    {"arch": "gfx950", "cus": 256, "workload": 0, "bucket": 15, "d": 0, '
        '"tile": 64, "map": 1, "flags": 0, "ms": 1.15},\n'
        '    {"arch": "gfx950", "cus": 256, "workload": 2, "bucket": 14, "d": 0, '
        '"tile": 64, "map": 4, "flags": 1, "ms": 0.088}\n  ]\n}\n')
    tm.tune_cache_clear()
    tm.tune_cache_load(str(src))
    out = tmp_path / "out.json"
    tm.tune_cache_save(str(out))
    txt = out.read_text()
    assert txt.count('"arch": "gfx950"') == 2
    assert '"bucket": 15' in txt and '"tile": 64, "map": 1' in txt
    assert '"flags": 1, "ms": 0.088' in txt
    tm.tune_cache_clear()
    with pytest.raises(tm.TrimapError):
        tm.tune_cache_load(str(tmp_path / "missing.json"))
