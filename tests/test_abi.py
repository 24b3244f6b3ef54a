"""The C-ABI library loads and exports every function include/*.h declares.

No compute call is made here (no GPU in this test)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for mt in re.finditer(r"^[A-Za-z_][\w \*]*?\b(cor_\w+)\s*\(", txt, flags=re.M):
            names.add(mt.group(1))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["cor_utv", "cor_utv_ex", "cor_utv_batched", "cor_server_create",
              "cor_server_submit", "cor_server_wait", "cor_quantize", "cor_omega"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1810_07323_amd as cu

    if not os.path.exists(cu.LIB_PATH):
        pytest.fail("libcorutv.so not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(cu.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert set(cu._SIGS) == _declared()


def test_host_only_entry_points():
    import paper_1810_07323_amd as cu

    L = cu.lib()
    assert L.cor_status_string(cu.COR_E_INVAL) == b"invalid argument"
    # workspace sizing is pure host arithmetic
    b = cu.cor_workspace_bytes(8000, 8000, 110, cu.COR_F32)
    assert b > 8000 * 110 * 8 * 4
    assert cu.cor_workspace_bytes(10, 10, 1, cu.COR_F32) == 0
    assert cu.cor_workspace_bytes(10, 10, 300, cu.COR_F32) == 0


def test_tuning_table_json_round_trip(tmp_path):
    """cor_tune_load / cor_tune_save are host-only: a table written by hand is
    read, written back with the same entries, and malformed files are refused."""
    import json

    import paper_1810_07323_amd as cu

    cu.lib()
    assert cu.cor_tune_clear() == cu.COR_OK
    src = tmp_path / "tune.json"
    src.write_text(json.dumps({"version": 1, "entries": [
        {"m": 20000, "n": 10000, "l": 220, "prec": 0, "s_ax": 3, "s_atx": 6,
         "us_ax": 1690.0, "us_atx": 1710.0},
        {"m": 8000, "n": 8000, "l": 110, "prec": 1, "s_ax": 4, "s_atx": 8}]}))
    assert cu.cor_tune_load(str(src)) == cu.COR_OK
    out = tmp_path / "out.json"
    assert cu.cor_tune_save(str(out)) == cu.COR_OK
    got = json.loads(out.read_text())
    ent = sorted((e["m"], e["n"], e["l"], e["prec"], e["s_ax"], e["s_atx"]) for e in got["entries"])
    assert ent == [(8000, 8000, 110, 1, 4, 8), (20000, 10000, 220, 0, 3, 6)]
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps({"version": 1, "entries": [
        {"m": 100, "n": 100, "l": 10, "prec": 0, "s_ax": 0, "s_atx": 2}]}))
    assert cu.cor_tune_load(str(bad)) == cu.COR_E_INVAL
    assert cu.cor_tune_load(str(tmp_path / "missing.json")) == cu.COR_E_INVAL
    assert cu.cor_tune_clear() == cu.COR_OK
    assert cu.cor_tune_save(str(out)) == cu.COR_OK
    assert json.loads(out.read_text())["entries"] == []
