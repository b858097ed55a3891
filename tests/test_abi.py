"""The C-ABI library loads and exports every entry point that include/dg2.h declares.

CPU-only: loads the library without calling into the GPU.
"""
import ctypes
import os
import re

import pytest

from paper_2010_02003_amd import dg2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dg2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg2_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for required in ("dg2_create", "dg2_destroy", "dg2_set_dem_corners", "dg2_set_manning",
                     "dg2_set_boundary", "dg2_set_inflow_hydrograph", "dg2_step", "dg2_run_to",
                     "dg2_read_gauges"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(dg2.LIB_PATH), reason="libdg2.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(dg2.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    assert sorted(dg2.exported_symbols()) == _declared()


def test_config_struct_matches_header_layout():
    # int32 nx, ny | 4 doubles | int32 prec, variant | 5 doubles | pointer
    assert ctypes.sizeof(dg2.Config) == 8 + 32 + 8 + 40 + 8
    assert dg2.Config.hip_stream.offset == 88


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(dg2, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        dg2.load_library(str(tmp_path / "nope.so"))
