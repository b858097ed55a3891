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


def test_config_struct_matches_header_layout(tmp_path):
    """The ctypes mirror of dg2_config against the C compiler's layout of the
    header's struct (size and every field offset)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    fields = [f[0] for f in dg2.Config._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"dg2.h\"\nint main(void) {\n"
                   '  printf("%zu\\n", sizeof(dg2_config));\n'
                   + "".join('  printf("%%zu\\n", offsetof(dg2_config, %s));\n' % f for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(dg2.Config)
    assert out[1:] == [getattr(dg2.Config, f).offset for f in fields]


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(dg2, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        dg2.load_library(str(tmp_path / "nope.so"))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for several it exits with a message
    before it touches a device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
