"""The C-ABI library loads and exports every entry point include/gsp.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsp.h")
LIB = os.path.join(ROOT, "paper_2402_11454_amd", "libgsp.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("gsp_create", "gsp_destroy", "gsp_load_csr", "gsp_run", "gsp_get_membership",
                 "gsp_get_modularity", "gsp_modularity", "gsp_step_move", "gsp_step_split", "gsp_step_aggregate"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgsp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2402_11454_amd as gsp
    monkeypatch.setattr(gsp, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gsp, "_lib", None)
    with pytest.raises(ImportError):
        gsp.lib()


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; --gpus N > 1 exits with a message (status 2)
    before touching a GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
