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


def _c_layout(tmp_path, header_dir, header, structs):
    """{struct: (sizeof, {field: offset})} of C structs, from a program
    compiled with gcc against the header."""
    import subprocess
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{header}"', "int main(void) {"]
    for name, fields in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", header_dir, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    res = {}
    for line in out.splitlines():
        s, f, v = line.split()
        size, offs = res.setdefault(s, [0, {}])
        if f == "size":
            res[s][0] = int(v)
        else:
            offs[f] = int(v)
    return res


def _check_layout(layout, cname, ctype):
    size, offs = layout[cname]
    assert ctypes.sizeof(ctype) == size, cname
    for f, _ in ctype._fields_:
        assert getattr(ctype, f).offset == offs[f], (cname, f)


def test_binding_structs_match_the_header(tmp_path):
    """Every field of the binding's Options, Stats and KernelStat sits at the
    offset the C compiler gives gsp_options, gsp_stats and gsp_kernel_stat,
    and the sizes agree (a field added on one side only would shift the
    rest)."""
    import paper_2402_11454_amd as gsp
    structs = {"gsp_options": [f for f, _ in gsp.Options._fields_],
               "gsp_stats": [f for f, _ in gsp.Stats._fields_],
               "gsp_kernel_stat": [f for f, _ in gsp.KernelStat._fields_]}
    layout = _c_layout(tmp_path, os.path.join(ROOT, "include"), "gsp.h", structs)
    _check_layout(layout, "gsp_options", gsp.Options)
    _check_layout(layout, "gsp_stats", gsp.Stats)
    _check_layout(layout, "gsp_kernel_stat", gsp.KernelStat)


def test_oracle_structs_match_its_header(tmp_path):
    import oracle
    structs = {"orc_options": [f for f, _ in oracle._Options._fields_],
               "orc_stats": [f for f, _ in oracle._Stats._fields_],
               "orc_trace": [f for f, _ in oracle._Trace._fields_]}
    layout = _c_layout(tmp_path, os.path.join(ROOT, "oracle"), "oracle.h", structs)
    _check_layout(layout, "orc_options", oracle._Options)
    _check_layout(layout, "orc_stats", oracle._Stats)
    _check_layout(layout, "orc_trace", oracle._Trace)
