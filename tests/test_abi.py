"""The C-ABI library loads and exports every entry point include/dsd.h declares (CPU only)."""
import ctypes
import os
import re

from paper_1906_00341_amd import dsd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dsd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dsd_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_path():
    syms = declared_symbols()
    for s in ("dsd_build_csr", "dsd_clique_degrees", "dsd_clique_core", "dsd_core_app", "dsd_core_exact"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(dsd.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(dsd.EXPORTS) == declared_symbols()


def test_status_strings():
    lib = dsd.load()
    for code, name in dsd.STATUS.items():
        assert dsd.status_str(code) == name
    assert lib.dsd_last_error() is not None


def test_null_and_bad_arguments_are_rejected_without_touching_a_gpu():
    lib = dsd.load()
    h = ctypes.c_void_p()
    assert lib.dsd_build_csr(-1, 0, None, None, 0, None, ctypes.byref(h)) == -1
    assert lib.dsd_build_csr(3, 2, None, None, 0, None, ctypes.byref(h)) == -1
    assert lib.dsd_build_csr(3, 0, None, None, 7, None, ctypes.byref(h)) == -1
    assert lib.dsd_graph_free(None) == 0
    assert lib.dsd_clique_degrees(None, 3, 0, None, None) == -1


def test_batch_and_server_arguments_are_rejected_without_touching_a_gpu():
    lib = dsd.load()
    res = (dsd.Result * 1)()
    assert lib.dsd_batch_run(-1, None, None, 0, 0, None, res) == -1
    assert lib.dsd_batch_run(0, None, None, 0, 0, None, res) == 0          # empty batch
    assert lib.dsd_batch_run(1, None, None, 0, 0, None, res) == -1         # NULL arrays
    g = (ctypes.c_void_p * 1)(None)
    hs = (ctypes.c_int * 1)(3)
    assert lib.dsd_batch_run(1, g, hs, 0, 0, None, res) == -1              # NULL handle
    assert lib.dsd_batch_run(1, g, hs, 9, 0, None, res) == -1              # unknown op
    s = ctypes.c_void_p()
    assert lib.dsd_server_create(0, 4, ctypes.byref(s)) == -1
    assert lib.dsd_server_create(1 << 30, 0, ctypes.byref(s)) == -1
    t = ctypes.c_uint64()
    assert lib.dsd_server_submit(None, None, 3, 0, 0, None, ctypes.byref(t)) == -1
    assert lib.dsd_server_wait(None, 1, 0, None) == -1
    assert lib.dsd_server_cancel(None, 1) == -1
    assert lib.dsd_server_destroy(None) == 0


def test_struct_layouts_match_the_header(tmp_path):
    # the binding's ctypes structures against the header, compiled by the C
    # compiler: every field at the same offset, the same total size
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no C compiler")
    structs = {"dsd_stats": dsd.Stats, "dsd_result": dsd.Result, "dsd_rational": dsd.Rational,
               "dsd_tune_result": dsd.TuneResult}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dsd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
