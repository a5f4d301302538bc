"""CPU checks of the C ABI: the library loads, and exports every function
that include/hsd.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsd.h")
LIB = os.path.join(ROOT, "paper_2304_06340_amd", "libhsd.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(hsd_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hsd_create_mesh", "hsd_freq_rule", "hsd_distance", "hsd_distance_grad",
                     "hsd_submit", "hsd_poll", "hsd_init", "hsd_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd.so not built")
def test_product_library_exports_only_the_header():
    """The C functions libhsd.so exports are exactly those include/hsd.h
    declares; the test hooks live in libhsd_testhooks.so only."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if " T hsd" in ln})
    assert exported == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd.so not built")
def test_binding_covers_the_header():
    from paper_2304_06340_amd import _lib
    assert set(declared_functions()) == set(_lib.exported_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd.so not built")
def test_params_default_and_version():
    from paper_2304_06340_amd import _lib
    L = _lib.load()
    p = _lib.Params()
    L.hsd_params_default(ctypes.byref(p))
    assert p.s == 1.0 and p.form == 0 and p.method == 0 and p.taylor_tau == 1e-2
    assert b"hsd" in L.hsd_version()
    assert L.hsd_last_error() == b""


def test_struct_sizes_match_header():
    """ctypes mirrors of the header structs have the C layout sizes."""
    from paper_2304_06340_amd import _lib
    assert ctypes.sizeof(_lib.Params) == 88
    assert ctypes.sizeof(_lib.Result) == 48


def test_struct_layouts_match_c_compiler(tmp_path):
    """Every ctypes mirror against sizeof/offsetof from a C compiler reading
    include/hsd.h itself."""
    import shutil
    import subprocess
    from paper_2304_06340_amd import _lib
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    mirrors = {"hsd_params": _lib.Params, "hsd_result": _lib.Result, "hsd_rule_desc": _lib.RuleDesc,
               "hsd_server_cfg": _lib.ServerCfg, "hsd_request": _lib.Request,
               "hsd_request_times": _lib.RequestTimes, "hsd_surface_desc": _lib.SurfaceDesc}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hsd.h"', 'int main(void) {']
    for cname, cls in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, *_ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, *_ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
