"""The C-ABI library loads and exports every symbol include/mf.h declares (CPU only:
no call here touches a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1109_1146_amd", "libmfard.so")
HDR = os.path.join(ROOT, "include", "mf.h")


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1109_1146_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mf_create_grid", "mf_set_caps", "mf_solve", "mf_flow_value", "mf_min_cut",
                     "mf_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(mf_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for f in declared_functions():
        assert hasattr(lib, f)


def test_binding_declares_the_same_names():
    from paper_1109_1146_amd import mf
    assert set(mf.EXPORTED) == set(declared_functions())


def test_pure_host_entry_points(lib):
    # mf_status_str and mf_discharge_bytes_per_vertex do not touch the device
    lib.mf_status_str.restype = ctypes.c_char_p
    assert lib.mf_status_str(0) == b"ok"
    assert lib.mf_status_str(6) == b"sweep limit reached"
    lib.mf_discharge_bytes_per_vertex.restype = ctypes.c_int64
    assert lib.mf_discharge_bytes_per_vertex(8) == (2 * 8 + 5) * 4


def test_no_cpu_fallback_when_library_missing(tmp_path):
    from paper_1109_1146_amd import mf
    saved = mf._lib
    try:
        mf._lib = None
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            mf.load(str(tmp_path / "nope.so"))
    finally:
        mf._lib = saved


def _c_layout(tmp_path, struct, fields):
    """offsetof of each field and sizeof of a struct of include/mf.h, by gcc."""
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mf.h"', 'int main(void) {']
    for f in fields:
        lines.append(f'    printf("%zu\\n", offsetof({struct}, {f}));')
    lines += [f'    printf("%zu\\n", sizeof({struct}));', '    return 0;', '}']
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    return [int(x) for x in out]


@pytest.mark.parametrize("name", ["mf_solve_opts", "mf_solve_stats"])
def test_binding_structs_match_the_header(tmp_path, name):
    """The ctypes structures of the binding have the C layout of include/mf.h."""
    from paper_1109_1146_amd import mf
    cls = getattr(mf, name)
    fields = [f[0] for f in cls._fields_]
    c = _c_layout(tmp_path, name, fields)
    py = [getattr(cls, f).offset for f in fields] + [ctypes.sizeof(cls)]
    assert c == py, dict(zip(fields + ["sizeof"], zip(c, py)))
