"""The C-ABI library loads and exports every entry point its header declares
(no GPU work: symbol lookup only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tcspmv.h")
LIB = os.path.join(ROOT, "paper_1103_2405_amd", "libtcspmv.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("tc_build_tiled", "tc_spmv", "tc_spmm", "tc_pagerank", "tc_hits", "tc_rwr", "tc_export_format",
              "tc_handle_info", "tc_destroy", "tc_last_error", "tc_csr_spmv"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run python -m paper_1103_2405_amd.build)")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_knows_every_symbol():
    from paper_1103_2405_amd import tc
    assert set(tc.EXPORTED) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_rejected_without_gpu_work():
    from paper_1103_2405_amd import tc
    lib = tc.load_library()
    assert lib.tc_build_tiled(None, None, None, None) == tc.TC_EINVAL
    assert b"NULL" in lib.tc_last_error()
    assert lib.tc_handle_info(None, None) == tc.TC_EINVAL
    assert lib.tc_spmv(None, None, None, None) == tc.TC_EINVAL
    lib.tc_destroy(None)


def test_struct_layouts_match_the_binding(tmp_path):
    # compile a probe against the header and compare every field offset and
    # struct size with the ctypes mirrors in the binding
    import subprocess
    from paper_1103_2405_amd import tc
    structs = {"tc_csr": tc.CCsr, "tc_build_opts": tc.CBuildOpts, "tc_info": tc.CInfo,
               "tc_format_view": tc.CFormatView, "tc_timing": tc.CTiming}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tcspmv.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                               text=True).stdout.split("\n") if line)
    for cname, py in structs.items():
        assert int(got["%s size" % cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(py, fname).offset, (cname, fname)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_options_rejected_without_gpu_work():
    # option checks come before any device work (the CSR pointers are never
    # read here, so placeholders do)
    import ctypes
    from paper_1103_2405_amd import tc
    lib = tc.load_library()
    fake = 0x1000
    A = tc.CCsr(10, 10, 5, fake, fake, fake)
    h = ctypes.c_void_p()
    for field, value in [("value_map", 2), ("kernel", 2), ("split_len", -2), ("xcd_groups", 65), ("wl_policy", 3)]:
        o = tc.CBuildOpts()
        lib.tc_build_opts_default(ctypes.byref(o))
        setattr(o, field, value)
        assert lib.tc_build_tiled(ctypes.byref(A), ctypes.byref(o), None, ctypes.byref(h)) == tc.TC_EINVAL, field
        assert not h.value
    o = tc.CBuildOpts()
    lib.tc_build_opts_default(ctypes.byref(o))
    o.value_map, o.kernel = 1, 1  # the value map serves the composite kernel only
    assert lib.tc_build_tiled(ctypes.byref(A), ctypes.byref(o), None, ctypes.byref(h)) == tc.TC_EINVAL
    assert lib.tc_refresh_values(None, None, None) == tc.TC_EINVAL
    assert lib.tc_gather_rows(None, 0, None, -1, 1, None, None) == tc.TC_EINVAL
    assert lib.tc_gather_rows(None, 0, None, 5, 0, None, None) == tc.TC_EINVAL
