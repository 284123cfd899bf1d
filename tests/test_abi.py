"""The C-ABI library builds for gfx950, loads on the host and exports every
entry point include/setd.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "setd.h")
LIB = os.path.join(ROOT, "paper_2511_22510_amd", "libsetd.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(setd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_named_calls():
    names = declared()
    for n in ("setd_plan_create", "setd_step", "setd_observe", "setd_submit"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsetd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsetd.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2511_22510_amd import setd
    assert sorted(setd.SIGNATURES) == declared()


def test_descriptor_layout_matches_header():
    """ctypes struct offsets equal the C struct's (checked with the host compiler)."""
    import subprocess
    import tempfile
    from paper_2511_22510_amd import setd
    fields = [f[0] for f in setd.setd_desc._fields_]
    src = '#include <stdio.h>\n#include <stddef.h>\n#include "setd.h"\nint main(void){\n'
    src += 'printf("%zu\\n", sizeof(setd_desc));\n'
    for f in fields:
        src += 'printf("%%zu\\n", offsetof(setd_desc, %s));\n' % f
    src += 'printf("%zu\\n", sizeof(setd_plan_info_t));\n}\n'
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = [int(v) for v in subprocess.check_output([exe]).split()]
    assert out[0] == ctypes.sizeof(setd.setd_desc)
    assert out[1:1 + len(fields)] == [getattr(setd.setd_desc, f).offset for f in fields]
    assert out[-1] == ctypes.sizeof(setd.setd_plan_info_t)


def test_sde_descriptor_layout_matches_header():
    import subprocess
    import tempfile
    from paper_2511_22510_amd import setd
    fields = [f[0] for f in setd.setd_sde_desc._fields_]
    src = '#include <stdio.h>\n#include <stddef.h>\n#include "setd.h"\nint main(void){\n'
    src += 'printf("%zu\\n", sizeof(setd_sde_desc));\n'
    for f in fields:
        src += 'printf("%%zu\\n", offsetof(setd_sde_desc, %s));\n' % f
    src += '}\n'
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = [int(v) for v in subprocess.check_output([exe]).split()]
    assert out[0] == ctypes.sizeof(setd.setd_sde_desc)
    assert out[1:] == [getattr(setd.setd_sde_desc, f).offset for f in fields]
