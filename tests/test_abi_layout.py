"""The ctypes mirrors of the public structs in include/qrng_ext.h have the C
compiler's layout: size and every field's offset, checked by compiling a
small C program against the header (host only, no GPU)."""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2402_14607_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MIRRORS = {
    "ext_params": binding.ExtParams,
    "ext_batch_item": binding.BatchItem,
    "ext_server_config": binding.ServerConfig,
    "ext_server_stats": binding.ServerStats,
    "ext_sim_config": binding.SimConfig,
    "ext_sim_result": binding.SimResult,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qrng_ext.h"', "int main(void) {"]
    for cname, cls in MIRRORS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, *_ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        table[(cname, field)] = int(value)
    return table


@pytest.mark.parametrize("cname", sorted(MIRRORS))
def test_struct_layout(c_layout, cname):
    cls = MIRRORS[cname]
    assert ctypes.sizeof(cls) == c_layout[(cname, "size")], cname
    for fname, *_ in cls._fields_:
        assert getattr(cls, fname).offset == c_layout[(cname, fname)], (cname, fname)


def test_stream_open_prototype(tmp_path):
    """ext_stream_open takes the stream's own (n_bits, m_bits): the header's
    prototype has that signature (a C function-pointer assignment that fails
    to compile otherwise) and the binding declares the same argument types."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "proto.c"
    src.write_text('#include "qrng_ext.h"\n'
                   "int (*f)(ext_ctx *, uint64_t, uint32_t, ext_stream **) = ext_stream_open;\n")
    subprocess.run([cc, "-std=c99", "-Werror", "-Wincompatible-pointer-types", "-c", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(tmp_path / "proto.o")],
                   check=True)
    args = list(binding.load().ext_stream_open.argtypes)
    assert args == [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                    ctypes.POINTER(ctypes.c_void_p)]
