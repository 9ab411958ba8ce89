"""CPU checks of the C-ABI boundary: the library builds, loads and exports every declared symbol.

No compute call is made here (there is no GPU in this environment).
"""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "im.h")
LIB = os.path.join(ROOT, "paper_2105_04023_amd", "libhipfuser.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(im_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2105_04023_amd import build

        build.build()
    return LIB


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for n in ["im_build_sketches", "im_estimate", "im_estimate_all", "im_select_seeds", "im_ctx_create",
              "im_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib_path], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binds(lib_path):
    from paper_2105_04023_amd import _binding

    lib = _binding.load(lib_path)
    for n in declared_functions():
        assert hasattr(lib, n)
    assert set(_binding.EXPORTED) <= set(declared_functions())
    assert lib.im_version().startswith(b"hipfuser")
    assert lib.im_last_error() == b""


def test_library_is_gfx950_code_object(lib_path):
    # the device code object bundled in the library is built for gfx950 only
    blob = open(lib_path, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob
    assert b"gfx942" not in blob and b"gfx90a" not in blob


def test_bytes_needed_is_host_only(lib_path):
    from paper_2105_04023_amd import _binding

    lib = _binding.load(lib_path)
    n, m, R = 1 << 20, 16 << 20, 256
    b = lib.im_sketch_bytes_needed(n, m, R, 0)
    assert b > 3 * n * R  # three register buffers dominate
    assert lib.im_sketch_bytes_needed(n, m, 6, 0) == 0  # R not a multiple of 4
    assert lib.im_sketch_bytes_needed(0, m, R, 0) == 0


def test_ctypes_structs_match_the_c_layout(tmp_path):
    """Every struct the binding mirrors has the size and field offsets of include/im.h (gcc)."""
    import ctypes

    from paper_2105_04023_amd import _binding as B

    structs = [B.im_csr, B.im_probs, B.im_build_opts, B.im_select_opts, B.im_step, B.im_sketch_info,
               B.im_sweep_rec, B.im_select_stats, B.im_batch_job, B.im_batch_opts, B.im_batch_job_result,
               B.im_batch_stats, B.im_server_opts, B.im_request, B.im_response, B.im_server_stats]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "im.h"', "int main(void) {"]
    for s in structs:
        lines.append(f'printf("{s.__name__} %zu\\n", sizeof({s.__name__}));')
        for f, _ in s._fields_:
            lines.append(f'printf("{s.__name__}.{f} %zu\\n", offsetof({s.__name__}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for s in structs:
        assert int(out[s.__name__]) == ctypes.sizeof(s), s.__name__
        for f, _ in s._fields_:
            assert int(out[f"{s.__name__}.{f}"]) == getattr(s, f).offset, (s.__name__, f)
