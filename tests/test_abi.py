"""The C ABI library builds for gfx950, loads, and exports every function
that include/szi.h declares; host-side argument checks.  CPU only: no call
here launches GPU work."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2312_05492_amd as szi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "szi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sz_[a-z_]+)\s*\(", src)))


def test_header_declares_the_api():
    names = _declared()
    for n in ["sz_compress", "sz_decompress", "sz_compress_batch", "sz_decompress_batch",
              "sz_serialize", "sz_upload", "sz_result_free", "sz_result_read", "sz_ctx_create",
              "sz_ctx_destroy", "sz_last_error", "sz_params_default"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = szi.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", szi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sz_[a-z_]+)\b", out))
    for n in _declared():
        assert n in exported, n
        assert hasattr(lib, n)


def test_library_holds_gfx950_code():
    # the offload bundle of the library we built names its target
    data = open(szi.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_params_default():
    p = szi.SzParams()
    szi.lib().sz_params_default(C.byref(p))
    assert p.eb_mode == szi.EB_REL and p.eb == 1e-3
    assert list(p.interp) == [3, 3, 3] and p.order[0] == -1
    assert p.radius == 512 and p.huff_chunk == 1024 and p.alpha == 0.0


def test_null_arguments_rejected_without_gpu():
    L = szi.lib()
    assert L.sz_ctx_create(None, 0, 0) == -1
    assert L.sz_compress(None, None, None, None, None, None) == -1
    assert L.sz_decompress(None, None, None, None) == -1
    assert L.sz_ctx_destroy(None) == 0
    assert L.sz_last_error(None) == b"no context"


def test_struct_layouts_match_header():
    # sizes of the ABI structs as the C compiler lays them out
    code = r'''
#include <stdio.h>
#include <stddef.h>
#include "szi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(sz_dims), sizeof(sz_params),
         sizeof(sz_result), offsetof(sz_result, header), offsetof(sz_result, internal),
         sizeof(sz_request), offsetof(sz_request, src), offsetof(sz_request, d_out),
         sizeof(sz_completion), offsetof(sz_completion, result));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(src, "w").write(code)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        got = list(map(int, subprocess.run([exe], capture_output=True, text=True).stdout.split()))
    assert got == [C.sizeof(szi.SzDims), C.sizeof(szi.SzParams), C.sizeof(szi.SzResult),
                   szi.SzResult.header.offset, szi.SzResult.internal.offset,
                   C.sizeof(szi.SzRequest), szi.SzRequest.src.offset, szi.SzRequest.d_out.offset,
                   C.sizeof(szi.SzCompletion), szi.SzCompletion.result.offset]
