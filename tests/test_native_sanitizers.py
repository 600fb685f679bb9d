"""The oracle's C core and the library's blob parser built with the host
compiler under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU code
is built or run): the oracle on fields of many small shapes with every
buffer sized exactly; the parser on oracle blobs, their truncations and bit
flips, and header and section edits with their CRCs made valid again.
CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2312_05492_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2312_05492_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")


def _compiler(name):
    c = shutil.which(name)
    if not c:
        pytest.skip("%s not found" % name)
    return c


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("build failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


def test_oracle_core_under_sanitizers(tmp_path):
    exe = str(tmp_path / "szo_run")
    _build([_compiler("gcc"), "-std=c99", "-ffp-contract=off", *SAN, "-I", os.path.join(ROOT, "oracle"),
            os.path.join(NATIVE, "szo_run.c"), "-lm", "-o", exe])
    out = _run([exe])
    assert "0 failed" in out


def test_blob_parser_under_sanitizers(tmp_path):
    exe = str(tmp_path / "blob_fuzz")
    _build([_compiler("g++"), "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            os.path.join(CSRC, "blob.cpp"), os.path.join(NATIVE, "blob_fuzz.cpp"), "-o", exe])
    O.build(force=False)
    cases = [
        # a smooth 2D field: its words are elided
        (synth.climate_field(931, shape=(90, 180)), dict(eb=1e-3)),
        # a rough 3D field: words as they are, outliers at a tight bound
        (synth.spectral_field((20, 24, 40), seed=932), dict(eb=1e-5)),
        # an odd radius and a small chunk
        (synth.spectral_field((17, 33, 50), seed=933, beta=3.0), dict(eb=1e-3, R=3, chunk=256)),
    ]
    files = []
    flags = []
    for k, (x, kw) in enumerate(cases):
        blob = O.compress(x, O.Params(shape=x.shape, **kw)).blob()
        flags.append(int(np.frombuffer(blob[124:128], dtype="<u4")[0]))
        f = tmp_path / ("case%d.szi" % k)
        f.write_bytes(blob)
        files.append(str(f))
    assert flags[0] == O.FLAG_WORDS_ELIDED and flags[1] == 0   # both word forms are covered
    out = _run([exe, *files])
    assert "0 failed" in out
