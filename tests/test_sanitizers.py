"""Host code under AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer.

Two programs are built with gcc/g++ and the sanitizers on, and run on small
seeded point sets (CPU only):
- the oracle (every exported routine), with the tree-walk product checked
  against the dense K~ it defines (Section 2.1);
- the library's host-only code: the inspector (Section 3.1 compression and
  Section 5 inspector-p1) and the representation reader and validator, fed the
  inspector's own files and truncated or byte-damaged copies of them.

Any invalid access, leak or undefined operation aborts the program and fails
the test.  The library's sources are compiled as plain C++: the two files used
here make no HIP calls.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1812_07152_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
       "-fsanitize=address,undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, f"{' '.join(map(str, cmd[:3]))} ... failed:\n{p.stdout[-2000:]}\n{p.stderr[-6000:]}"
    return p


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    _run(["gcc", "-std=c99", "-fopenmp", *SAN, os.path.join(ROOT, "oracle", "hm_oracle.c"),
          os.path.join(HERE, "oracle_main.c"), "-o", str(exe), "-lm"])
    p = _run([str(exe), str(tmp_path / "oracle.hmc")], env=ENV, timeout=300)
    assert "oracle sanitizer run ok" in p.stdout


def test_host_inspector_and_reader_under_sanitizers(tmp_path):
    # the library's host-only sources, as C++ files of the build directory
    srcs = []
    for name in ("hm_inspect", "hm_store"):
        dst = tmp_path / (name + ".cpp")
        shutil.copy(os.path.join(CSRC, name + ".hip"), dst)
        srcs.append(str(dst))
    exe = tmp_path / "host_san"
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
          *srcs, os.path.join(HERE, "host_main.cpp"), "-o", str(exe), "-lpthread"])
    p = _run([str(exe), str(tmp_path)], env=ENV, timeout=600)
    assert "host sanitizer run ok" in p.stdout
