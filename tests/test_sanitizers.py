"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code (no GPU).

* The FP64 oracle (plain C) with gcc -fsanitize=address,undefined, driven over
  every point-set kind, randomisation and map in bases 2 and 3
  (tests/sanitize/oracle_driver.c).
* The HIP library's host code (argument validation, level planning, the C ABI)
  with the sanitizers on the host side only (-Xarch_host), driven through every
  refusal path of the ABI, which ends before any device call
  (tests/sanitize/host_driver.cpp).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2305_11645_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
          "-O1", "-std=c11", "-ffp-contract=off", "-fopenmp", os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"])
    res = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "4"}, timeout=300)
    assert "oracle driver: ok" in res.stdout


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC] + SAN_HOST
    srcs = [f for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_driver")
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include")] + SAN_HOST
         + ["-x", "c++", os.path.join(HERE, "host_driver.cpp"), "-x", "none"] + objs + ["-o", exe])
    # leak checking is off: the HIP runtime keeps process-lifetime allocations
    res = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"}, timeout=300)
    assert "host driver: ok" in res.stdout
