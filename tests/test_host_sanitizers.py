"""Host code under the address and undefined-behaviour sanitizers (CPU only).

Two programs under ``tests/sanitize/`` are built here with
``-fsanitize=address,undefined -fno-sanitize-recover=all`` and run:

* ``host_tables_check.cpp`` with the library's host-only plan construction
  (``csrc/tables.cpp``, ``csrc/geometry.cpp``): sweep tables, backprojector
  tile lists, CSR and the stored copies on seven geometries, with the
  invariants the kernels rely on, and the argument rejections;
* ``oracle_check.c`` with the FP64 oracle (``oracle/eptv_oracle.c``, OpenMP on
  two threads): every entry point on three small geometries, every
  reconstruct variant with every stats array.

Any sanitizer report aborts the program, which fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1009_2288_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r.stdout


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "abort_on_error=0:halt_on_error=1:detect_leaks=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    return env


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_tables_check")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{CSRC}",
          os.path.join(CSRC, "tables.cpp"), os.path.join(CSRC, "geometry.cpp"),
          os.path.join(ROOT, "tests", "sanitize", "host_tables_check.cpp"), "-o", exe])
    out = _run([exe], env=_env())
    assert "all checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c99", *SAN, "-fopenmp", f"-I{os.path.join(ROOT, 'oracle')}",
          os.path.join(ROOT, "oracle", "eptv_oracle.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
          "-o", exe, "-lm"])
    out = _run([exe], env=_env())
    assert "all checks passed" in out
