"""The library's host code (octree, interaction lists, operator cache) and the oracle's C helpers
built with AddressSanitizer and UndefinedBehaviorSanitizer by the host compilers (g++, gcc; no
GPU code) and run over ordinary and edge-case inputs: any out-of-bounds access, use after free,
leak or undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_02043_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-fopenmp"]


def _run(exe, cwd):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([str(exe)], cwd=cwd, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_code_under_sanitizers(tmp_path):
    exe = tmp_path / "host_code_asan"
    subprocess.run(["g++", "-std=c++17"] + SAN + ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                    os.path.join(CSRC, "tree_host.cpp"), os.path.join(CSRC, "opcache.cpp"),
                    os.path.join(ROOT, "tests", "sanitize", "host_code_asan.cpp"), "-o", str(exe)], check=True)
    assert "ok" in _run(exe, tmp_path)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_c_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_c_asan"
    subprocess.run(["gcc", "-std=c11"] + SAN + [os.path.join(ROOT, "oracle", "csrc", "direct.c"),
                    os.path.join(ROOT, "oracle", "csrc", "ewald_tp.c"),
                    os.path.join(ROOT, "tests", "sanitize", "oracle_c_asan.c"), "-o", str(exe), "-lm"], check=True)
    assert "ok" in _run(exe, tmp_path)
