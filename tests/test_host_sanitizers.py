"""Sanitized host builds: the library's block-space map header (the same inline
code the kernels run) and the C oracle, compiled with AddressSanitizer and
UndefinedBehaviorSanitizer by the host compilers and run on the CPU."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _build_and_run(cmd, exe):
    subprocess.check_call(cmd, cwd=os.path.dirname(exe))
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_maps_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check_maps")
        _build_and_run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_1610_07394_amd", "csrc"),
                        "-o", exe, os.path.join(HOST, "check_maps.cpp")], exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check_oracle")
        _build_and_run(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off", "-o", exe,
                        os.path.join(HOST, "check_oracle.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"],
                       exe)
