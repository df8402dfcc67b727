"""The C ABI from plain C: tests/c_abi/ooc_example.c is compiled with gcc
against include/ooc.h and linked with the built library (no Python in the
call path).  On the CPU only compiling and linking is checked; on the GPU the
program runs a tiled product (FP64, then split-BF16 and split-INT8), a
Cholesky factorisation and a Cholesky solve, and checks them exactly."""
import os
import subprocess

import pytest

import paper_1808_05056_amd as ooc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_abi", "ooc_example.c")


def _build(tmp_path):
    exe = str(tmp_path / "ooc_example")
    libdir = os.path.dirname(ooc.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), SRC, "-o", exe,
           "-L", libdir, "-looc", f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    return exe


def test_c_example_compiles_and_links(tmp_path):
    assert os.path.exists(_build(tmp_path))


@pytest.mark.gpu
def test_c_example_runs(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout
