"""Invariants of the work plans of the Gram (plan_gram, lower tiles) and of
the Hilbert coupling (plan_rect, every tile of an M x N product), both in
csrc/k_dgemm.hip, checked on the host: tests/gram_plan_check.cpp is compiled
against the built library and run for 15 Gram orders and 8 coupling shapes,
each with 5 CU counts.  Every tile of the product appears once, whole or as
all of its pieces; piece units are distinct and in range; the summing
entries name the split tiles; the XCDs hold the same number of tiles to
within one; the pieces of each XCD fit in one round of its resident
workgroups.  Pure host code: no device is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2509_14185_amd")
LIB = os.path.join(PKG, "libgn.so")


def test_gram_plan_invariants(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not installed")
    assert os.path.exists(LIB), "libgn.so is missing: run __graft_entry__.build() first"
    exe = str(tmp_path / "gram_plan_check")
    cmd = [hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "gram_plan_check.cpp"), "-o", exe, "-L", PKG, "-lgn", f"-Wl,-rpath,{PKG}"]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "all invariants hold" in r.stdout
