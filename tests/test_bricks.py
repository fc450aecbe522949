"""Host check (no GPU) that the stencil sweeps cover the lattice: a small program compiled
against the library's headers and linked to liba2a.so runs the library's own brick choice and
both sweep orders on the workload lattices and the shapes the GPU tests use, and finds every
checkerboard site of a parity visited exactly once."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1405_4524_amd", "_build")
LATTICES = [(32, 32, 32, 64), (24, 24, 24, 48), (16, 16, 16, 32), (8, 8, 8, 16), (4, 4, 4, 8), (2, 2, 2, 2),
            (4, 2, 6, 4), (6, 4, 4, 10), (8, 8, 8, 8), (4, 4, 6, 8), (2, 2, 2, 4), (4, 2, 2, 8), (12, 12, 12, 24),
            (6, 4, 4, 12)]


def test_stencil_sweeps_visit_every_site_once(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    lib = os.path.join(BUILD, "liba2a.so")
    if not os.path.exists(hipcc) or not os.path.exists(lib):
        pytest.skip("hipcc or the built library is missing")
    exe = str(tmp_path / "brick_check")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_1405_4524_amd", "csrc"),
                           os.path.join(ROOT, "tests", "brick_check.cpp"), "-L", BUILD, "-la2a",
                           "-Wl,-rpath," + BUILD, "-o", exe], stderr=subprocess.DEVNULL)
    args = [str(d) for lat in LATTICES for d in lat]
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.strip().splitlines()
    assert len(lines) == len(LATTICES) and all(line.endswith("bijection") for line in lines), r.stdout
