"""The TSC stencil resolution of the GPU path (Sect. 2.2, W_TSC with the
level fallback; TscCache::gather in device.h) built for the host and checked
against 27 direct octree lookups per stencil on random periodic and
non-periodic trees (tests/host/tsc_ids_check.cpp).  The ids at level 0 come
from per-axis Morton spreads and those at refined levels from the 8 shared
parents; a wrong spread, parent choice or octant bit gives another cell's
payload and fails here."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_tsc_ids_match_direct_lookups(tmp_path):
    exe = str(tmp_path / "tsc_ids_check")
    cmd = [HIPCC, "-x", "hip", "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "paper_2111_08744_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "tsc_ids_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
    assert "0 mismatches" in r.stdout, r.stdout
