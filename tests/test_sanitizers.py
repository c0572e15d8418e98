"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle's entry points on a small refined tree (gcc), and the host paths of
the library's C ABI (argument and tree validation, workspace sizes, the
host part of the grid build with central differences) with the host code
compiled by hipcc with the sanitizers on the host pass.  The drivers
live in tests/sanitize/; a sanitizer report aborts them."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.slow


def _write_grid(cells, path):
    with open(path, "wb") as f:
        f.write(np.float64(cells.box).tobytes())
        f.write(np.array([cells.n0, cells.max_level, int(cells.periodic)], np.int32).tobytes())
        f.write(np.int64(cells.n_cells).tobytes())
        f.write(np.ascontiguousarray(cells.level, np.uint8).tobytes())
        f.write(np.ascontiguousarray(cells.ijk, np.int32).tobytes())
        f.write(np.ascontiguousarray(cells.phi, np.float64).tobytes())
        f.write(np.ascontiguousarray(cells.grad, np.float64).tobytes())


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, (cmd[:3], r.stdout[-2000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
@pytest.mark.parametrize("periodic", [True, False])
def test_oracle_under_sanitizers(tmp_path, periodic):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=gnu11", "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "oracle"),
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          "-o", exe, "-lm", "-lpthread"])
    grid = str(tmp_path / "grid.bin")
    _write_grid(synth.random_amr_cells(8, 80.0, 2, seed=3, periodic=periodic), grid)
    r = _run([exe, grid], env=ENV)
    assert "oracle driver ok" in r.stdout


HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_abi_host_paths_under_sanitizers(tmp_path):
    """The library's sources built for gfx950 with the sanitizers on the host
    pass only (every -fsanitize behind -Xarch_host), linked with the driver;
    the device code is never launched."""
    from concurrent.futures import ThreadPoolExecutor
    csrc = os.path.join(ROOT, "paper_2111_08744_amd", "csrc")
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", *host_san, "-I", os.path.join(ROOT, "include")]
    srcs = [os.path.join(csrc, f) for f in ("mpath_host.cpp", "grid.hip", "cast.hip", "adjoint.hip", "lensing.hip",
                                            "finder.hip", "probe.hip")]
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"))
    objs = [str(tmp_path / (os.path.splitext(os.path.basename(s))[0] + ".o")) for s in srcs]
    with ThreadPoolExecutor(4) as ex:
        list(ex.map(lambda so: _run([HIPCC, *flags, "-c", so[0], "-o", so[1]]), zip(srcs, objs)))
    exe = str(tmp_path / "abi_driver")
    _run([HIPCC, "--offload-arch=gfx950", *host_san, *objs, "-o", exe])
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = _run([exe], env=env)
    assert "abi driver ok" in r.stdout
