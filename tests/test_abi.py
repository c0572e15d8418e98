"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/mpath.h declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpath.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpath_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_2111_08744_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libmpath.so is not built (python -m paper_2111_08744_amd.build)")
    return _abi


def test_exports_every_declared_symbol(abi):
    L = abi.lib()
    names = declared_symbols()
    assert "mpath_cast" in names and "mpath_grid_build" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_status_strings(abi):
    L = abi.lib()
    assert b"gfx950" in L.mpath_version()
    assert L.mpath_status_string(abi.MPATH_ERR_NOT_FULL_TREE) == b"not a full octree"


def _desc(abi, n0=4, level=None, ijk=None, max_level=0):
    d = abi.mpath_grid_desc()
    d.box, d.n0, d.max_level, d.periodic, d.value_dtype = 100.0, n0, max_level, 1, abi.MPATH_F64
    if level is None:
        ii, jj, kk = np.meshgrid(*(np.arange(n0),) * 3, indexing="ij")
        ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int32)
        level = np.zeros(len(ijk), np.uint8)
    phi = np.zeros(len(level))
    grad = np.zeros((len(level), 3))
    keep = (level, ijk, phi, grad)
    d.n_cells = len(level)
    d.level, d.ijk, d.phi, d.grad = (a.ctypes.data for a in keep)
    return d, keep


def test_workspace_size_and_argument_checks(abi):
    L = abi.lib()
    n = C.c_size_t()
    d, keep = _desc(abi)
    assert L.mpath_grid_workspace_bytes(C.byref(d), C.byref(n)) == abi.MPATH_OK
    assert n.value >= 64 * (16 + 4 + 8)
    d.n0 = 3    # not a power of two
    assert L.mpath_grid_workspace_bytes(C.byref(d), C.byref(n)) == abi.MPATH_ERR_INVALID_ARG
    assert b"power of two" in L.mpath_last_error()
    d, keep = _desc(abi)
    d.value_dtype = 7
    assert L.mpath_grid_workspace_bytes(C.byref(d), C.byref(n)) == abi.MPATH_ERR_INVALID_ARG
    d, keep = _desc(abi)
    d.n_cells = 10      # fewer than the coarse grid
    assert L.mpath_grid_workspace_bytes(C.byref(d), C.byref(n)) == abi.MPATH_ERR_NOT_FULL_TREE
    assert L.mpath_grid_workspace_bytes(None, C.byref(n)) == abi.MPATH_ERR_INVALID_ARG


def test_grid_build_rejects_bad_trees_before_any_device_work(abi):
    """Tree validation runs on the host before any upload."""
    L = abi.lib()
    ii, jj, kk = np.meshgrid(*(np.arange(4),) * 3, indexing="ij")
    coarse = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int32)
    kids = np.array([[2 * 1 + (o & 1), 2 * 2 + ((o >> 1) & 1), 2 * 3 + (o >> 2)] for o in range(8)], np.int32)
    cz = abi.mpath_cosmo(0.3, 0.7, 0.7)
    h = C.c_void_p()
    for bad_kids, code in [(kids[:7], abi.MPATH_ERR_NOT_FULL_TREE),                       # 7 children
                           (np.concatenate([kids[:7], kids[:1]]), abi.MPATH_ERR_NOT_FULL_TREE)]:  # repeat
        ijk = np.concatenate([coarse, bad_kids])
        level = np.concatenate([np.zeros(64, np.uint8), np.ones(len(bad_kids), np.uint8)])
        d, keep = _desc(abi, 4, level, ijk, max_level=1)
        big = 1 << 20
        rc = L.mpath_grid_build(C.byref(d), C.byref(cz), C.c_void_p(1), big, None, C.byref(h))
        assert rc == code, L.mpath_last_error()
    # non-flat cosmology
    d, keep = _desc(abi)
    cz2 = abi.mpath_cosmo(0.3, 0.6, 0.7)
    assert L.mpath_grid_build(C.byref(d), C.byref(cz2), C.c_void_p(1), 1 << 20, None, C.byref(h)) == \
        abi.MPATH_ERR_UNSUPPORTED
    # workspace too small
    assert L.mpath_grid_build(C.byref(d), C.byref(cz), C.c_void_p(1), 16, None, C.byref(h)) == \
        abi.MPATH_ERR_WORKSPACE_TOO_SMALL


def test_count_rays(abi):
    from paper_2111_08744_amd import CastConfig
    cfg = CastConfig([[0, 0, 0], [1, 1, 1]], [0.5, 1.0], 4, pix_first=[0, 10], pix_count=[5, 7])
    assert cfg.n_rays() == 12
    assert CastConfig([0, 0, 0], 0.5, 16).n_rays() == 3072


def test_gather_probe_argument_checks(abi):
    """Every rejected argument returns before any launch (the table pointer
    here is never dereferenced)."""
    L = abi.lib()
    fake = C.c_void_p(1 << 20)
    out = C.c_void_p(1 << 21)
    ok = dict(table=fake, nbytes=1 << 16, rec=64, u=4, waves=8, iters=2)
    cases = [dict(table=None), dict(table=C.c_void_p((1 << 20) + 8)), dict(rec=32), dict(nbytes=32),
             dict(u=3), dict(waves=0), dict(waves=(1 << 24) + 1), dict(iters=0)]
    for bad in cases:
        a = {**ok, **bad}
        rc = L.mpath_gather_probe(a["table"], a["nbytes"], a["rec"], a["u"], a["waves"], a["iters"], 1, out, None)
        assert rc == abi.MPATH_ERR_INVALID_ARG, (bad, L.mpath_last_error())
    assert L.mpath_gather_probe(fake, 1 << 16, 64, 4, 8, 2, 1, None, None) == abi.MPATH_ERR_INVALID_ARG


def test_lensing_entry_points_reject_bad_arguments(abi):
    """Checked before any device work (no grid or device memory is touched)."""
    L = abi.lib()
    fake = C.c_void_p(1 << 20)
    assert L.mpath_lensing_maps(fake, -1, fake, None) == abi.MPATH_ERR_INVALID_ARG
    assert L.mpath_lensing_maps(None, 4, fake, None) == abi.MPATH_ERR_INVALID_ARG
    assert L.mpath_lensing_maps(None, 0, None, None) == abi.MPATH_OK
    from paper_2111_08744_amd import CastConfig
    d = CastConfig([0, 0, 0], 0.5, 4).desc()
    n = C.c_size_t()
    assert L.mpath_finite_beam_workspace_bytes(None, C.byref(d), C.byref(n)) == abi.MPATH_ERR_INVALID_ARG
    for eps in (0.0, -1e-3, 0.2, float("nan")):
        assert L.mpath_finite_beam(fake, C.byref(d), eps, fake, None, fake, 1 << 30, None) == \
            abi.MPATH_ERR_INVALID_ARG


def test_caller_directions_ray_count(abi):
    """With caller directions pix_count alone sets the rays per observer."""
    import torch
    from paper_2111_08744_amd import CastConfig
    cfg = CastConfig([[0, 0, 0], [1, 1, 1]], [0.5, 1.0], 4, pix_count=[500, 7])
    cfg.dirs = torch.zeros((507, 3), dtype=torch.float64)   # any non-NULL pointer: only counted here
    d = cfg.desc()
    assert d.dirs and not d.pix_first
    assert cfg.n_rays() == 507


def test_finder_rejects_missing_arguments(abi):
    L = abi.lib()
    d = abi.mpath_finder_desc()
    n = C.c_size_t()
    assert L.mpath_find_geodesics_workspace_bytes(None, C.byref(d), C.byref(n)) == abi.MPATH_ERR_INVALID_ARG
    assert L.mpath_find_geodesics_workspace_bytes(C.c_void_p(1 << 20), None, C.byref(n)) == \
        abi.MPATH_ERR_INVALID_ARG
    o = abi.mpath_finder_out()
    assert L.mpath_find_geodesics(None, C.byref(d), C.byref(o), None, 0, None) == abi.MPATH_ERR_INVALID_ARG


def test_born_beam_rejects_missing_grid(abi):
    L = abi.lib()
    from paper_2111_08744_amd import CastConfig
    d = CastConfig([0, 0, 0], 0.5, 4).desc()
    assert L.mpath_born_beam(None, C.byref(d), None, None, None, 0, None) == abi.MPATH_ERR_INVALID_ARG


def test_healpix_dirs_argument_checks(abi):
    """Rejected before any device work: nside outside [1, 8192], a pixel
    range outside the sky, no output array."""
    L = abi.lib()
    for nside, first, count, ptr in ((0, 0, 1, 16), (8193, 0, 1, 16), (2, -1, 1, 16), (2, 40, 9, 16), (2, 0, 4, None)):
        assert L.mpath_healpix_dirs(nside, first, count, ptr, None) == abi.MPATH_ERR_INVALID_ARG, (nside, first, count)
