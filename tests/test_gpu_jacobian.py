"""Forward-mode distortion matrix (mpath_cast_jacobian): the two tangents of
every ray carried through the cast give A = d beta / d theta and dz5/dtheta
of the same discrete map as the reverse sweep, checked against the oracle's
complex-step Jacobian (the bars of the reverse-sweep tests: largest |dA|
5e-6, median 2e-7; dz/dtheta 1e-5 of its scale), against the reverse sweep
itself, and the cast's own outputs against the plain cast bit for bit."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import oracle_dirs

pytestmark = pytest.mark.gpu

COSMO = (0.3, 0.7, 0.7)
OBS = [250.0, 250.0, 250.0]


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2111_08744_amd as M
    return M


@pytest.fixture(scope="module")
def gauss64():
    return synth.make_cells("gauss64")


def _np(t):
    return t.detach().cpu().numpy()


def _run(M, grid, cfg):
    import torch
    out = M.jacobian(grid, cfg)
    torch.cuda.synchronize()
    return out


def _check(M, grid, cells, cfg, p, dirs, tag):
    """Tangent A and dz/dtheta against the oracle's complex step."""
    import torch
    out = _run(M, grid, cfg)
    ref = M.cast(grid, cfg)
    torch.cuda.synchronize()
    for k in ("beta", "alpha", "z5", "phi_src", "n_steps", "status", "hash"):
        assert torch.equal(out[k], ref[k]) or np.array_equal(_np(out[k]), _np(ref[k]), equal_nan=True), k
    jac = _np(out["jac"]).astype(np.float64)
    dz = _np(out["dz_dtheta"]).astype(np.float64)
    A, dzo, rec = O.jacobian_cs(lambda d, t: O.cast_cs(O.Field.grid(cells), O.cosmo(*COSMO), p, d, dtheta=t), dirs)
    assert np.array_equal(_np(out["hash"]).view(np.uint32), rec["hash"])
    assert np.all(rec["status"] == O.REACHED)
    dA = np.abs(jac - A).reshape(-1, 4).max(1)
    lens = np.abs(A - np.eye(2)).reshape(-1, 4).max(1)
    rz = np.abs(dz - dzo).max(1) / np.abs(dzo).max()
    print(f"{tag}: {len(dirs)} rays, |A - I| up to {lens.max():.2e}; |A_tan - A_oracle| max {dA.max():.2e} "
          f"median {np.median(dA):.2e}; dz/dtheta rel max {rz.max():.2e}", flush=True)
    assert lens.max() > 1e-4
    assert dA.max() < 5e-6 and np.median(dA) < 2e-7
    assert rz.max() < 1e-5
    return out


def test_tangent_jacobian_uniform(M, gauss64):
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(OBS, 0.3, 4, steps_per_cell=10)
    _check(M, grid, gauss64, cfg, O.params(OBS, z_src=0.3, steps_per_cell=10), oracle_dirs(4, [0], [192]), "uniform")


def test_tangent_jacobian_amr(M):
    cells = synth.random_amr_cells(16, 125.0, 3, seed=5)
    grid = M.Grid(cells, COSMO)
    obs = [40.0, 70.0, 90.0]
    cfg = M.CastConfig(obs, 0.1, 2, steps_per_cell=4, adaptive=True)
    _check(M, grid, cells, cfg, O.params(obs, z_src=0.1, steps_per_cell=4, adaptive=True), oracle_dirs(2, [0], [48]),
           "random AMR tree")


def test_tangent_jacobian_deep_amr(M):
    """Five refinement levels around haloes (the depth of the 512^3 + 5 level
    light cone)."""
    cells = synth.make_cells("amr_deep")
    grid = M.Grid(cells, COSMO, aux=False)
    cfg = M.CastConfig(OBS, 0.3, 4, pix_first=[0], pix_count=[48], steps_per_cell=4, adaptive=True)
    _check(M, grid, cells, cfg, O.params(OBS, z_src=0.3, steps_per_cell=4, adaptive=True),
           O.pix2vec_nest(4, np.arange(48)), "five levels")


def test_tangent_matches_reverse_sweep(M, gauss64):
    """The same derivative by the two modes: forward tangents and the
    checkpointed reverse sweep, on 3072 rays (rounding differs: float32
    stage arithmetic on either side)."""
    import torch
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(OBS, 0.5, 16, steps_per_cell=10, checkpoint_every=32)
    fwd = M.cast(grid, cfg)
    rev = M.adjoint(grid, cfg, fwd, jacobian=True)
    cfg0 = M.CastConfig(OBS, 0.5, 16, steps_per_cell=10)
    tan = _run(M, grid, cfg0)
    torch.cuda.synchronize()
    d = np.abs(_np(tan["jac"]).astype(np.float64) - _np(rev["jac"]).astype(np.float64)).reshape(-1, 4).max(1)
    dz = np.abs(_np(tan["dz_dtheta"]).astype(np.float64) - _np(rev["dz_dtheta"]).astype(np.float64)).max(1)
    scale = np.abs(_np(rev["dz_dtheta"])).max()
    print(f"tangent vs reverse: |dA| max {d.max():.2e} median {np.median(d):.2e}; dz/dtheta {dz.max() / scale:.2e}",
          flush=True)
    assert d.max() < 5e-6 and np.median(d) < 2e-7
    assert dz.max() < 1e-5 * scale


def test_tangent_edge_cases(M, gauss64):
    """Rays that leave a non-periodic box get NaN derivatives; an empty ray
    list casts nothing; unsupported options are refused."""
    import torch
    from paper_2111_08744_amd import _abi
    cells = synth.random_amr_cells(16, 125.0, 2, seed=8, periodic=False)
    grid = M.Grid(cells, COSMO)
    out = _run(M, grid, M.CastConfig([60.0, 62.0, 58.0], 0.2, 4, steps_per_cell=4, adaptive=True))
    st = _np(out["status"])
    assert np.all(st == M.MPATH_RAY_LEFT_DOMAIN)
    assert np.all(np.isnan(_np(out["jac"]))) and np.all(np.isnan(_np(out["dz_dtheta"])))
    g64 = M.Grid(gauss64, COSMO)
    empty = _run(M, g64, M.CastConfig([[250.0, 250.0, 250.0]], [0.3], 4, [0], [0], steps_per_cell=10))
    assert empty["jac"].shape == (0, 2, 2)
    with pytest.raises(_abi.MpathError):
        M.jacobian(g64, M.CastConfig(OBS, 0.3, 4, steps_per_cell=10, checkpoint_every=32))
    with pytest.raises(_abi.MpathError):
        M.jacobian(g64, M.CastConfig(OBS, 0.3, 4, steps_per_cell=10, order=2))
    with pytest.raises(_abi.MpathError):
        M.jacobian(g64, M.CastConfig(OBS, 300.0, 4, stop_kind="chi", steps_per_cell=10, stop_surface="chi"))
