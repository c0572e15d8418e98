"""GPU casts to iso-chi, iso-lambda and iso-z surfaces (Sect. 2.4: maps on
iso-p surfaces at the values of an FLRW photon) against the oracle, and the
finite beam stopped on such a surface (Sect. 2.3.2: the beam's rays may stop
on another parameter than the reference)."""
import numpy as np
import pytest

import oracle as O
import synth
from oracle import lensing as OL
from parity import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

COSMO = (0.3, 0.7, 0.7)
SURF = {"chi": O.SURF_CHI, "lambda": O.SURF_LAMBDA, "z": O.SURF_Z}


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2111_08744_amd as M
    return M


def _print(*a):
    print(*a, flush=True)


def _oracle(cells, obs, z, nside, spc, adaptive, surface):
    n = 12 * nside * nside
    p = O.params(obs, z_src=z, steps_per_cell=spc, adaptive=adaptive, surface=surface)
    return O.cast(O.Field.grid(cells), O.cosmo(*COSMO), p, O.pix2vec_nest(nside, np.arange(n)))


@pytest.mark.parametrize("name", ["chi", "lambda", "z"])
def test_uniform_grid_surfaces(M, name):
    """768 rays (nside 8) to the z = 0.5 surface of each kind on the 64^3
    grid: the same parity bar as the iso-eta casts, z0 (from each end
    point's own scale factor) with the relative bar of z5."""
    cells = synth.make_cells("gauss64")
    obs = [250.3, 249.6, 250.9]
    grid = M.Grid(cells, COSMO)
    _print(f"iso-{name} cast: uniform 64^3, nside 8, z = 0.5")
    g = run_gpu(grid, M.CastConfig(obs, 0.5, 8, steps_per_cell=10, stop_surface=name))
    o = _oracle(cells, obs, 0.5, 8, 10, False, SURF[name])
    _print(compare(g, o, z0_own=True))
    if name == "z":
        assert np.abs(g["z5"] - 0.5).max() < 1e-9
    if name == "chi":
        cz = O.cosmo(*COSMO)
        assert np.abs(g["chi"] / (O.eta0(cz) - O.eta_of_a(cz, 1 / 1.5)) - 1).max() < 1e-9


@pytest.mark.parametrize("name", ["chi", "z"])
def test_amr_surfaces(M, name):
    """The refined halo grid with adaptive steps (rays near level boundaries
    may take the other branch: at most 2 %)."""
    cells = synth.make_cells("amr_halo_small")
    obs = [125.3, 124.6, 125.9]
    grid = M.Grid(cells, COSMO)
    g = run_gpu(grid, M.CastConfig(obs, 0.3, 4, steps_per_cell=4, adaptive=True, stop_surface=name))
    o = _oracle(cells, obs, 0.3, 4, 4, True, SURF[name])
    _print(f"iso-{name} AMR:", compare(g, o, z0_own=True))


def test_finite_beam_on_chi_surface(M):
    """Finite-beam matrices with every ray of the beam stopped on the iso-chi
    surface, against the oracle's four-ray beams on the same surface (bar as
    for the iso-eta beams)."""
    cells = synth.make_cells("gauss64")
    obs = [250.0, 250.0, 250.0]
    eps = 5e-3
    grid = M.Grid(cells, COSMO)
    res = M.finite_beam(grid, M.CastConfig(obs, 0.5, 4, steps_per_cell=10, stop_surface="chi"), eps)
    A = res["A"].cpu().numpy().astype(np.float64)
    assert (res["status"].cpu().numpy() == 0).all()
    field = O.Field.grid(cells)
    p = O.params(obs, z_src=0.5, steps_per_cell=10, surface=O.SURF_CHI)
    Ao, _ = OL.finite_beam(lambda d: O.cast(field, O.cosmo(*COSMO), p, d), O.pix2vec_nest(4, np.arange(192)), eps)
    d = np.abs(A - Ao).max()
    _print(f"iso-chi finite beam: max |A - A_oracle| {d:.3e}")
    assert np.abs(Ao - np.eye(2)).max() > 1e-3
    assert d < 2e-6


def test_surface_rejections(M):
    cells = synth.make_cells("gauss32")
    grid = M.Grid(cells, COSMO)
    obs = [125.0, 125.0, 125.0]
    for kw in ({"order": 2}, {"checkpoint_every": 8}, {"surfaces": [0.1]}):
        with pytest.raises(M.MpathError):
            M.cast(grid, M.CastConfig(obs, 0.3, 2, steps_per_cell=4, stop_surface="chi", **kw))
    cfg = M.CastConfig(obs, 0.3, 2, steps_per_cell=4, stop_surface="lambda")
    with pytest.raises(M.MpathError):
        M.infinitesimal_beam(grid, cfg)
    with pytest.raises(M.MpathError):
        M.born_beam(grid, cfg)
    with pytest.raises(M.MpathError):
        M.cast(grid, M.CastConfig(obs, 0.3, 2, stop_surface=9))
    static = M.Grid(cells, (0.0, 0.0, 0.7))
    with pytest.raises(M.MpathError):
        M.cast(static, M.CastConfig(obs, 50.0, 2, stop_kind="chi", stop_surface="z"))
