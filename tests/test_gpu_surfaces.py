"""One cast through several stop surfaces (maps at several source redshifts
from one run) against the oracle's multi-surface cast."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare, run_gpu

pytestmark = pytest.mark.gpu

COSMO = (0.3, 0.7, 0.7)


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2111_08744_amd as M
    return M


def _print(*a):
    print(*a, flush=True)


def _blocks(g, n, nb):
    return [{k: v[b * n:(b + 1) * n] for k, v in g.items()} for b in range(nb)]


@pytest.mark.parametrize("grid_name,obs,zs,spc,adaptive", [
    ("gauss64", [250.0, 250.0, 250.0], [0.2, 0.5, 0.9], 10, False),
    ("amr_halo_small", [125.0, 125.0, 125.0], [0.1, 0.25, 0.4], 4, True)])
def test_surfaces_match_oracle(M, grid_name, obs, zs, spc, adaptive):
    cells = synth.make_cells(grid_name)
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(obs, zs[-1], 8, steps_per_cell=spc, adaptive=adaptive, surfaces=zs[:-1])
    _print("surfaces", zs, grid_name)
    g = run_gpu(grid, cfg)
    n = 768
    p = O.params(obs, z_src=zs[0], steps_per_cell=spc, adaptive=adaptive)
    o = O.cast_surfaces(O.Field.grid(cells), O.cosmo(*COSMO), p, zs, O.pix2vec_nest(8, np.arange(n)))
    blocks = _blocks(g, n, len(zs))
    for k in range(len(zs)):
        _print(f"surface {k} (z = {zs[k]}):", compare(blocks[k], o[k]))
    # up to the first landing a multi-surface ray is the single-surface ray
    first = run_gpu(grid, M.CastConfig(obs, zs[0], 8, steps_per_cell=spc, adaptive=adaptive))
    for k in ("beta", "z5", "n_steps", "hash", "status", "alpha", "phi_src"):
        assert np.array_equal(blocks[0][k], first[k]), k
    assert (np.diff(np.stack([b["n_steps"] for b in blocks]), axis=0) > 0).all()


def test_surfaces_argument_errors(M):
    cells = synth.make_cells("gauss64")
    grid = M.Grid(cells, COSMO)
    obs = [250.0, 250.0, 250.0]
    for bad in ([0.5, 0.2], [0.3, 0.9], [0.0]):          # not increasing; beyond the stop; z = 0
        with pytest.raises(RuntimeError):
            M.cast(grid, M.CastConfig(obs, 0.8, 2, surfaces=bad))
    with pytest.raises(RuntimeError):
        M.cast(grid, M.CastConfig(obs, 0.8, 2, surfaces=[0.3], checkpoint_every=32))
