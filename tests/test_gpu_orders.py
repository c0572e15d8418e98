"""NGP and TSC casts (Sect. 2.2, W_NGP and W_TSC with the level fallback)
against the FP64 oracle with the same interpolation order."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare, run_gpu, run_oracle

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


@pytest.mark.parametrize("order", [0, 2])
def test_uniform_orders_match_oracle(M, order):
    """64^3 grid, 768 rays (nside 8) to z = 0.5, 10 steps per cell.  With NGP
    the field jumps at cell faces, so a ray whose float32 position sits
    within rounding of a face may read the other cell; such rays are rare."""
    cells = synth.make_cells("gauss64")
    obs = [250.0, 250.0, 250.0]
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(obs, 0.5, 8, steps_per_cell=10, order=order)
    _print("order", order, "uniform 64^3, nside 8, z = 0.5")
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(cells, order=order), O.cosmo(*COSMO), obs, 0.5, 8, [0], [768], 10, False)
    s = compare(g, o)
    _print(s)
    cic = run_gpu(grid, M.CastConfig(obs, 0.5, 8, steps_per_cell=10))
    assert not np.array_equal(cic["beta"], g["beta"])          # a different interpolant


@pytest.mark.parametrize("order", [0, 2])
def test_amr_orders_match_oracle(M, order):
    """Refined grid, adaptive steps: the TSC fallback is taken per leaf cell."""
    cells = synth.make_cells("amr_halo_small")
    obs = [125.0, 125.0, 125.0]
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(obs, 0.4, 8, steps_per_cell=4, adaptive=True, order=order)
    _print("order", order, "amr halo small, nside 8, z = 0.4")
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(cells, order=order), O.cosmo(*COSMO), obs, 0.4, 8, [0], [768], 4, True)
    _print(compare(g, o))


def test_orders_finite_beam_and_unsupported_paths(M):
    """A finite beam with TSC rays; checkpoints (the adjoint) and the
    infinitesimal beam are CIC only."""
    cells = synth.make_cells("gauss64")
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig([250.0, 250.0, 250.0], 0.3, 2, steps_per_cell=10, order=2)
    res = M.finite_beam(grid, cfg, 5e-3)
    A = res["A"].cpu().numpy()
    assert np.isfinite(A).all() and (res["status"].cpu().numpy() == 0).all()
    with pytest.raises(RuntimeError):
        M.cast(grid, M.CastConfig([250.0, 250.0, 250.0], 0.3, 2, order=2, checkpoint_every=32))
    with pytest.raises(RuntimeError):
        M.infinitesimal_beam(grid, cfg)
    with pytest.raises(RuntimeError):
        M.cast(grid, M.CastConfig([250.0, 250.0, 250.0], 0.3, 2, order=3))
