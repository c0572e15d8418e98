"""GPU lensing products against the oracle: casts along caller-given initial
directions, the finite-beam distortion matrix (Sect. 2.3.2) and its
decomposition into convergence, shear, rotation and magnification
(Sect. 2.3)."""
import numpy as np
import pytest

import oracle as O
import synth
from oracle import lensing as OL
from parity import ARCSEC, beta_to_vec, compare, run_gpu

pytestmark = pytest.mark.gpu

COSMO = (0.3, 0.7, 0.7)
CENTRE = [250.0, 250.0, 250.0]


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


def _print(*a):
    print(*a, flush=True)


def _random_dirs(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_caller_directions_match_oracle(M, gauss64):
    """500 random initial directions (not pixel centres) to z = 0.5 on the
    64^3 grid: the same parity bar as the pixel casts."""
    dirs = _random_dirs(500, 11)
    _print("caller directions: 500 random rays, uniform 64^3, z = 0.5")
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(CENTRE, 0.5, 16, pix_count=[500], dirs=_cuda(dirs), steps_per_cell=10)
    g = run_gpu(grid, cfg)
    p = O.params(CENTRE, z_src=0.5, steps_per_cell=10, adaptive=False)
    o = O.cast(O.Field.grid(gauss64), O.cosmo(*COSMO), p, dirs)
    _print(compare(g, o))


def test_pixel_centres_as_caller_directions(M, gauss64):
    """Pixel centres passed as directions give the pixel cast (to the last
    bits of the two HEALPix evaluations)."""
    grid = M.Grid(gauss64, COSMO)
    a = run_gpu(grid, M.CastConfig(CENTRE, 0.3, 4, steps_per_cell=10))
    dirs = O.pix2vec_nest(4, np.arange(192))
    b = run_gpu(grid, M.CastConfig(CENTRE, 0.3, 4, pix_count=[192], dirs=_cuda(dirs), steps_per_cell=10))
    assert np.array_equal(a["n_steps"], b["n_steps"]) and np.array_equal(a["status"], b["status"])
    va, vb = beta_to_vec(a["beta"]), beta_to_vec(b["beta"])
    sep = np.arctan2(np.linalg.norm(np.cross(va, vb), axis=1), np.sum(va * vb, 1)) / ARCSEC
    assert sep.max() < 1e-6
    assert np.abs(a["z5"] - b["z5"]).max() < 1e-14


def _oracle_beam(cells, obs, z, dirs, eps):
    field = O.Field.grid(cells)
    c = O.cosmo(*COSMO)
    p = O.params(obs, z_src=z, steps_per_cell=10, adaptive=False)
    A, ref = OL.finite_beam(lambda d: O.cast(field, c, p, d), dirs, eps)
    return A, ref


def test_finite_beam_matches_oracle(M, gauss64):
    """Finite-beam matrices of 192 pixel rays (nside 4) to z = 0.5 with a
    semi-aperture of 5e-3 rad, against the oracle's four-ray beams.  The
    end points agree to the deflection bar (1e-3 arcsec), i.e. to about
    5e-9 chi; divided by 2 chi tan(eps) that bounds the matrix difference by
    about 1e-6."""
    eps = 5e-3
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(CENTRE, 0.5, 4, steps_per_cell=10)
    _print("finite beam: nside 4, z = 0.5, eps", eps)
    res = M.finite_beam(grid, cfg, eps)
    A = res["A"].cpu().numpy().astype(np.float64)
    assert (res["status"].cpu().numpy() == 0).all()
    Ao, ref = _oracle_beam(gauss64, CENTRE, 0.5, O.pix2vec_nest(4, np.arange(192)), eps)
    d = np.abs(A - Ao).max()
    lens = np.abs(Ao - np.eye(2)).max()
    _print(f"max |A - A_oracle| {d:.3e}, max |A_oracle - I| {lens:.3e}")
    assert lens > 1e-3          # the beams are lensed
    assert d < 2e-6


def test_finite_beam_ragged_observers_and_caller_directions(M, gauss64):
    """Two observers with different source redshifts and ray counts, caller
    directions: each beam lands in its own slot of the five-ray layout."""
    eps = 4e-3
    obs = np.array([[100.0, 200.0, 300.0], [400.0, 120.0, 60.0]])
    z = np.array([0.2, 0.45])
    counts = [37, 90]
    dirs = _random_dirs(sum(counts), 5)
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(obs, z, 16, pix_count=counts, dirs=_cuda(dirs), steps_per_cell=10)
    res = M.finite_beam(grid, cfg, eps)
    A = res["A"].cpu().numpy().astype(np.float64)
    assert (res["status"].cpu().numpy() == 0).all()
    starts = np.concatenate([[0], np.cumsum(counts)])
    for j in range(2):
        sl = slice(starts[j], starts[j + 1])
        Ao, _ = _oracle_beam(gauss64, obs[j], z[j], dirs[sl], eps)
        d = np.abs(A[sl] - Ao).max()
        _print(f"observer {j}: max |A - A_oracle| {d:.3e}")
        assert d < 2e-6


def test_finite_beam_empty(M, gauss64):
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(CENTRE, 0.5, 4, pix_first=[0], pix_count=[0], steps_per_cell=10)
    res = M.finite_beam(grid, cfg, 1e-3)
    assert res["A"].shape == (0, 2, 2)


def test_lensing_maps(M):
    """kappa, gamma, omega, mu of matrices composed from known values, and
    against the oracle's decomposition of the same float32 matrices."""
    import torch
    rng = np.random.default_rng(3)
    n = 4096
    k, g1, g2 = rng.normal(0, 0.05, (3, n))
    w = rng.normal(0, 0.02, n)
    A32 = OL.compose(k, g1, g2, w).astype(np.float32)
    out = M.lensing_maps(_cuda(A32)).cpu().numpy().astype(np.float64)
    ko, g1o, g2o, wo, muo = OL.decompose(A32.astype(np.float64))
    for col, ref in enumerate((ko, g1o, g2o, wo)):
        assert np.abs(out[:, col] - ref).max() < 1e-6, col
    assert np.abs(out[:, 4] / muo - 1).max() < 1e-6
    for col, ref in enumerate((k, g1, g2, w)):        # the composed values come back
        assert np.abs(out[:, col] - ref).max() < 1e-6, col
    assert M.lensing_maps(torch.empty((0, 2, 2), dtype=torch.float32, device="cuda")).shape == (0, 5)


def _inf_compare(M, cells, obs, z, nside, spc, adaptive, max_bad_frac=0.0):
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(obs, z, nside, steps_per_cell=spc, adaptive=adaptive)
    res = M.infinitesimal_beam(grid, cfg)
    A = res["A"].cpu().numpy().astype(np.float64)
    plain = run_gpu(grid, cfg)
    # the sampling leaves the integration itself untouched
    for k in ("beta", "z5", "n_steps", "status", "hash"):
        got = res[k].cpu().numpy()
        if k == "hash":
            got = got.view(np.uint32)
        assert np.array_equal(got, plain[k]), k
    n = 12 * nside * nside
    dirs = O.pix2vec_nest(nside, np.arange(n))
    p = O.params(obs, z_src=z, steps_per_cell=spc, adaptive=adaptive)
    Ao, rec = O.infinitesimal(O.Field.grid(cells), O.cosmo(*COSMO), p, dirs)
    ok = rec["status"] == O.REACHED
    assert np.array_equal(ok, plain["status"] == 0)
    d = np.abs(A[ok] - Ao[ok]).max(axis=(1, 2))
    lens = np.abs(Ao[ok] - np.eye(2)).max(axis=(1, 2))
    bad = d > 1e-6
    _print(f"infinitesimal beam: max |A - A_oracle| {d.max():.3e}, median {np.median(d):.3e}, "
           f"max |A_oracle - I| {lens.max():.3e}, {bad.sum()} of {ok.sum()} above 1e-6")
    assert lens.max() > 1e-3
    assert bad.sum() <= max_bad_frac * ok.sum()
    assert np.isnan(A[~ok]).all()
    return d


def test_infinitesimal_beam_matches_oracle_uniform(M, gauss64):
    """Uniform 64^3 grid, 192 rays (nside 4) to z = 0.5, 10 steps per cell:
    the Hessian comes from differences of the float32 interpolated force, so
    the matrices agree to about 1e-7 relative to the field scale."""
    _print("infinitesimal beam, uniform 64^3, nside 4, z = 0.5")
    _inf_compare(M, gauss64, CENTRE, 0.5, 4, 10, False)


def test_infinitesimal_beam_amr(M):
    """Refined grid with adaptive steps: the derivation step follows the leaf
    size.  A sample point within rounding of a leaf boundary may take the
    other leaf's step on one side; such rays must be rare."""
    cells = synth.make_cells("amr_halo_small")
    _print("infinitesimal beam, amr halo small, nside 4, z = 0.4")
    _inf_compare(M, cells, [125.0, 125.0, 125.0], 0.4, 4, 4, True, max_bad_frac=0.02)


@pytest.mark.parametrize("grid_name,obs,z,spc,adaptive", [
    ("gauss64", [250.3, 249.6, 250.9], 0.5, 10, False),
    ("amr_halo_small", [125.3, 124.6, 125.9], 0.4, 4, True)])
def test_born_beam_matches_oracle(M, grid_name, obs, z, spc, adaptive):
    """Born approximation along the straight lines of 192 pixel directions:
    the same samples as the oracle (the step rule along the line), so the
    matrices agree to the float32 field arithmetic; close to the
    infinitesimal beam along the actual geodesics (weak lensing).  The
    observer sits off the cell faces: from a point on a face, the lines of
    the equatorial pixels run inside that face for their whole length, where
    rounding alone picks the leaf cell (and, on a refined grid, the step)."""
    cells = synth.make_cells(grid_name)
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(obs, z, 4, steps_per_cell=spc, adaptive=adaptive)
    res = M.born_beam(grid, cfg)
    A = res["A"].cpu().numpy().astype(np.float64)
    assert (res["status"].cpu().numpy() == 0).all()
    dirs = O.pix2vec_nest(4, np.arange(192))
    p = O.params(obs, z_src=z, steps_per_cell=spc, adaptive=adaptive)
    Ao, rec = O.born(O.Field.grid(cells), O.cosmo(*COSMO), p, dirs)
    assert (rec["status"] == O.REACHED).all()
    d = np.abs(A - Ao).max(axis=(1, 2))
    lens = np.abs(Ao - np.eye(2)).max(axis=(1, 2))
    _print(f"Born beam ({grid_name}): max |A - A_oracle| {d.max():.3e}, max |A_oracle - I| {lens.max():.3e}, "
           f"{(d > 1e-6).sum()} of {len(d)} above 1e-6")
    assert lens.max() > 1e-3
    assert (d > 1e-6).sum() <= (0.02 * len(d) if adaptive else 0)
    inf = M.infinitesimal_beam(grid, cfg)["A"].cpu().numpy().astype(np.float64)
    assert np.abs(inf - A).max() < 0.2 * lens.max()


def test_healpix_dirs_are_the_pixel_cast_directions(M, gauss64):
    """mpath_healpix_dirs gives the directions the pixel casts start along:
    casting along them reproduces the pixel cast bit for bit, and they match
    the oracle's NESTED pixel centres to rounding."""
    d = M.healpix_dirs(8, 100, 400)
    o = O.pix2vec_nest(8, np.arange(100, 500))
    assert np.abs(d.cpu().numpy() - o).max() < 1e-15
    grid = M.Grid(gauss64, COSMO)
    a = run_gpu(grid, M.CastConfig(CENTRE, 0.3, 8, pix_first=[100], pix_count=[400], steps_per_cell=10))
    b = run_gpu(grid, M.CastConfig(CENTRE, 0.3, 8, pix_count=[400], dirs=d, steps_per_cell=10))
    for k in ("beta", "z5", "n_steps", "status", "hash"):
        assert np.array_equal(a[k], b[k]), k
    assert M.healpix_dirs(4, 0, 0).shape == (0, 3)
