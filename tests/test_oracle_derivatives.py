"""Pins of the oracle's exact (complex-step) derivatives against central finite
differences of its own forward map, and of the distortion-matrix algebra
(Eq. for A in Sect. 2.3)."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def grid(O):
    cells = synth.make_cells("gauss32")
    return cells, O.Field.grid(cells)


def _fd_agreement(fd, cs, rel, global_scale=False):
    """Fraction of rays whose FD and complex-step derivatives agree to `rel`
    (relative to the ray's own derivative size), and the worst disagreement.
    A finite difference that straddles a CIC kink (a stage point crossing a
    cell-centre plane between the two perturbed rays) differs at O(1); such
    rays are rare at these step sizes."""
    fd = np.atleast_2d(fd.T).T
    cs = np.atleast_2d(cs.T).T
    scale = np.maximum(np.abs(cs).max(axis=-1), 1e-300)
    if global_scale:
        scale = np.full_like(scale, scale.max())
    err = np.abs(fd - cs).max(axis=-1) / scale
    return np.mean(err < rel), err.max()


def test_direction_derivative_matches_fd(O, grid):
    cells, f = grid
    c = O.cosmo()
    p = O.params([125.0, 125.0, 125.0], z_src=0.3, steps_per_cell=4)
    dirs = O.pix2vec_nest(2, np.arange(48))
    e1, e2 = O.screen_basis(dirs)
    unit = lambda v: v / np.linalg.norm(v, axis=1, keepdims=True)
    for b, e in enumerate((e1, e2)):
        dth = np.zeros((len(dirs), 2))
        dth[:, b] = 1.0
        out, tan = O.cast_cs(f, c, p, dirs, dtheta=dth)
        # step chosen where rounding noise (~1/eps) and truncation meet
        eps = 1e-6
        rp, rm = O.cast(f, c, p, unit(dirs + np.tan(eps) * e)), O.cast(f, c, p, unit(dirs - np.tan(eps) * e))
        frac, worst = _fd_agreement((rp["r"] - rm["r"]) / (2 * eps), tan["r"], 1e-7)
        assert frac >= 0.9 and worst < 1e-2, (frac, worst)
        frac, worst = _fd_agreement((rp["z5"] - rm["z5"]) / (2 * eps), tan["z5"], 3e-6, global_scale=True)
        assert frac >= 0.9, (frac, worst)


def test_cell_value_derivative_matches_fd(O, grid):
    cells, f = grid
    c = O.cosmo()
    p = O.params([125.0, 125.0, 125.0], z_src=0.3, steps_per_cell=4)
    dirs = O.pix2vec_nest(2, np.arange(48))
    rng = np.random.default_rng(3)
    dphi = rng.standard_normal(cells.n_cells) * 1e-5
    dgrad = rng.standard_normal((cells.n_cells, 3)) * 1e-6
    out, tan = O.cast_cs(f, c, p, dirs, dphi=dphi, dgrad=dgrad)
    eps = 1e-3

    def shifted(s):
        cc = synth.Cells(cells.box, cells.n0, cells.max_level, cells.periodic, cells.level, cells.ijk,
                         cells.phi + s * dphi, cells.grad + s * dgrad)
        return O.cast(O.Field.grid(cc), c, p, dirs)

    rp, rm = shifted(eps), shifted(-eps)
    for key, rel in (("sep2", 1e-6), ("z5", 1e-5), ("phi_s", 1e-6), ("r", 1e-6), ("alpha", 1e-6)):
        frac, worst = _fd_agreement((rp[key] - rm[key]) / (2 * eps), tan[key], rel)
        assert frac >= 0.9 and worst < 1e-2, (key, frac, worst)
    # sep2 = |alpha|^2
    assert np.allclose(out["sep2"], np.sum(out["alpha"] ** 2, 1), rtol=1e-10)


def test_decompose_inverts_compose(O):
    rng = np.random.default_rng(0)
    k, g1, g2 = rng.normal(0, 0.05, (3, 200))
    w = rng.normal(0, 0.01, 200)
    A = O.compose(k, g1, g2, w)
    kk, gg1, gg2, ww, mu = O.decompose(A)
    assert np.allclose([kk, gg1, gg2, ww], [k, g1, g2, w], atol=1e-14)
    assert np.allclose(mu, 1.0 / ((1 - k) ** 2 - g1 ** 2 - g2 ** 2), rtol=1e-12)
    # a pure rotation has kappa = gamma = 0 and mu = 1
    kk, gg1, gg2, ww, mu = O.decompose(O.compose(0.0, 0.0, 0.0, 0.3))
    assert abs(kk) < 1e-15 and abs(gg1) < 1e-15 and abs(gg2) < 1e-15 and ww == pytest.approx(0.3)
