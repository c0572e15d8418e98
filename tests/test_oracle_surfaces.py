"""Pins of the oracle's cast through several stop surfaces (one photon lands
on each surface in turn and continues)."""
import numpy as np

import synth

OBS = np.array([250.0, 250.0, 250.0])


def test_first_surface_is_the_single_cast(O):
    """Up to the first landing the photon does exactly what a cast to that
    surface does."""
    cells = synth.make_cells("gauss64")
    f = O.Field.grid(cells)
    c = O.cosmo(0.3, 0.7, 0.7)
    dirs = O.pix2vec_nest(2, np.arange(48))
    p = O.params(OBS, z_src=0.2, steps_per_cell=10)
    multi = O.cast_surfaces(f, c, p, [0.2, 0.5, 0.9], dirs)
    single = O.cast(f, c, p, dirs)
    for k in ("r", "z5", "n_steps", "hash", "status", "k"):
        assert np.array_equal(multi[0][k], single[k]), k
    assert (multi["status"] == O.REACHED).all()
    assert (np.diff(multi["n_steps"], axis=0) > 0).all()      # steps accumulate
    # the last surface: the same geodesic up to the step grid the landings shift
    last = O.cast(f, c, O.params(OBS, z_src=0.9, steps_per_cell=10), dirs)
    sep = np.arctan2(np.linalg.norm(np.cross(multi[2]["r"], last["r"]), axis=1), np.sum(multi[2]["r"] * last["r"], 1))
    assert sep.max() < 2e-7      # about 0.04 arcsec: the discretisation of interpolant kinks


def test_flrw_surfaces(O):
    """Phi = 0: on every surface the photon sits at chi(z_k) along n and
    1 + z5 = 1 / a(eta_k)."""
    f = O.Field.linear([0.0, 0.0, 0.0])
    c = O.cosmo(0.3, 0.7, 0.7)
    dirs = O.pix2vec_nest(1, np.arange(12))
    zs = [0.1, 0.45, 1.0, 2.0]
    multi = O.cast_surfaces(f, c, O.params([0, 0, 0], z_src=zs[0], ds=2.0), zs, dirs)
    for k, z in enumerate(zs):
        rec = multi[k]
        assert np.allclose(np.linalg.norm(rec["r"], axis=1), O.chi_of_z(c, z), rtol=1e-9)
        assert np.allclose(rec["r"] / np.linalg.norm(rec["r"], axis=1, keepdims=True), dirs, atol=1e-14)
        assert np.allclose(rec["z5"], z, rtol=1e-9)
