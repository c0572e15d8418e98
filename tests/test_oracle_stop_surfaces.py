"""Pins of the oracle's stop surfaces (Sect. 2.4: maps on iso-p surfaces,
p in {a, eta, chi, z, lambda}, at the value p takes for an FLRW photon):
the affine parameter of the FLRW photon in closed form and against the
integrated photon, the equivalence of all surfaces without perturbations,
and the definition of each surface on a lensed grid."""
import numpy as np
import pytest

import synth

COSMO = (0.3, 0.7, 0.7)
H0 = 1.0 / 2997.92458
SURFS = {"eta": 0, "chi": 1, "lambda": 2, "z": 3}


def _zero_grid():
    phi = np.zeros((16, 16, 16))
    return synth.uniform_cells(phi, np.zeros((16, 16, 16, 3)), 256.0)


def test_lambda_of_a_einstein_de_sitter(O):
    """H = H0 a^-3/2: lambda(a) = int_a^1 a'^(3/2) da' / H0 = 2 (1 - a^(5/2)) / (5 H0)."""
    c = O.cosmo(1.0, 0.0, 0.7)
    for a in (0.05, 0.3, 0.5, 0.9, 1.0):
        assert O.lambda_of_a(c, a) == pytest.approx(2 * (1 - a ** 2.5) / (5 * H0), rel=1e-12, abs=1e-12)


def test_flrw_photon_affine_parameter(O):
    """An unperturbed photon integrated to the iso-eta surface carries the
    affine parameter lambda(a_s) of the quadrature (RK4 and Simpson agree)."""
    c = O.cosmo(*COSMO)
    f = O.Field.grid(_zero_grid())
    for z in (0.1, 0.7, 2.0):
        r = O.cast(f, c, O.params([1.0, 2.0, 3.0], z_src=z, steps_per_cell=4), O.pix2vec_nest(1, np.arange(4)))
        assert np.allclose(r["lam"], O.lambda_of_a(c, 1 / (1 + z)), rtol=1e-10, atol=0)


def test_surfaces_coincide_without_perturbations(O):
    """Phi = 0: the photon's eta, chi, lambda and z are the FLRW relations of
    one another, so every surface stops it at the same point, to the RK4
    error of k0 over steps of 4 Mpc/h: ~2e-12 in z, which the z and lambda
    surfaces turn into ~7e-9 Mpc/h in eta (divided by a'/a ~ 3e-4)."""
    c = O.cosmo(*COSMO)
    f = O.Field.grid(_zero_grid())
    dirs = O.pix2vec_nest(2, np.arange(0, 48, 5))
    z = 0.8
    a_s = 1 / (1 + z)
    eta_s = O.eta_of_a(c, a_s)
    for name, k in SURFS.items():
        r = O.cast(f, c, O.params([3.0, 5.0, 7.0], z_src=z, steps_per_cell=4, surface=k), dirs)
        assert (r["status"] == O.REACHED).all(), name
        assert np.abs(r["eta"] - eta_s).max() < 2e-8, name
        assert np.abs(r["chi"] - (O.eta0(c) - eta_s)).max() < 2e-8, name
        assert np.abs(r["z5"] - z).max() < 1e-10, name
        assert np.abs(r["lam"] / O.lambda_of_a(c, a_s) - 1).max() < 1e-11, name


@pytest.fixture(scope="module")
def lensed(O):
    cells = synth.make_cells("gauss32")
    return O.Field.grid(cells)


def test_each_surface_holds_its_parameter(O, lensed):
    """On a lensed grid each surface holds its own parameter at the end
    point (the landing converges), and the surfaces are distinct.  The
    redshift surface converges more slowly than the others: z5 takes Phi
    interpolated at the end point, whose derivative along the ray jumps at
    cell faces, while the Newton slope uses the interpolated gradient, so two
    iterations leave ~3e-11 (four reach 2e-15)."""
    c = O.cosmo(*COSMO)
    dirs = O.pix2vec_nest(2, np.arange(48))
    z = 0.3
    a_s = 1 / (1 + z)
    obs = [125.3, 124.6, 125.9]
    p = lambda k: O.params(obs, z_src=z, steps_per_cell=4, surface=k)
    eta = O.cast(lensed, c, p(0), dirs)
    chi = O.cast(lensed, c, p(1), dirs)
    lam = O.cast(lensed, c, p(2), dirs)
    zz = O.cast(lensed, c, p(3), dirs)
    for r in (eta, chi, lam, zz):
        assert (r["status"] == O.REACHED).all()
    chi_s = O.eta0(c) - O.eta_of_a(c, a_s)
    assert np.abs(chi["chi"] / chi_s - 1).max() < 1e-13
    assert np.abs(lam["lam"] / O.lambda_of_a(c, a_s) - 1).max() < 1e-13
    assert np.abs(zz["z5"] - z).max() < 1e-10
    assert np.abs(eta["eta"] - O.eta_of_a(c, a_s)).max() < 1e-9
    # lensing separates them: the end points differ at first order in Phi
    for r in (chi, lam, zz):
        d = np.abs(r["eta"] - eta["eta"])
        assert d.max() > 1e-4 and d.max() < 1.0
    # z0 is the FLRW redshift of the end point's own scale factor
    a_end = np.array([O.a_of_eta(c, e) for e in chi["eta"]])
    assert np.allclose(chi["z0"], 1 / a_end - 1, rtol=0, atol=1e-14)


def test_surface_rejections(O, lensed):
    c = O.cosmo(*COSMO)
    with pytest.raises(ValueError):
        O.cast(lensed, O.cosmo(0.0, 0.0, 0.7), O.params([1.0, 1.0, 1.0], chi=50.0, surface=3), [[1.0, 0.0, 0.0]])
    with pytest.raises(ValueError):
        O.cast(lensed, c, O.params([1.0, 1.0, 1.0], z_src=0.1, surface=7), [[1.0, 0.0, 0.0]])
