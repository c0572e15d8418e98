"""Pins of the oracle's background cosmology (conformal time, a(eta), a'/a)
against direct quadrature and the Einstein-de Sitter closed form.

Sect. 2.2 needs a(eta) and a'(eta) in the fiducial cosmology (the paper reads
them from precomputed tables); the oracle evaluates them exactly."""
import numpy as np
import pytest
from scipy.integrate import quad

H0 = 1.0 / 2997.92458   # h/Mpc, c = 1


def eta_quadrature(om, ol, a):
    # eta(a) = int_0^a da' / (a'^2 H(a')); with a = y^2 the integrand is regular at 0
    f = lambda y: 2.0 * y / (y ** 4 * H0 * np.sqrt(om / y ** 6 + ol))
    return quad(f, 0.0, np.sqrt(a), epsabs=0.0, epsrel=1e-13, limit=400)[0]


@pytest.mark.parametrize("om", [0.3, 0.25, 1.0])
def test_eta_matches_quadrature(O, om):
    c = O.cosmo(om, 1.0 - om, 0.7)
    for a in [1e-3, 0.05, 0.2, 1 / 3, 0.5, 2 / 3, 0.9, 1.0, 1.1]:
        ref = eta_quadrature(om, 1.0 - om, a)
        assert abs(O.eta_of_a(c, a) / ref - 1.0) < 1e-12, a


def test_einstein_de_sitter_closed_form(O):
    c = O.cosmo(1.0, 0.0, 0.7)
    for a in [0.01, 0.3, 1.0]:
        assert O.eta_of_a(c, a) == pytest.approx(2.0 * np.sqrt(a) / H0, rel=1e-14)
        eta = 2.0 * np.sqrt(a) / H0
        assert O.a_of_eta(c, eta) == pytest.approx(a, rel=1e-14)
        # a = (H0 eta / 2)^2 => a'/a = 2/eta
        assert O.conformal_hubble(c, eta) == pytest.approx(2.0 / eta, rel=1e-13)


def test_a_of_eta_inverts(O):
    c = O.cosmo()
    for a in np.linspace(0.02, 1.05, 37):
        assert O.a_of_eta(c, O.eta_of_a(c, a)) == pytest.approx(a, rel=2e-15, abs=0)


def test_conformal_hubble_is_dlna_deta(O):
    c = O.cosmo()
    for eta in [500.0, 3000.0, 7000.0, 9900.0]:
        D = lambda d: (np.log(O.a_of_eta(c, eta + d)) - np.log(O.a_of_eta(c, eta - d))) / (2 * d)
        d = 1e-3 * eta
        fd = (4.0 * D(d / 2) - D(d)) / 3.0       # Richardson: O(d^4)
        assert O.conformal_hubble(c, eta) == pytest.approx(fd, rel=1e-8)


def test_static_universe(O):
    c = O.STATIC
    assert O.eta0(c) == 0.0
    assert O.a_of_eta(c, -123.0) == 1.0
    assert O.conformal_hubble(c, -5.0) == 0.0


def test_rejects_non_flat(O):
    assert O.lib().or_cosmo_check(O.cosmo(0.3, 0.6, 0.7)) != 0
