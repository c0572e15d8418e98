"""Pins of the oracle's time-dependent potential (Sect. 2.2: the dPhi/deta
terms of the geodesic equations and dPhi/deta from a double-layer light
cone; Sect. 2.5: the ISW term of z4) by values the equations fix on their
own: closed forms for a spatially constant potential with a constant time
derivative, an independent ODE solution for a time derivative linear in
position, and exact cases of the double-layer difference quotient."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synth

COSMO = (0.3, 0.7, 0.7)
H0 = 1.0 / 2997.92458          # H0 / c in h / Mpc


def _uniform(n, box, phi, tdot, periodic=True):
    """Uniform grid with constant Phi, zero gradient and dPhi/deta from tdot(x)."""
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int32)
    centres = (ijk + 0.5) * (box / n)
    return synth.Cells(box=box, n0=n, max_level=0, periodic=periodic, level=np.zeros(len(ijk), np.uint8),
                       ijk=ijk, phi=np.full(len(ijk), phi), grad=np.zeros((len(ijk), 3)),
                       dphi_deta=tdot(centres))


def test_constant_time_derivative_closed_forms(O):
    """Phi = phi0 everywhere, grad Phi = 0, dPhi/deta = T.  The equations
    give dk0/dl = -2 H k0^2 (the two T terms cancel: FLRW), so z5 = z0; and
    d ln(|k| / |k0|) / d eta = 2 T, so with m0 = sqrt((1 + 2 phi0)/(1 - 2 phi0))
    the photon covers chi = m0 (1 - exp(-2 T D)) / (2 T) over D = eta_0 -
    eta_s, in a straight line.  The ISW integral is T D and
    z4 = z0 - 2 (1 + z0) T D (z1 = z0 for a constant Phi).  A dropped or
    mis-signed T term moves chi (by 2 T D ~ 5%) or z5."""
    phi0, T = 2e-5, 2e-5
    cells = _uniform(8, 64.0, phi0, lambda x: np.full(len(x), T))
    c = O.cosmo(*COSMO)
    obs = [10.0, 20.0, 30.0]
    p = O.params(obs, z_src=0.5, steps_per_cell=4)
    dirs = O.pix2vec_nest(2, np.arange(48))
    r = O.cast(O.Field.grid(cells), c, p, dirs)
    assert (r["status"] == O.REACHED).all()
    D = O.eta0(c) - r["eta"]
    m0 = np.sqrt((1 + 2 * phi0) / (1 - 2 * phi0))
    chi = m0 * (1 - np.exp(-2 * T * D)) / (2 * T)
    assert 2 * T * D.min() > 0.04
    assert np.abs(r["chi"] / chi - 1).max() < 1e-10
    assert np.abs(r["isw"] / (T * D) - 1).max() < 1e-12
    assert np.abs(r["z5"] - r["z0"]).max() < 1e-10
    z0 = r["z0"]
    assert np.abs(r["z4"] - (z0 - 2 * (1 + z0) * T * D)).max() < 1e-13
    assert np.abs(r["alpha"]).max() < 1e-12
    # a static grid carries no ISW term
    s = O.cast(O.Field.grid(_uniform(8, 64.0, phi0, lambda x: np.zeros(len(x)))), c, p, dirs)
    assert (s["isw"] == 0).all() and np.array_equal(s["z4"], s["z1"])


def test_linear_time_derivative_against_an_ode_solver(O):
    """dPhi/deta = t0 + t . x (reproduced exactly by CIC) on a non-periodic
    grid, Phi constant, no gradient: the photon runs straight, and with
    tau = eta_0 - eta the equations reduce to d chi/d tau = m,
    dm/d tau = -2 T m, dI/d tau = T at x = x_obs + chi n; solved here by an
    independent adaptive integrator at tight tolerances.  The oracle's RK4
    error falls 16-fold per halving of the step (4e-10 at 8 steps per cell);
    at 32 steps per cell it is below 2e-12."""
    t0, tv = 1e-5, np.array([2e-8, -1e-8, 3e-8])
    phi0 = -1e-5
    cells = _uniform(16, 2000.0, phi0, lambda x: t0 + x @ tv, periodic=False)
    c = O.cosmo(*COSMO)
    obs = np.array([300.0, 320.0, 310.0])
    p = O.params(obs, z_src=0.3, steps_per_cell=32)
    rng = np.random.default_rng(4)
    dirs = np.abs(rng.standard_normal((6, 3))) + 0.2
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = O.cast(O.Field.grid(cells), c, p, dirs)
    assert (r["status"] == O.REACHED).all()
    D = O.eta0(c) - r["eta"]
    m0 = np.sqrt((1 + 2 * phi0) / (1 - 2 * phi0))
    for i, n in enumerate(dirs):
        def f(tau, y):
            T = t0 + (obs + y[0] * n) @ tv
            return [y[1], -2 * T * y[1], T]
        sol = solve_ivp(f, (0.0, D[i]), [0.0, m0, 0.0], method="DOP853", rtol=1e-13, atol=1e-15)
        chi, _, I = sol.y[:, -1]
        assert r["chi"][i] == pytest.approx(chi, rel=1e-11)
        assert r["isw"][i] == pytest.approx(I, rel=1e-11)
    assert np.abs(r["alpha"]).max() < 1e-12


def test_double_layer_exact_cases(O):
    """Phi quadratic in a: the difference quotient is dPhi/da at the midpoint
    exactly; times a' there.  In Einstein-de Sitter a' = H0 sqrt(a) (from
    eta = 2 sqrt(a) / H0); in LCDM a' is checked against a centred
    difference of the oracle's own a(eta)."""
    rng = np.random.default_rng(8)
    c0, c1, c2 = rng.normal(0, 1e-5, (3, 50))
    a1 = rng.uniform(0.3, 0.9, 50)
    a2 = a1 + rng.uniform(-0.05, 0.05, 50)
    am = 0.5 * (a1 + a2)
    phi = lambda a: c0 + c1 * a + c2 * a * a
    eds = O.cosmo(1.0, 0.0, 0.7)
    got = O.double_layer(phi(a1), phi(a2), a1, a2, eds)
    assert np.allclose(got, (c1 + 2 * c2 * am) * H0 * np.sqrt(am), rtol=1e-9, atol=0)
    lcdm = O.cosmo(*COSMO)
    got = O.double_layer(phi(a1), phi(a2), a1, a2, lcdm)
    h = 1e-2
    adot = np.array([(O.a_of_eta(lcdm, O.eta_of_a(lcdm, a) + h) - O.a_of_eta(lcdm, O.eta_of_a(lcdm, a) - h)) / (2 * h)
                     for a in am])
    assert np.allclose(got, (c1 + 2 * c2 * am) * adot, rtol=1e-8, atol=0)
    # equal layers: no time derivative
    assert (O.double_layer(phi(a1), phi(a1), a1, a2, lcdm) == 0).all()


def test_library_double_layer_matches_oracle(O):
    """The library's host ingest of the double layer against the oracle on
    the synthetic layers of the uniform 64^3 grid (no GPU needed)."""
    import paper_2111_08744_amd as M
    try:
        M._abi.lib()
    except OSError:
        pytest.skip("the HIP library is not built")
    c1 = synth.make_cells("gauss64")
    c2 = synth.make_cells("gauss64_layer2")
    a1, a2 = synth.ISW_LAYER_A
    want = O.double_layer(c1.phi, c2.phi, a1, a2, O.cosmo(*COSMO))
    got = M.double_layer(c1.phi, c2.phi, a1, a2, COSMO)
    assert np.abs(want).max() > 1e-10
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    with pytest.raises(M.MpathError):
        M.double_layer(c1.phi[:4], c2.phi[:4], 0.5, 0.5, COSMO)
    with pytest.raises(M.MpathError):
        M.double_layer(c1.phi[:4], c2.phi[:4], 0.5, 0.6, (0.0, 0.0, 0.7))
