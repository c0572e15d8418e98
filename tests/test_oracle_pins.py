"""Physics pins of the oracle's integrator (Sect. 2.2-2.5): closed forms and
invariants that the discrete method must reproduce, chosen so that a dropped
term, a wrong sign or factor, or a transposed index in the geodesic equations,
the step rule, the landing or the observables fails at least one of them.

  P1  Phi = 0: straight rays, |x_s - x_o| = eta_0 - eta_s, 1 + z = 1/a, a^2 k0 conserved
  P13 Phi = 0 in a static universe: step count floor(chi/ds) + 1
  P2  constant gradient, static: transverse displacement -g_perp lambda^2, bend
      2 |g_perp| lambda, z5 = z1 = Phi_o - Phi_s (first order); the deflection
      alpha = +g_perp chi component by component on (e_phi, -e_theta)
  P3  static potential in FLRW: a^2 k0 = exp(-2 (Phi_s - Phi_o)) exactly, and
      z1 = z5 + O(Phi^2)
  P4  point mass, static: total deflection 4 m / b (Born, first order)
  P5  quadratic potential: A = I - chi_s^2/3 H_perp (eq. infinitesimal A) for the
      exact (complex-step) Jacobian, the infinitesimal beam and the finite beam
  P6  time reversal returns to the observer
  P7  the null condition stays satisfied to O(Phi^2)
"""
import numpy as np
import pytest

import synth

OBS = np.array([250.0, 250.0, 250.0])


def sep(u, v):
    return np.arctan2(np.linalg.norm(np.cross(u, v), axis=-1), np.sum(u * v, axis=-1))


@pytest.mark.parametrize("om", [0.3, 1.0])
def test_p1_flrw_straight_rays(O, om):
    c = O.cosmo(om, 1 - om, 0.7)
    dirs = O.pix2vec_nest(4, np.arange(192))
    zero = synth.uniform_cells(np.zeros((16, 16, 16)), np.zeros((16, 16, 16, 3)), 500.0)
    for f, p in [(O.Field.linear([0, 0, 0]), O.params(OBS, z_src=0.8, ds=0.7)),
                 (O.Field.grid(zero), O.params(OBS, z_src=0.8, steps_per_cell=4))]:
        out = O.cast(f, c, p, dirs)
        assert np.all(out["status"] == O.REACHED)
        a_s = 1 / 1.8
        eta_s = O.eta_of_a(c, a_s)
        assert np.max(sep(out["r"], dirs)) < 1e-14       # rounding only
        assert np.allclose(out["chi"], O.eta0(c) - eta_s, rtol=1e-13)
        assert np.allclose(out["eta"], eta_s, rtol=1e-14)
        assert np.allclose(1 + out["z5"], 1 / a_s, rtol=1e-12)
        assert np.allclose(out["z0"], 0.8, rtol=1e-14) and np.allclose(out["z1"], 0.8, rtol=1e-14)
        # a^2 k0 is conserved (k0 = -1 at the observer, a_0 = 1)
        assert np.allclose(a_s ** 2 * out["k"][:, 0], -1.0, rtol=1e-12)
        # |k| = |k0| without perturbation
        assert np.allclose(np.linalg.norm(out["k"][:, 1:], axis=1), -out["k"][:, 0], rtol=1e-13)
        assert np.abs(out["alpha"]).max() < 1e-14


def test_p13_step_count_static(O):
    zero = synth.uniform_cells(np.zeros((8, 8, 8)), np.zeros((8, 8, 8, 3)), 100.0)
    f = O.Field.grid(zero)
    dirs = O.pix2vec_nest(1, np.arange(12))
    for n_steps_cell, chi in [(4, 123.4), (10, 77.7), (1, 250.05)]:
        p = O.params([50.0, 50.0, 50.0], chi=chi, steps_per_cell=n_steps_cell)
        out = O.cast(f, O.STATIC, p, dirs)
        ds = 12.5 / n_steps_cell
        assert np.all(out["n_steps"] == int(np.floor(chi / ds)) + 1)
        assert np.allclose(out["chi"], chi, rtol=1e-14)
        # max_steps stops the ray early
        p2 = O.params([50.0, 50.0, 50.0], chi=chi, steps_per_cell=n_steps_cell, max_steps=5)
        out2 = O.cast(f, O.STATIC, p2, dirs)
        assert np.all(out2["status"] == O.MAX_STEPS) and np.all(out2["n_steps"] == 5)
        assert np.all(np.isnan(out2["z5"]))


def test_p2_constant_gradient(O):
    g = np.array([2e-8, -1e-8, 3e-8])
    phi0 = 1e-6
    f = O.Field.linear(g, phi0=phi0)
    dirs = O.pix2vec_nest(2, np.arange(48))
    chi = 300.0
    out = O.cast(f, O.STATIC, O.params([0, 0, 0], chi=chi, ds=0.5), dirs)
    assert np.all(out["status"] == O.REACHED)
    lam = chi                               # affine length to first order (|k0| = 1, a = 1)
    for i, n in enumerate(dirs):
        gp = g - n * (n @ g)
        xperp = out["r"][i] - n * (out["r"][i] @ n)
        # x_perp = -g_perp lambda^2 (first order)
        assert np.allclose(xperp, -gp * lam ** 2, rtol=0, atol=20 * np.linalg.norm(g) ** 2 * lam ** 3 + 1e-12)
        kh = out["k"][i, 1:] / np.linalg.norm(out["k"][i, 1:])
        kperp = kh - n * (kh @ n)
        assert np.allclose(kperp, -2 * gp * lam, rtol=0, atol=20 * np.linalg.norm(g) ** 2 * lam ** 2 + 1e-14)
    # z = Phi_o - Phi_s to first order
    dphi = out["phi_o"] - out["phi_s"]
    assert np.allclose(out["z5"], dphi, rtol=0, atol=10 * np.max(np.abs(dphi)) ** 2 + 1e-15)
    assert np.max(np.abs(dphi)) > 1e-6      # the test is not trivial
    # z1 (Sect. 2.5, FLRW redshift plus the potential term): z0 = 0 in a
    # static universe, so z1 is the gravitational shift Phi_o - Phi_s that
    # z5 carries at first order; its sign is fixed by z5 above
    assert np.all(out["z0"] == 0.0)
    assert np.allclose(out["z1"], out["z5"], rtol=0, atol=10 * np.max(np.abs(dphi)) ** 2 + 1e-15)


def _spherical_frame(n):
    """Unit vectors of the spherical coordinates at directions n: e_theta =
    dn/dtheta and e_phi = (dn/dphi)/sin(theta) of
    n = (sin t cos p, sin t sin p, cos t)."""
    t = np.arccos(np.clip(n[:, 2], -1, 1))
    p = np.arctan2(n[:, 1], n[:, 0])
    e_t = np.stack([np.cos(t) * np.cos(p), np.cos(t) * np.sin(p), -np.sin(t)], 1)
    e_p = np.stack([-np.sin(p), np.cos(p), np.zeros_like(p)], 1)
    return e_t, e_p


def test_p2_deflection_components(O):
    """Lens equation beta = theta - alpha (Sect. 2.3) with alpha on the screen
    basis (e1, e2) = (e_phi, -e_theta): for Phi = g.x in a static universe
    the photon ends displaced by -g_perp chi^2, so beta - theta = -g_perp chi
    and alpha = +g_perp chi, i.e. alpha_1 = chi g.e_phi and
    alpha_2 = -chi g.e_theta (first order).  Independently of g, the end
    direction satisfies r_hat = n - alpha_1 e1 - alpha_2 e2 to second order
    in the deflection.  A flipped sign of alpha, a flipped e2 or swapped
    components fail here."""
    g = np.array([2e-8, -1e-8, 3e-8])
    f = O.Field.linear(g, phi0=1e-6)
    dirs = O.pix2vec_nest(2, np.arange(48))
    chi = 300.0
    out = O.cast(f, O.STATIC, O.params([0, 0, 0], chi=chi, ds=0.5), dirs)
    assert np.all(out["status"] == O.REACHED)
    e_t, e_p = _spherical_frame(dirs)
    a1 = chi * (e_p @ g)
    a2 = -chi * (e_t @ g)
    big = np.hypot(a1, a2)
    assert big.max() > 5e-6                             # the test is not trivial
    tol = 20 * np.linalg.norm(g) ** 2 * chi ** 3 + 1e-14
    assert np.allclose(out["alpha"][:, 0], a1, rtol=0, atol=tol)
    assert np.allclose(out["alpha"][:, 1], a2, rtol=0, atol=tol)
    rh = out["r"] / np.linalg.norm(out["r"], axis=1, keepdims=True)
    d = rh - dirs
    assert np.allclose(np.sum(d * e_p, 1), -out["alpha"][:, 0], rtol=0, atol=4 * big.max() ** 2)
    assert np.allclose(np.sum(d * -e_t, 1), -out["alpha"][:, 1], rtol=0, atol=4 * big.max() ** 2)


@pytest.mark.parametrize("kind", ["quadratic", "point"])
def test_p3_redshift_identity(O, kind):
    """d ln(a^2 |k0|)/d lambda = -2 dPhi/dlambda for a static Phi, hence
    a_s^2 |k0_s| = exp(-2 (Phi_s - Phi_o)) with a_o = 1, |k0_o| = 1."""
    c = O.cosmo()
    if kind == "quadratic":
        H = np.array([[2e-10, 5e-11, 0], [5e-11, -1e-10, 3e-11], [0, 3e-11, 1e-10]])
        f = O.Field.quadratic(H, OBS + [30.0, -20.0, 10.0], phi0=-2e-5)
    else:
        f = O.Field.point(1e-3, OBS + [200.0, 50.0, 100.0], soft=5.0)
    dirs = O.pix2vec_nest(2, np.arange(48))
    out = O.cast(f, c, O.params(OBS, z_src=0.3, ds=0.4), dirs)
    a_s = 1 / 1.3
    lhs = a_s ** 2 * (-out["k"][:, 0])
    rhs = np.exp(-2 * (out["phi_s"] - out["phi_o"]))
    assert np.max(np.abs(lhs / rhs - 1)) < 1e-11
    assert np.max(np.abs(out["phi_s"] - out["phi_o"])) > 1e-7      # not trivial
    # z5 from the same quantities: 1 + z5 = a_s |k0_s| (1 + Phi_s) / (1 + Phi_o)
    assert np.allclose(1 + out["z5"], a_s * (-out["k"][:, 0]) * (1 + out["phi_s"]) / (1 + out["phi_o"]), rtol=1e-14)
    # z1 = z0 + (1 + z0)(Phi_o - Phi_s) (Sect. 2.5) is z5 to first order in
    # Phi: the two differ by O(Phi^2) only, while the potential term itself
    # is of order Phi (a flipped sign of Phi_o - Phi_s fails by 2x it)
    dphi = np.abs(out["phi_s"] - out["phi_o"])
    phimax = max(np.abs(out["phi_o"]).max(), np.abs(out["phi_s"]).max())
    assert np.all(np.abs(out["z5"] - out["z1"]) <= 10 * phimax ** 2 * (1 + out["z0"]))
    assert np.all(out["z0"] == pytest.approx(0.3, rel=1e-13))


def test_p4_point_mass_deflection(O):
    m, b, D = 1e-6, 2.0, 4000.0
    f = O.Field.point(m, [D, b, 0.0], soft=0.0)
    n = np.array([[1.0, 0.0, 0.0]])
    chi = 2 * D
    out = O.cast(f, O.STATIC, O.params([0, 0, 0], chi=chi, ds=0.02), n)
    k = out["k"][0, 1:]
    bend = np.arctan2(k[1], k[0])              # towards the mass (+y)
    born = 2 * m / b * (D / np.hypot(b, D) - (-D) / np.hypot(b, D))
    assert bend == pytest.approx(born, rel=2e-3)
    assert born == pytest.approx(4 * m / b, rel=1e-6)


def _quadratic_setup(O):
    # centre direction on the equator (nside 16, face 4, x = 8, y = 7): moving
    # along the sphere there does not rotate the (e_phi, e_theta) frame, so the
    # small deflections of the off-centre rays add no basis rotation to A
    n0 = O.pix2vec_nest(16, [1130])[0]
    assert abs(n0[2]) < 1e-15
    P = np.eye(3) - np.outer(n0, n0)
    M = np.array([[3.0, 1.0, -0.5], [1.0, -2.0, 0.7], [-0.5, 0.7, 1.5]])
    chis = O.chi_of_z(O.cosmo(), 0.25)
    H = P @ M @ P
    H *= 1e-4 / (np.abs(H).max() * chis ** 2)
    # rays within ~0.008 rad of n0: its descendants at nside 128
    dirs = O.pix2vec_nest(128, np.arange(1130 * 64, 1130 * 64 + 64, 4))
    return H, dirs, chis


def test_p5_quadratic_jacobian(O):
    """Constant Hessian, transverse to the rays: all three distortion
    matrices equal I - chi_s^2/3 H_perp up to O((H chi_s^2)^2) and, for the
    exact Jacobian and the finite beam, terms of order Phi along the ray
    (Shapiro delay; here |Phi| ~ 1e-8 against a lensing signal of 3e-5)."""
    c = O.cosmo()
    H, dirs, chis = _quadratic_setup(O)
    f = O.Field.quadratic(H, OBS)
    p = O.params(OBS, z_src=0.25, ds=1.0)
    A_cs, dz, out = O.jacobian_cs(lambda d, t: O.cast_cs(f, c, p, d, dtheta=t), dirs)
    A_inf, _ = O.infinitesimal(f, c, p, dirs, h_deriv=1.0)
    A_fb, _ = O.finite_beam(lambda d: O.cast(f, c, p, d), dirs, eps=1e-6)
    for i, n in enumerate(dirs):
        e1, e2 = O.screen_basis(n)
        E = np.stack([e1, e2])
        exp = np.eye(2) - chis ** 2 / 3.0 * (E @ H @ E.T)
        assert np.abs(exp - np.eye(2)).max() > 1e-5         # non-trivial lensing
        assert np.allclose(A_cs[i], exp, rtol=0, atol=1e-7), (A_cs[i], exp)
        assert np.allclose(A_inf[i], exp, rtol=0, atol=1e-9)
        assert np.allclose(A_fb[i], A_cs[i], rtol=0, atol=5e-9)


def test_p5_born_quadratic(O):
    """Born approximation along the straight line of a constant Hessian:
    int_0^chi_s (chi_s - chi) chi / chi_s dchi = chi_s^2 / 6 gives
    A = I - chi_s^2/3 H_perp exactly up to the trapezoid error of a quadratic
    integrand, (ds/chi_s)^2 relative; Phi = 0 gives the identity."""
    c = O.cosmo()
    H, dirs, chis = _quadratic_setup(O)
    f = O.Field.quadratic(H, OBS)
    p = O.params(OBS, z_src=0.25, ds=1.0)
    A, rec = O.born(f, c, p, dirs, h_deriv=1.0)
    assert (rec["status"] == O.REACHED).all()
    for i, n in enumerate(dirs):
        e1, e2 = O.screen_basis(n)
        E = np.stack([e1, e2])
        lens = chis ** 2 / 3.0 * (E @ H @ E.T)
        assert np.abs(lens).max() > 1e-5
        assert np.allclose(A[i], np.eye(2) - lens, rtol=0, atol=10 * np.abs(lens).max() / chis ** 2)
    A0, _ = O.born(O.Field.linear([0.0, 0.0, 0.0]), c, p, dirs, h_deriv=1.0)
    assert np.abs(A0 - np.eye(2)).max() < 1e-15


def test_p6_time_reversal(O):
    c = O.cosmo()
    f = O.Field.point(3e-4, OBS + [150.0, 30.0, -20.0], soft=3.0)
    n = O.pix2vec_nest(2, [5])[0]
    phi_o = f.probe(OBS)[1]
    y0 = np.concatenate([[O.eta0(c)], OBS, [-1.0], n * np.sqrt((1 + 2 * phi_o) / (1 - 2 * phi_o))])
    rng = np.random.default_rng(1)
    dl = rng.uniform(0.3, 0.9, size=500)
    st, y1 = O.integrate_steps(f, c, y0, dl)
    assert st == 0 and np.linalg.norm(y1[1:4] - OBS) > 250
    y1r = y1.copy()
    y1r[4:] *= -1
    st, y2 = O.integrate_steps(f, c, y1r, dl[::-1])
    assert st == 0
    assert np.abs(y2[1:4] - OBS).max() < 1e-9
    assert y2[0] == pytest.approx(y0[0], abs=1e-9)
    assert np.allclose(-y2[4:], y0[4:], rtol=1e-10)


@pytest.mark.parametrize("m", [1e-3, 1e-4])
def test_p7_null_condition(O, m):
    """The first-order geodesic equations keep k^nu k_nu = 0 up to O(Phi^2):
    the drift scales with the square of the potential and not with the step.
    (On a grid the stored gradient is not the exact derivative of the
    interpolated Phi, and the drift then measures that mismatch instead.)"""
    c = O.cosmo()
    obs = np.array([125.0, 125.0, 125.0])
    f = O.Field.point(m, obs + [100.0, 50.0, 30.0], soft=5.0)
    dirs = O.pix2vec_nest(2, np.arange(48))
    drift = []
    for ds in (2.0, 0.5):
        out = O.cast(f, c, O.params(obs, z_src=0.3, ds=ds), dirs)
        assert np.all(out["status"] == O.REACHED)
        phimax = max(np.abs(out["phi_o"]).max(), np.abs(out["phi_s"]).max())
        assert out["max_null"].max() < 200 * phimax ** 2
        drift.append(out["max_null"].max())
    assert drift[0] == pytest.approx(drift[1], rel=0.05)


def test_p12_steps_per_cell_convergence(O):
    """Sect. 3.4: results with 4 steps per cell are converged relative to 8
    (here: the change of beta is a small fraction of the deflection)."""
    c = O.cosmo()
    f = O.Field.grid(synth.make_cells("gauss32"))
    dirs = O.pix2vec_nest(2, np.arange(48))
    r = {}
    for n in (1, 4, 8):
        r[n] = O.cast(f, c, O.params([125.0, 125.0, 125.0], z_src=0.3, steps_per_cell=n), dirs)
    defl = np.sqrt(r[8]["sep2"])
    d4 = sep(r[4]["r"], r[8]["r"])
    d1 = sep(r[1]["r"], r[8]["r"])
    assert np.median(d4 / defl) < 0.02
    assert np.median(d1) > np.median(d4)


def _with_nan(cells, ijk, field):
    """Copy of a uniform grid with a NaN in one cell's potential or gradient."""
    import copy
    c = copy.deepcopy(cells)
    n = c.n0
    i = (ijk[0] * n + ijk[1]) * n + ijk[2]
    assert tuple(c.ijk[i]) == tuple(ijk)
    if field == "phi":
        c.phi[i] = np.nan
    else:
        c.grad[i, 1] = np.nan
    return c


def test_t6_nonfinite(O):
    """Status NONFINITE (Sect. 2.2 stop conditions): a NaN in one cell's
    gradient stops exactly the rays whose stencils meet that cell, during the
    step that meets it (that step is not counted), and leaves every other ray
    bit for bit as on the clean grid; a NaN potential in the observer's
    stencil makes the initial |k| NaN, so every ray stops in its first step."""
    cells = synth.make_cells("gauss32")
    obs = [125.0, 125.0, 125.0]
    dirs = O.pix2vec_nest(4, np.arange(192))
    p = O.params(obs, z_src=0.2, steps_per_cell=4)
    clean = O.cast(O.Field.grid(cells), O.cosmo(), p, dirs)
    out = O.cast(O.Field.grid(_with_nan(cells, (18, 16, 16), "grad")), O.cosmo(), p, dirs)
    hit = out["status"] == O.NONFINITE
    assert 0 < hit.sum() < len(dirs) // 2
    assert np.all(out["status"][~hit] == O.REACHED) and np.all(clean["status"] == O.REACHED)
    for k in ("r", "z5", "alpha", "n_steps", "hash"):
        assert np.array_equal(out[k][~hit], clean[k][~hit]), k
    assert np.all(out["n_steps"][hit] < clean["n_steps"][hit])
    assert np.all(out["n_steps"][hit] >= 1)          # the cell is a few cells from the observer
    # the rays stopped are those pointing at the cell (centre 2.5 cells along +x)
    cen = (np.array([18, 16, 16]) + 0.5) * 250.0 / 32 - obs
    cos = dirs @ (cen / np.linalg.norm(cen))
    assert cos[hit].min() > cos[~hit].min() and np.median(cos[hit]) > np.median(cos[~hit])
    out0 = O.cast(O.Field.grid(_with_nan(cells, (16, 16, 16), "phi")), O.cosmo(), p, dirs)
    assert np.all(out0["status"] == O.NONFINITE) and np.all(out0["n_steps"] == 0)
