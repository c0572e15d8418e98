"""Pins of the oracle's geodesic finder (Sect. 2.5): closed forms that the
Newton iteration on the initial direction must reproduce."""
import numpy as np

from oracle import catalog
from oracle.lensing import angular_separation


def _dirs(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_no_potential_gives_beta(O):
    """Phi = 0: rays are straight, so theta = beta at the first cast."""
    f = O.Field.linear([0.0, 0.0, 0.0])
    beta = _dirs(12, 1)
    src = 700.0 * beta
    theta, it, sep = catalog.find_geodesics(f, O.STATIC, [0, 0, 0], src, ds=1.0, tol=1e-12)
    assert (it == 0).all()
    assert angular_separation(theta, beta).max() < 1e-14


def test_constant_gradient_offset(O):
    """Phi = g.x in a static universe bends a ray by x_perp = -g_perp lambda^2,
    so the image of a source at distance chi along beta is seen along
    theta = beta + g_perp chi to first order (g_perp transverse to beta)."""
    g = np.array([2e-8, -1e-8, 3e-8])
    f = O.Field.linear(g)
    beta = _dirs(16, 2)
    chi = 300.0
    theta, it, sep = catalog.find_geodesics(f, O.STATIC, [0, 0, 0], chi * beta, ds=0.5, tol=1e-13,
                                            identity_iters=1)
    assert (it >= 1).all() and (it < 6).all()
    gp = g[None, :] - beta * (beta @ g)[:, None]
    expect = beta + gp * chi
    expect /= np.linalg.norm(expect, axis=1, keepdims=True)
    err = angular_separation(theta, expect)
    assert err.max() < 20 * (np.linalg.norm(g) * chi) ** 2
    assert (np.linalg.norm(gp, axis=1) * chi).min() > 1e-6     # the offset is resolved


def test_grid_roots_reach_the_sources(O):
    """On a lensed grid the found directions land on the sources (checked by
    an independent cast), and exact Newton from the start finds the same
    roots as the identity-then-exact schedule."""
    import synth
    cells = synth.make_cells("gauss64")
    f = O.Field.grid(cells)
    c = O.cosmo(0.3, 0.7, 0.7)
    obs = np.array([250.0, 250.0, 250.0])
    rng = np.random.default_rng(9)
    src = obs + _dirs(6, 3) * rng.uniform(300.0, 1200.0, 6)[:, None]
    t1, it1, s1 = catalog.find_geodesics(f, c, obs, src, tol=1e-11)
    t2, it2, s2 = catalog.find_geodesics(f, c, obs, src, tol=1e-11, identity_iters=0)
    assert (it1 >= 0).all() and (it2 >= 0).all()
    assert angular_separation(t1, t2).max() < 1e-10
    beta = (src - obs) / np.linalg.norm(src - obs, axis=1, keepdims=True)
    for i in range(len(src)):
        chi = np.linalg.norm(src[i] - obs)
        rec = O.cast(f, c, O.params(obs, chi=chi, steps_per_cell=10), t1[i][None])[0]
        assert angular_separation(rec["r"], beta[i]) < 1e-11
    assert angular_separation(t1, beta).max() > 1e-6      # the sources are lensed


def test_grid_search_fallback(O):
    """Sources left unconverged by two identity-Jacobian iterations go to the
    grid search: every round's best separation does not grow (the centre
    candidate is the previous best direction), they converge, and the roots
    are those of the exact Newton iteration (within the tolerance over the
    smallest singular value of A, ~1)."""
    import synth
    cells = synth.make_cells("gauss64")
    f = O.Field.grid(cells)
    c = O.cosmo(0.3, 0.7, 0.7)
    obs = np.array([250.0, 250.0, 250.0])
    rng = np.random.default_rng(9)
    src = obs + _dirs(4, 3) * rng.uniform(300.0, 1200.0, 4)[:, None]
    tol = 1e-11
    t0, it0, s0 = catalog.find_geodesics(f, c, obs, src, tol=tol, max_iter=2, identity_iters=2)
    assert (it0 == -1).all()
    t1, it1, s1 = catalog.find_geodesics(f, c, obs, src, tol=tol, max_iter=2, identity_iters=2,
                                         grid_rounds=30, grid_n=5)
    assert (it1 >= 2).all() and (s1 < tol).all()
    tn, itn, _ = catalog.find_geodesics(f, c, obs, src, tol=tol)
    assert (itn >= 0).all()
    assert angular_separation(t1, tn).max() < 3 * tol
    beta = (src - obs) / np.linalg.norm(src - obs, axis=1, keepdims=True)
    for i in range(len(src)):
        chi = np.linalg.norm(src[i] - obs)
        p = O.params(obs, chi=chi, steps_per_cell=10)
        _, r, _, seps = catalog.grid_search(f, c, p, t0[i], beta[i], 2.0 * s0[i], 5, 30, tol)
        assert r >= 0 and all(b <= a for a, b in zip(seps, seps[1:]))
