"""Geodesic finder of the oracle (Sect. 2.5).  TEST INFRASTRUCTURE ONLY.

For a source at comoving position x_src seen from x_obs, the comoving
angular position beta is the direction of x_src - x_obs and chi its
distance.  The initial direction theta is sought such that the photon,
stopped on the source's light-cone surface eta_s = eta_0 - chi, arrives in
the direction beta.  Newton iteration theta_{i+1} = theta_i - A^-1
(beta_i - beta) (the paper's root finder), with the identity in place of A
for the first iterations as the paper does, then the exact Jacobian (complex
step).  All 2-vectors are on the screen bases e1 = e_phi, e2 = -e_theta: at
theta_i on the theta side, at beta_i on the beta side, the bases of A.

Sources still unconverged after max_iter go to the paper's last-resort
root finder: photons are launched along a regular grid of directions
centred on the current theta, theta moves to the grid point whose photon
lands nearest the source, and the grid shrinks every round.
"""
from __future__ import annotations

import numpy as np

from . import REACHED, cast, cast_cs, params
from .lensing import angular_separation, jacobian_cs, screen_basis

NOT_CONVERGED, NOT_REACHED = -1, -2


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def newton_update(theta, beta_i, beta, A):
    """One step: residual beta - beta_i as screen components at beta_i,
    d_a = f_a(beta_i) . beta (zero exactly when beta_i = beta), solve
    A dtheta = d and move theta along its own screen basis."""
    f1, f2 = screen_basis(beta_i)
    d = np.array([f1 @ beta, f2 @ beta])
    dth = np.linalg.solve(A, d)
    e1, e2 = screen_basis(theta)
    return _unit(theta + dth[0] * e1 + dth[1] * e2)


def grid_candidates(theta, w, g):
    """The g x g grid of directions around theta spanning +-w on its screen
    plane: theta + a D e1 + b D e2, normalised, D = 2 w / (g - 1), for
    a, b in -(g-1)/2 .. (g-1)/2, candidate (b + h) g + (a + h) (a the fast
    index)."""
    e1, e2 = screen_basis(theta)
    h = (g - 1) // 2
    D = 2.0 * w / (g - 1)
    out = []
    for b in range(-h, h + 1):
        for a in range(-h, h + 1):
            out.append(_unit(theta + a * D * e1 + b * D * e2))
    return np.array(out)


def grid_search(field, c, p, theta, beta, w0, g, rounds, tol):
    """The last-resort root finder: rounds of g x g candidate casts around
    theta, starting at half-width w0, each round moving theta to the best
    candidate (the first of equal ones) and shrinking the half-width to
    the previous spacing, 2 w / (g - 1).  Returns (theta, round of
    convergence or -1, sep, the best separation of every round)."""
    w = w0
    best_seps = []
    sep = np.nan
    for r in range(rounds):
        cand = grid_candidates(theta, w, g)
        rec = cast(field, c, p, cand)
        seps = np.where(rec["status"] == REACHED, angular_separation(rec["r"], beta), np.inf)
        k = int(np.argmin(seps))
        if not np.isfinite(seps[k]):
            return theta, -1, sep, best_seps
        theta, sep = cand[k], seps[k]
        best_seps.append(sep)
        if sep < tol:
            return theta, r, sep, best_seps
        w = 2.0 * w / (g - 1)
    return theta, -1, sep, best_seps


def find_geodesics(field, c, obs, src, steps_per_cell=10, adaptive=False, tol=1e-10, max_iter=10,
                   identity_iters=3, max_steps=1 << 40, ds=0.0, grid_rounds=0, grid_n=5):
    """Returns theta [n, 3], n_iter [n] (iteration of convergence, counting
    the first cast as 0; max_iter + r: converged in round r of the grid
    search; -1 not converged, -2 a cast did not reach the source), sep [n]
    (angle between the last end direction and beta, rad).  ds: step length
    for analytic fields (grid fields use steps_per_cell).  grid_rounds > 0:
    sources unconverged after max_iter go to the grid search, its first
    half-width twice the last Newton separation."""
    obs = np.asarray(obs, float)
    src = np.atleast_2d(np.asarray(src, float))
    r = src - obs
    chi = np.linalg.norm(r, axis=1)
    beta = r / chi[:, None]
    n = len(src)
    theta = beta.copy()
    n_iter = np.full(n, NOT_CONVERGED, np.int64)
    sep = np.full(n, np.nan)
    for i in range(n):
        p = params(obs, chi=chi[i], steps_per_cell=steps_per_cell, adaptive=adaptive, max_steps=max_steps, ds=ds)
        th = beta[i].copy()
        for it in range(max_iter):
            if it >= identity_iters:
                A, _, out = jacobian_cs(lambda d, dt: cast_cs(field, c, p, d, dtheta=dt), th[None])
                A, rec = A[0], out[0]
            else:
                A, rec = np.eye(2), cast(field, c, p, th[None])[0]
            if rec["status"] != REACHED:
                n_iter[i] = NOT_REACHED
                break
            bi = _unit(rec["r"])
            sep[i] = angular_separation(bi, beta[i])
            if sep[i] < tol:
                n_iter[i] = it
                break
            th = newton_update(th, bi, beta[i], A)
        if n_iter[i] == NOT_CONVERGED and grid_rounds > 0:
            th, r, s, _ = grid_search(field, c, p, th, beta[i], 2.0 * sep[i], grid_n, grid_rounds, tol)
            if r >= 0:
                n_iter[i] = max_iter + r
            if np.isfinite(s):
                sep[i] = s
        theta[i] = th
    return theta, n_iter, sep
