"""Distortion matrix helpers of the oracle (Sect. 2.3).  TEST INFRASTRUCTURE ONLY.

All 2x2 matrices use the screen basis e1 = e_phi, e2 = -e_theta (the basis of
the finite-beam rays in Sect. 2.3.2), on the theta side at the initial
direction and on the beta side at the final angular position.
"""
from __future__ import annotations

import numpy as np


def screen_basis(n):
    """(e1, e2) = (e_phi, -e_theta) at unit vectors n[..., 3]."""
    n = np.asarray(n, float)
    ph = np.arctan2(n[..., 1], n[..., 0])
    th = np.arctan2(np.hypot(n[..., 0], n[..., 1]), n[..., 2])
    e1 = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], -1)
    e2 = np.stack([-np.cos(ph) * np.cos(th), -np.sin(ph) * np.cos(th), np.sin(th)], -1)
    return e1, e2


def angular_separation(u, v):
    """Great-circle angle between direction vectors (any length), radians."""
    u = np.asarray(u, float)
    v = np.asarray(v, float)
    cr = np.linalg.norm(np.cross(u, v), axis=-1)
    dt = np.sum(u * v, axis=-1)
    return np.arctan2(cr, dt)


def finite_beam(cast_fn, dirs, eps: float):
    """Finite-beam distortion matrix, Eq. (A-hat): four rays A, B, C, D at
    semi-aperture eps around each direction, stopped on the same iso-eta
    surface as the reference ray, finite differences of their end points
    projected on the beta screen of the reference ray and divided by
    2 chi_0 tan(eps).

    The printed second column, (xi_C - xi_D), gives -1 on the diagonal for a
    homogeneous universe with r_C = r - tan(eps) e2, r_D = r + tan(eps) e2;
    (xi_D - xi_C) is used so that A-hat -> identity without lensing.

    cast_fn(dirs[n,3]) -> oracle ray records.  Returns (A[n,2,2], ref records).
    """
    dirs = np.asarray(dirs, float)
    e1, e2 = screen_basis(dirs)
    te = np.tan(eps)

    def unit(v):
        return v / np.linalg.norm(v, axis=-1, keepdims=True)

    ref = cast_fn(dirs)
    xa = cast_fn(unit(dirs + te * e1))["r"]
    xb = cast_fn(unit(dirs - te * e1))["r"]
    xc = cast_fn(unit(dirs - te * e2))["r"]
    xd = cast_fn(unit(dirs + te * e2))["r"]
    chi0 = ref["chi"]
    f1, f2 = screen_basis(ref["r"])
    A = np.empty((len(dirs), 2, 2))
    den = 2.0 * chi0 * te
    A[:, 0, 0] = np.sum((xa - xb) * f1, -1) / den
    A[:, 1, 0] = np.sum((xa - xb) * f2, -1) / den
    A[:, 0, 1] = np.sum((xd - xc) * f1, -1) / den
    A[:, 1, 1] = np.sum((xd - xc) * f2, -1) / den
    return A, ref


def jacobian_cs(cast_cs_fn, dirs):
    """Exact distortion matrix A_ab = e~_a(beta) . dr/dtheta_b / |r| and dz5/dtheta_b
    from two complex-step passes (theta perturbed along e1, then e2)."""
    dirs = np.asarray(dirs, float)
    n = len(dirs)
    out, t1 = cast_cs_fn(dirs, np.tile([1.0, 0.0], (n, 1)))
    _, t2 = cast_cs_fn(dirs, np.tile([0.0, 1.0], (n, 1)))
    f1, f2 = screen_basis(out["r"])
    chi = out["chi"]
    A = np.empty((n, 2, 2))
    for b, t in enumerate((t1, t2)):
        A[:, 0, b] = np.sum(f1 * t["r"], -1) / chi
        A[:, 1, b] = np.sum(f2 * t["r"], -1) / chi
    dz = np.stack([t1["z5"], t2["z5"]], -1)
    return A, dz, out


def compose(kappa, g1, g2, omega):
    """Eq. (A): A = R(omega) [[1 - kappa - g1, -g2], [-g2, 1 - kappa + g1]]."""
    kappa, g1, g2, omega = map(np.asarray, (kappa, g1, g2, omega))
    c, s = np.cos(omega), np.sin(omega)
    S = np.empty(kappa.shape + (2, 2))
    S[..., 0, 0] = 1 - kappa - g1
    S[..., 0, 1] = -g2
    S[..., 1, 0] = -g2
    S[..., 1, 1] = 1 - kappa + g1
    R = np.empty_like(S)
    R[..., 0, 0] = c
    R[..., 0, 1] = -s
    R[..., 1, 0] = s
    R[..., 1, 1] = c
    return R @ S


def decompose(A):
    """Invert Eq. (A) for kappa, gamma1, gamma2, omega and mu = 1/det A.

    With A = R(w) S: A11 + A22 = 2 cos w (1-k), A21 - A12 = 2 sin w (1-k),
    so tan w = (A21 - A12)/(A11 + A22) and 1 - k is half the norm of that pair;
    then S = R(-w) A gives g1 = (S22 - S11)/2, g2 = -(S12 + S21)/2."""
    A = np.asarray(A, float)
    tr = A[..., 0, 0] + A[..., 1, 1]
    rot = A[..., 1, 0] - A[..., 0, 1]
    omega = np.arctan2(rot, tr)
    one_k = 0.5 * np.hypot(tr, rot)
    c, s = np.cos(omega), np.sin(omega)
    # S = R(-w) A
    S11 = c * A[..., 0, 0] + s * A[..., 1, 0]
    S12 = c * A[..., 0, 1] + s * A[..., 1, 1]
    S21 = -s * A[..., 0, 0] + c * A[..., 1, 0]
    S22 = -s * A[..., 0, 1] + c * A[..., 1, 1]
    g1 = 0.5 * (S22 - S11)
    g2 = -0.5 * (S12 + S21)
    mu = 1.0 / (A[..., 0, 0] * A[..., 1, 1] - A[..., 0, 1] * A[..., 1, 0])
    return 1.0 - one_k, g1, g2, omega, mu
