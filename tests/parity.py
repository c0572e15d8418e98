"""Helpers shared by the GPU parity tests: run the same seeded workload through
the HIP library (via its C ABI) and through the FP64 oracle, and compare.

Tolerances (the parity bar of the method's observables):
  * deflection: angular separation of the end-point directions r_s - x_obs,
    GPU vs oracle, <= 1e-3 arcsec;
  * observed redshift: |z5_gpu - z5_oracle| / z5_oracle <= 1e-7.
They apply to every ray whose discrete decisions (leaf level of each step and
stencil level of each sub-step, summarised by the FNV hash both sides
compute) are identical.  A ray whose FP32/FP64 position sits within rounding
of an AMR boundary may legitimately take the other branch there; such rays
are counted and must be rare.
"""
from __future__ import annotations

import numpy as np

import oracle as O

ARCSEC = np.pi / 180 / 3600
TOL_ARCSEC = 1e-3
TOL_Z = 1e-7


def run_gpu(grid, cfg):
    import paper_2111_08744_amd as M
    import torch
    out = M.cast(grid, cfg)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if not k.startswith("_")}
    res["hash"] = res["hash"].view(np.uint32)
    return res


def oracle_dirs(nside, pix_first, pix_count):
    pix = np.concatenate([np.arange(f, f + c) for f, c in zip(pix_first, pix_count)])
    return O.pix2vec_nest(nside, pix)


def run_oracle(field, cosmo, obs, stop, nside, pix_first, pix_count, steps_per_cell, adaptive,
               stop_kind="z", max_steps=1 << 40, ray_index=None):
    """Oracle records of every ray (or of the rays listed in ray_index, in the
    GPU's numbering: observer by observer, pixel order)."""
    obs = np.atleast_2d(obs)
    stop = np.atleast_1d(stop)
    counts = np.asarray(pix_count)
    firsts = np.asarray(pix_first)
    starts = np.concatenate([[0], np.cumsum(counts)])
    n = int(starts[-1])
    idx = np.arange(n) if ray_index is None else np.asarray(ray_index)
    rec = np.zeros(len(idx), O.RAY_DTYPE)
    which = np.searchsorted(starts, idx, side="right") - 1
    for j in np.unique(which):
        sel = np.nonzero(which == j)[0]
        pix = firsts[j] + (idx[sel] - starts[j])
        dirs = O.pix2vec_nest(nside, pix)
        kw = {"z_src": stop[j]} if stop_kind == "z" else {"chi": stop[j]}
        p = O.params(obs[j], steps_per_cell=steps_per_cell, adaptive=adaptive, max_steps=max_steps, **kw)
        rec[sel] = O.cast(field, cosmo, p, dirs)
    return rec


def beta_to_vec(beta):
    th, ph = beta[:, 0], beta[:, 1]
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)


def compare(gpu, ora, idx=None, isw_tol=0.0, z0_own=False):
    """Element-by-element comparison; returns a summary dict.  Asserts.
    Every ray must take the oracle's branches (its decision hash: leaf and
    stencil levels of every stage) and then agree within the bars.
    isw_tol: absolute bar on the ISW integral (0 for a static potential,
    where both sides must give exactly 0 and z4 = z1).  z0_own: z0 is the
    FLRW redshift of each end point's own scale factor (iso-chi, -lambda and
    -z surfaces), which moves with the end point: the relative bar of z5;
    otherwise it is the stop's, equal on both sides."""
    g = {k: (v if idx is None else v[idx]) for k, v in gpu.items()}
    n = len(ora)
    assert np.array_equal(g["status"], ora["status"]), "status differs"
    same = g["hash"] == ora["hash"]
    n_flip = int(n - same.sum())
    assert n_flip == 0, f"{n_flip} of {n} rays took a different branch"
    assert np.array_equal(g["n_steps"][same], ora["n_steps"][same])
    vg = beta_to_vec(g["beta"])
    vo = ora["r"] / np.linalg.norm(ora["r"], axis=1, keepdims=True)
    sep = np.arctan2(np.linalg.norm(np.cross(vg, vo), axis=1), np.sum(vg * vo, 1)) / ARCSEC
    reached = ora["status"] == O.REACHED
    summary = {"n": n, "n_flip": n_flip, "max_sep_arcsec": float(sep[same].max(initial=0.0))}
    assert summary["max_sep_arcsec"] <= TOL_ARCSEC, summary
    ok = same & reached
    if ok.any():
        relz = np.abs(g["z5"][ok] - ora["z5"][ok]) / np.abs(ora["z5"][ok])
        summary["max_rel_z"] = float(relz.max())
        assert summary["max_rel_z"] <= TOL_Z, summary
        # deflection vector (float32 output): absolute agreement in arcsec
        dal = np.abs(g["alpha"][ok] - ora["alpha"][ok]).max() / ARCSEC
        summary["max_alpha_arcsec"] = float(dal)
        assert dal <= 2 * TOL_ARCSEC, summary
        # Phi at the end point: float32 payload, relative to the field scale
        dphi = np.abs(g["phi_src"][ok] - ora["phi_s"][ok]).max()
        summary["max_dphi"] = float(dphi)
        assert dphi <= 1e-6 * max(np.abs(ora["phi_s"]).max(), 1e-12), summary
        if z0_own:
            assert np.all(np.abs(g["z0"][ok] - ora["z0"][ok]) <= TOL_Z * np.abs(ora["z0"][ok])), summary
        else:
            assert np.all(g["z0"][ok] == ora["z0"][ok])
        if "z1" in g:
            # z0 plus the potential term (Sect. 2.5): relative bar, with an
            # absolute floor at the level of float32 cell values (the term is
            # all of z1 in a static background, where z0 = 0)
            dz1 = np.abs(g["z1"][ok] - ora["z1"][ok])
            summary["max_dz1"] = float(dz1.max())
            assert np.all(dz1 <= TOL_Z * np.abs(ora["z1"][ok]) + 1e-11), summary
        if "isw" in g:
            # ISW integral (Sect. 2.5): float32 dPhi/deta samples and
            # per-step sums; z4 = z1 - 2 (1 + z0) isw inherits both bars
            disw = np.abs(g["isw"][ok] - ora["isw"][ok])
            summary["max_disw"] = float(disw.max())
            assert np.all(disw <= isw_tol), summary
            dz4 = np.abs(g["z4"][ok] - ora["z4"][ok])
            summary["max_dz4"] = float(dz4.max())
            assert np.all(dz4 <= TOL_Z * np.abs(ora["z4"][ok]) + 1e-11 + 2 * (1 + ora["z0"][ok]) * isw_tol), summary
    return summary
