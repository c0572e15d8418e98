"""GPU adjoint (reverse sweep over checkpoints) against the FP64 oracle's
complex-step derivatives of the same discrete map, through the C ABI.

Checked quantities:
  * the distortion matrix A_ab = d beta_a / d theta_b and d z5 / d theta_b
    (Sect. 2.3, 2.5) per ray, against the oracle's exact derivative of the
    same RK4 / CIC / landing map (two complex-step passes);
  * the loss gradient with respect to the cell values (phi, grad phi), by
    directional derivatives: <dL/dvalues, delta> against the oracle's
    complex-step derivative along delta, for random delta and for single
    cells;
  * the derivative through a gradient defined as the central difference of
    phi, on a uniform periodic grid;
  * invariance of the results under the checkpoint interval, and the
    forward outputs of a checkpointed cast.

Tolerances.  The GPU state is FP32 (direction offset d and displacement dx)
with FP64 conformal time and |k0|; its path differs from the oracle's by
~1e-6 of a cell.  Derivatives inherit that relative error wherever the
interpolant is smooth; where a stage of one side falls across a cell-centre
plane (a kink of the CIC interpolant of the gradient) from the other, that
one stage's Jacobian differs by the jump of the second derivative, which
moves A by about (A - I) / (number of stages) ~ 1e-6 on such rare rays.
The outputs A and dz/dtheta are float32 (rounding 6e-8 on A ~ 1).  Bars:
5e-6 on the largest |A_gpu - A_oracle| of any ray and 2e-7 on the median,
1e-5 relative on dz/dtheta (1e-6 median) and on the directional loss
derivatives (float32 cell cotangents summed by atomics).
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity import oracle_dirs

pytestmark = pytest.mark.gpu

COSMO = (0.3, 0.7, 0.7)
OBS = [250.0, 250.0, 250.0]


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2111_08744_amd as M
    return M


@pytest.fixture(scope="module")
def gauss64():
    return synth.make_cells("gauss64")


def _cfg(M, z, nside, K, first=0, count=None, **kw):
    count = 12 * nside * nside if count is None else count
    return M.CastConfig(OBS, z, nside, [first], [count], steps_per_cell=10, checkpoint_every=K, **kw)


def _fwd(M, grid, cfg):
    import torch
    out = M.cast(grid, cfg)
    torch.cuda.synchronize()
    return out


def _np(t):
    return t.detach().cpu().numpy()


def _oracle_params(z, **kw):
    return O.params(OBS, z_src=z, steps_per_cell=10, adaptive=False, **kw)


def test_checkpointed_forward_equals_static(M, gauss64):
    grid = M.Grid(gauss64, COSMO)
    a = _fwd(M, grid, M.CastConfig(OBS, 0.3, 4, steps_per_cell=10, schedule=1))
    b = _fwd(M, grid, _cfg(M, 0.3, 4, 32))
    for k in ("beta", "alpha", "z5", "phi_src", "n_steps", "status", "hash"):
        assert np.array_equal(_np(a[k]), _np(b[k]), equal_nan=True), k


def test_jacobian_vs_oracle_complex_step(M, gauss64):
    """A and dz/dtheta of every ray of nside 4 (192 rays) to z = 0.3."""
    import torch
    grid = M.Grid(gauss64, COSMO)
    cfg = _cfg(M, 0.3, 4, 32)
    out = _fwd(M, grid, cfg)
    res = M.adjoint(grid, cfg, out, jacobian=True)
    torch.cuda.synchronize()
    jac, dz = _np(res["jac"]).astype(np.float64), _np(res["dz_dtheta"]).astype(np.float64)
    assert (_np(res["ray_status"]) == 0).all()     # every replay retraced its forward path
    field = O.Field.grid(gauss64)
    c = O.cosmo(*COSMO)
    p = _oracle_params(0.3)
    dirs = oracle_dirs(4, [0], [192])
    A, dzo, rec = O.jacobian_cs(lambda d, t: O.cast_cs(field, c, p, d, dtheta=t), dirs)
    same = _np(out["hash"]).view(np.uint32) == rec["hash"]
    _print("rays with the oracle's decisions:", same.sum(), "of", len(same))
    assert same.all()
    dA = np.abs(jac - A)[same].reshape(-1, 4).max(1)
    lens = np.abs(A - np.eye(2)).reshape(-1, 4).max(1)
    _print("|A - I| median", np.median(lens), "max", lens.max())
    _print("|A_gpu - A_oracle| median", np.median(dA), "p99", np.quantile(dA, 0.99), "max", dA.max())
    rz = np.abs(dz - dzo)[same].max(1) / np.abs(dzo).max()
    _print("dz/dtheta rel. diff median", np.median(rz), "max", rz.max(), "scale", np.abs(dzo).max())
    assert lens.max() > 1e-4                    # lensing is measurable here
    assert dA.max() < 5e-6 and np.median(dA) < 2e-7
    assert rz.max() < 1e-5 and np.median(rz) < 1e-6


def test_jacobian_independent_of_checkpoint_interval(M, gauss64):
    import torch
    grid = M.Grid(gauss64, COSMO)
    ref = None
    for K in (32, 1, 7, 100000):
        cfg = _cfg(M, 0.2, 2, K)
        out = _fwd(M, grid, cfg)
        res = M.adjoint(grid, cfg, out, jacobian=True)
        torch.cuda.synchronize()
        j = (_np(res["jac"]), _np(res["dz_dtheta"]))
        if ref is None:
            ref = j
        else:
            assert np.array_equal(j[0], ref[0]) and np.array_equal(j[1], ref[1]), K


def _loss_setup(M, cells, z, nside, K=32):
    import torch
    grid = M.Grid(cells, COSMO)
    cfg = _cfg(M, z, nside, K)
    out = _fwd(M, grid, cfg)
    alpha = out["alpha"].to(torch.float64)
    rng = np.random.default_rng(7)
    wz = rng.normal(size=alpha.shape[0])
    return grid, cfg, out, alpha, wz


def test_loss_gradient_directional(M, gauss64):
    """L = sum |alpha|^2 + sum w z5: <dL/dvalues, delta> against the oracle's
    complex-step derivative along random delta."""
    import torch
    grid, cfg, out, alpha, wz = _loss_setup(M, gauss64, 0.3, 4)
    res = M.adjoint(grid, cfg, out, dL_dalpha=2.0 * alpha, dL_dz=torch.tensor(wz, device="cuda"),
                    jacobian=True, cells=True)
    res1 = M.adjoint(grid, cfg, out, dL_dalpha=2.0 * alpha, dL_dz=torch.tensor(wz, device="cuda"), cells=True)
    torch.cuda.synchronize()
    g = _np(res["dL_dvalues"]).astype(np.float64)
    g1 = _np(res1["dL_dvalues"]).astype(np.float64)
    assert (_np(res["ray_status"]) == 0).all() and (_np(res1["ray_status"]) == 0).all()
    # the loss-only sweep and the combined one give the same cell gradient
    assert np.allclose(g, g1, rtol=1e-5, atol=1e-6 * np.abs(g).max())
    field = O.Field.grid(gauss64)
    c = O.cosmo(*COSMO)
    p = _oracle_params(0.3)
    dirs = oracle_dirs(4, [0], [192])
    a = _np(alpha)
    rng = np.random.default_rng(11)
    for trial in range(3):
        delta = rng.normal(size=(gauss64.n_cells, 4))
        delta[:, 0] *= 1e-5
        delta[:, 1:] *= 1e-5 / 7.8
        rec, tan = O.cast_cs(field, c, p, dirs, dphi=delta[:, 0], dgrad=delta[:, 1:])
        want = np.sum(2.0 * a * tan["alpha"]) + np.sum(wz * tan["z5"])
        got = np.sum(g * delta)
        _print(f"trial {trial}: adjoint {got:.9e} oracle {want:.9e} rel {abs(got - want) / abs(want):.2e}")
        assert abs(got - want) <= 1e-5 * abs(want)


def test_loss_gradient_single_cells(M, gauss64):
    """Per-cell derivatives on the cells with the largest gradients."""
    import torch
    grid, cfg, out, alpha, wz = _loss_setup(M, gauss64, 0.2, 2)
    res = M.adjoint(grid, cfg, out, dL_dalpha=2.0 * alpha, dL_dz=torch.tensor(wz, device="cuda"), cells=True)
    torch.cuda.synchronize()
    g = _np(res["dL_dvalues"]).astype(np.float64)
    field = O.Field.grid(gauss64)
    c = O.cosmo(*COSMO)
    p = _oracle_params(0.2)
    dirs = oracle_dirs(2, [0], [48])
    a = _np(alpha)
    top = np.argsort(-np.abs(g).max(1))[:4]
    for cell in top:
        for q in range(4):
            delta = np.zeros((gauss64.n_cells, 4))
            delta[cell, q] = 1.0
            _, tan = O.cast_cs(field, c, p, dirs, dphi=delta[:, 0], dgrad=delta[:, 1:])
            want = np.sum(2.0 * a * tan["alpha"]) + np.sum(wz * tan["z5"])
            got = g[cell, q]
            _print(f"cell {cell} comp {q}: adjoint {got:.6e} oracle {want:.6e}")
            assert abs(got - want) <= 1e-5 * np.abs(g[cell]).max() + 1e-12


def test_phi_total_central_difference(M, gauss64):
    """dL/dphi with grad phi = central difference of phi (periodic)."""
    import torch
    grid, cfg, out, alpha, wz = _loss_setup(M, gauss64, 0.3, 4)
    res = M.adjoint(grid, cfg, out, dL_dalpha=2.0 * alpha, dL_dz=torch.tensor(wz, device="cuda"), cells=True,
                    phi_total=True)
    torch.cuda.synchronize()
    gt = _np(res["dL_dphi_total"]).astype(np.float64)
    field = O.Field.grid(gauss64)
    c = O.cosmo(*COSMO)
    p = _oracle_params(0.3)
    dirs = oracle_dirs(4, [0], [192])
    a = _np(alpha)
    rng = np.random.default_rng(5)
    n = gauss64.n0
    d3 = rng.normal(size=(n, n, n)) * 1e-5
    dg3 = synth.central_gradient(d3, gauss64.box)
    ijk = gauss64.ijk
    dphi = d3[ijk[:, 0], ijk[:, 1], ijk[:, 2]]
    dgrad = dg3[ijk[:, 0], ijk[:, 1], ijk[:, 2]]
    _, tan = O.cast_cs(field, c, p, dirs, dphi=dphi, dgrad=dgrad)
    want = np.sum(2.0 * a * tan["alpha"]) + np.sum(wz * tan["z5"])
    got = np.sum(gt * dphi)
    _print(f"phi total: adjoint {got:.9e} oracle {want:.9e}")
    assert abs(got - want) <= 1e-5 * abs(want)


def test_autograd_function(M, gauss64):
    import torch
    grid = M.Grid(gauss64, COSMO)
    cfg = _cfg(M, 0.2, 2, 32)
    vals = torch.tensor(np.concatenate([gauss64.phi[:, None], gauss64.grad], 1), dtype=torch.float32,
                        device="cuda", requires_grad=True)
    alpha, z5 = M.cast_differentiable(vals, grid, cfg)
    loss = (alpha.double() ** 2).sum() + 3.0 * z5.sum()
    loss.backward()
    out = _fwd(M, grid, cfg)
    res = M.adjoint(grid, cfg, out, dL_dalpha=2.0 * out["alpha"],
                    dL_dz=torch.full((cfg.n_rays(),), 3.0, dtype=torch.float64, device="cuda"), cells=True)
    torch.cuda.synchronize()
    g_ref = _np(res["dL_dvalues"])
    g = _np(vals.grad)
    assert np.allclose(g, g_ref, rtol=1e-5, atol=1e-6 * np.abs(g_ref).max())


def test_autograd_stale_values_raise(M, gauss64):
    """The backward replays the forward on the grid's values: changing them
    between forward and backward (set_values, or a second
    cast_differentiable on the same grid) raises instead of returning a
    zero or partial gradient."""
    import torch
    grid = M.Grid(gauss64, COSMO)
    cfg = _cfg(M, 0.2, 2, 32)
    base = np.concatenate([gauss64.phi[:, None], gauss64.grad], 1)
    vals = torch.tensor(base, dtype=torch.float32, device="cuda", requires_grad=True)
    alpha, z5 = M.cast_differentiable(vals, grid, cfg)
    loss = (alpha.double() ** 2).sum()
    grid.set_values(torch.tensor(1.5 * base, dtype=torch.float32, device="cuda"))
    with pytest.raises(RuntimeError, match="changed between the forward"):
        loss.backward()
    vals2 = torch.tensor(base, dtype=torch.float32, device="cuda", requires_grad=True)
    a1, _ = M.cast_differentiable(vals2, grid, cfg)
    a2, _ = M.cast_differentiable((0.5 * vals2).detach().requires_grad_(), grid, cfg)
    with pytest.raises(RuntimeError, match="changed between the forward"):
        (a1.double() ** 2).sum().backward()
    # the latest one is still differentiable
    (a2.double() ** 2).sum().backward()


def test_amr_jacobian_vs_oracle(M):
    """Adaptive steps on a small random AMR tree (level fallback, landing)."""
    import torch
    cells = synth.random_amr_cells(16, 125.0, 3, seed=5)
    grid = M.Grid(cells, COSMO)
    obs = [40.0, 70.0, 90.0]
    cfg = M.CastConfig(obs, 0.1, 2, steps_per_cell=4, adaptive=True, checkpoint_every=32)
    out = M.cast(grid, cfg)
    res = M.adjoint(grid, cfg, out, jacobian=True)
    torch.cuda.synchronize()
    field = O.Field.grid(cells)
    c = O.cosmo(*COSMO)
    p = O.params(obs, z_src=0.1, steps_per_cell=4, adaptive=True)
    dirs = oracle_dirs(2, [0], [48])
    A, dzo, rec = O.jacobian_cs(lambda d, t: O.cast_cs(field, c, p, d, dtheta=t), dirs)
    same = _np(out["hash"]).view(np.uint32) == rec["hash"]
    jac = _np(res["jac"]).astype(np.float64)
    dA = np.abs(jac - A)[same].reshape(-1, 4).max(1)
    _print("AMR: same decisions", same.sum(), "of", len(same), "|dA| max", dA.max())
    assert same.all()
    assert dA.max() < 5e-6 and np.median(dA) < 2e-7


def test_adjoint_argument_errors(M, gauss64):
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(OBS, 0.1, 1, steps_per_cell=10)
    out = _fwd(M, grid, cfg)
    with pytest.raises(ValueError):
        M.adjoint(grid, cfg, out, jacobian=True)
    cells = synth.random_amr_cells(16, 125.0, 2, seed=5)
    g2 = M.Grid(cells, COSMO)
    cfg2 = M.CastConfig([40.0, 70.0, 90.0], 0.05, 1, steps_per_cell=4, adaptive=True, checkpoint_every=16)
    out2 = _fwd(M, g2, cfg2)
    with pytest.raises(M.MpathError):
        M.adjoint(g2, cfg2, out2, cells=True, phi_total=True)


def test_amr_loss_gradient_directional(M):
    """Cell gradient on an octree (stencils at several levels, fallback near
    refinement boundaries): <dL/dvalues, delta> against the oracle."""
    import torch
    cells = synth.random_amr_cells(16, 125.0, 3, seed=6)
    grid = M.Grid(cells, COSMO)
    obs = [40.0, 70.0, 90.0]
    cfg = M.CastConfig(obs, 0.1, 2, steps_per_cell=4, adaptive=True, checkpoint_every=16)
    out = M.cast(grid, cfg)
    alpha = out["alpha"].to(torch.float64)
    wz = np.random.default_rng(3).normal(size=alpha.shape[0])
    res = M.adjoint(grid, cfg, out, dL_dalpha=2.0 * alpha, dL_dz=torch.tensor(wz, device="cuda"), cells=True,
                    jacobian=True)
    torch.cuda.synchronize()
    assert (_np(res["ray_status"]) == 0).all()
    g = _np(res["dL_dvalues"]).astype(np.float64)
    field = O.Field.grid(cells)
    p = O.params(obs, z_src=0.1, steps_per_cell=4, adaptive=True)
    dirs = oracle_dirs(2, [0], [48])
    a = _np(alpha)
    rng = np.random.default_rng(12)
    for trial in range(2):
        delta = rng.normal(size=(cells.n_cells, 4)) * 1e-5
        _, tan = O.cast_cs(field, O.cosmo(*COSMO), p, dirs, dphi=delta[:, 0], dgrad=delta[:, 1:])
        want = np.sum(2.0 * a * tan["alpha"]) + np.sum(wz * tan["z5"])
        got = np.sum(g * delta)
        _print(f"AMR trial {trial}: adjoint {got:.9e} oracle {want:.9e}")
        assert abs(got - want) <= 1e-5 * abs(want)


def test_rays_without_derivative(M):
    """Rays that leave a non-periodic box get no derivative: NaN Jacobian,
    ray_status 1, and no contribution to the cell gradient."""
    import torch
    cells = synth.random_amr_cells(16, 125.0, 2, seed=8, periodic=False)
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig([60.0, 62.0, 58.0], 0.2, 2, steps_per_cell=4, adaptive=True, checkpoint_every=32)
    out = M.cast(grid, cfg)
    res = M.adjoint(grid, cfg, out, dL_dalpha=torch.ones((48, 2), device="cuda"), jacobian=True, cells=True)
    torch.cuda.synchronize()
    assert (_np(out["status"]) == M.MPATH_RAY_LEFT_DOMAIN).all()
    assert (_np(res["ray_status"]) == 1).all()
    assert np.isnan(_np(res["jac"])).all() and np.isnan(_np(res["dz_dtheta"])).all()
    assert (_np(res["dL_dvalues"]) == 0).all()


def test_amr_deep_jacobian_vs_oracle(M):
    """Adjoint distortion matrix on the five-level grid (a few rays through
    the refined haloes) against the oracle's complex-step Jacobian."""
    import torch
    cells = synth.make_cells("amr_deep")
    grid = M.Grid(cells, COSMO)
    obs = OBS
    cfg = M.CastConfig(obs, 0.3, 4, pix_first=[0], pix_count=[48], steps_per_cell=4, adaptive=True,
                       checkpoint_every=16)
    fwd = M.cast(grid, cfg)
    res = M.adjoint(grid, cfg, fwd, jacobian=True)
    torch.cuda.synchronize()
    jac = res["jac"].cpu().numpy().astype(np.float64)
    st = res["ray_status"].cpu().numpy()
    dirs = O.pix2vec_nest(4, np.arange(48))
    p = O.params(obs, z_src=0.3, steps_per_cell=4, adaptive=True)
    field = O.Field.grid(cells)
    A, dz, out = O.jacobian_cs(lambda d, t: O.cast_cs(field, O.cosmo(*COSMO), p, d, dtheta=t), dirs)
    ok = (st == 0) & (out["status"] == O.REACHED)
    assert ok.all() and (st == 0).all()
    d = np.abs(jac[ok] - A[ok]).max(axis=(1, 2))
    print("deep adjoint: max |dA|", d.max(), "median", np.median(d), flush=True)
    assert np.median(d) < 2e-7 and d.max() < 5e-6


def _gpu_end_dirs(M, grid, z, dirs):
    """End directions (unit vectors of x_s - x_obs) of GPU casts along dirs."""
    import torch
    from parity import beta_to_vec
    cfg = M.CastConfig(OBS, z, 16, pix_count=[len(dirs)], dirs=torch.from_numpy(np.ascontiguousarray(dirs)).cuda(),
                       steps_per_cell=10)
    out = _fwd(M, grid, cfg)
    assert (_np(out["status"]) == 0).all()
    return beta_to_vec(_np(out["beta"]))


def test_jacobian_vs_gpu_finite_differences(M, gauss64):
    """A of the reverse sweep against central differences of GPU casts: the
    192 pixel directions moved by +-1e-5 rad along e1, e2 (the screen basis
    at theta), the end directions read on the basis at the unperturbed end
    direction.  The end directions hold ~1e-11 rad; the float32 rounding
    along two neighbouring paths differs by ~1e-10 rad, i.e. ~1e-5 in the
    quotient, and a pair of paths straddling a cell face sees the kink of
    the CIC force (rare)."""
    from oracle.lensing import screen_basis
    grid = M.Grid(gauss64, COSMO)
    cfg = _cfg(M, 0.3, 4, 32)
    out = _fwd(M, grid, cfg)
    jac = _np(M.adjoint(grid, cfg, out, jacobian=True)["jac"]).astype(np.float64)
    dirs = oracle_dirs(4, [0], [192])
    e1, e2 = screen_basis(dirs)
    f1, f2 = screen_basis(_gpu_end_dirs(M, grid, 0.3, dirs))
    h = 1e-5
    unit = lambda v: v / np.linalg.norm(v, axis=1, keepdims=True)
    A = np.empty((len(dirs), 2, 2))
    for b, e in enumerate((e1, e2)):
        d = (_gpu_end_dirs(M, grid, 0.3, unit(dirs + h * e)) - _gpu_end_dirs(M, grid, 0.3, unit(dirs - h * e))) / (2 * h)
        A[:, 0, b] = np.sum(d * f1, 1)
        A[:, 1, b] = np.sum(d * f2, 1)
    diff = np.abs(jac - A).max(axis=(1, 2))
    lens = np.abs(A - np.eye(2)).max(axis=(1, 2))
    _print(f"reverse sweep vs GPU central differences: max {diff.max():.2e}, median {np.median(diff):.2e}, "
           f"|A - I| max {lens.max():.2e}")
    assert lens.max() > 1e-3
    assert np.median(diff) < 2e-5 and (diff > 1e-4).mean() <= 0.02


def test_jacobian_vs_oracle_infinitesimal_beam(M):
    """A of the reverse sweep (the exact derivative of the discrete map)
    against the oracle's infinitesimal beam (Sect. 2.3.1: the line-of-sight
    integral of the force Hessian, from differences of the interpolated
    force over the leaf size): two estimators of the same distortion that
    agree to first order in the lensing when the field is smooth on the cell
    scale.  A band-limited potential (Fourier modes with |n| <= 3 over the
    500 Mpc/h box, wavelengths >= 96 Mpc/h = 12 cells, rms 5e-5) keeps the
    difference of the two Hessians at O((k h)^2 / 6) ~ 4 % of the shortest
    modes; on the k^-3 Gaussian field the cell-scale part of the Hessian
    dominates and the two differ by up to half the signal.  The symmetric
    part of A is compared: its columns live on the e_phi basis at theta and
    its rows on the one at beta, which near the poles are rotated against
    each other by ~ alpha cot(theta) (an antisymmetric part of ~5e-4 here),
    while the beam integrates on one basis per point."""
    n, box = 64, 500.0
    ff = synth.fourier_field(box, 7, kmax=3, rms=5e-5)
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    centres = (np.stack([ii, jj, kk], -1).reshape(-1, 3) + 0.5) * (box / n)
    phi, grad = ff(centres)
    cells = synth.uniform_cells(phi.reshape(n, n, n), grad.reshape(n, n, n, 3), box)
    grid = M.Grid(cells, COSMO)
    cfg = _cfg(M, 0.3, 4, 32)
    out = _fwd(M, grid, cfg)
    jac = _np(M.adjoint(grid, cfg, out, jacobian=True)["jac"]).astype(np.float64)
    dirs = oracle_dirs(4, [0], [192])
    Ainf, rec = O.infinitesimal(O.Field.grid(cells), O.cosmo(*COSMO), _oracle_params(0.3), dirs)
    assert (rec["status"] == O.REACHED).all()
    sym = 0.5 * (jac + np.transpose(jac, (0, 2, 1)))
    diff = np.abs(sym - Ainf).max(axis=(1, 2))
    lens = np.abs(Ainf - np.eye(2)).max(axis=(1, 2))
    k_adj = 1 - 0.5 * (jac[:, 0, 0] + jac[:, 1, 1])
    k_inf = 1 - 0.5 * (Ainf[:, 0, 0] + Ainf[:, 1, 1])
    corr = np.corrcoef(k_adj, k_inf)[0, 1]
    _print(f"reverse sweep vs oracle infinitesimal beam: max |dA| {diff.max():.2e}, median {np.median(diff):.2e}, "
           f"|A - I| max {lens.max():.2e}, convergence correlation {corr:.5f}")
    assert lens.max() > 1e-3
    assert corr > 0.99 and diff.max() < 0.1 * lens.max()


def test_differentiated_full_size_sampled(M):
    """The differentiated benchmark configuration itself: all 2^20 rays
    (nside 512) to z = 1 on the 64^3 grid, checkpoints every 32 steps, the
    Jacobian and the loss gradient in the sweep the benchmark times; A and
    dz/dtheta of 48 seeded random rays against the oracle's complex step."""
    import torch
    w = synth.WORKLOADS["differentiated"]
    cells = synth.make_cells(w.grid)
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, steps_per_cell=w.steps_per_cell,
                       adaptive=w.adaptive, checkpoint_every=32)
    fwd = _fwd(M, grid, cfg)
    res = M.adjoint(grid, cfg, fwd, dL_dalpha=2 * fwd["alpha"], cells=True, jacobian=True)
    torch.cuda.synchronize()
    st = _np(res["ray_status"])
    assert (st == 0).all()
    idx = np.sort(np.random.default_rng(2026).choice(w.n_rays, 48, replace=False))
    jac = _np(res["jac"]).astype(np.float64)[idx]
    dz = _np(res["dz_dtheta"]).astype(np.float64)[idx]
    dirs = O.pix2vec_nest(w.nside, np.asarray(w.pix_first)[0] + idx)
    p = O.params(w.obs[0], z_src=float(np.atleast_1d(w.z_src)[0]), steps_per_cell=w.steps_per_cell,
                 adaptive=w.adaptive)
    A, dzo, rec = O.jacobian_cs(lambda d, t: O.cast_cs(O.Field.grid(cells), O.cosmo(*COSMO), p, d, dtheta=t), dirs)
    dA = np.abs(jac - A).reshape(-1, 4).max(1)
    rz = np.abs(dz - dzo).max(1) / np.abs(dzo).max()
    _print(f"full-size differentiated: max |dA| {dA.max():.2e}, median {np.median(dA):.2e}; "
           f"max rel dz/dtheta {rz.max():.2e}")
    assert dA.max() < 5e-6 and np.median(dA) < 2e-7
    assert rz.max() < 1e-5


def test_differentiated_full_size_cell_gradient(M):
    """The cell gradient of the differentiated configuration at full size
    (2^20 rays, every lane scattering through the per-wave tables and their
    evictions): (a) with dL/dalpha = 2 alpha on 256 seeded rays and 0 on the
    others, <dL/dvalues, delta> along two random directions against the
    oracle's complex-step directional derivative on those rays; (b) for
    L = sum |alpha|^2 over all rays, the one sweep against the sum of 16
    sweeps of 2^16 rays each: float32 atomic sums of up to 2^20 terms per
    cell (the observer's stencil takes one from every ray) round at about
    sqrt(2^20) 2^-24 = 6e-5 of the sum, the bar below."""
    import torch
    w = synth.WORKLOADS["differentiated"]
    cells = synth.make_cells(w.grid)
    grid = M.Grid(cells, COSMO)
    kw = dict(steps_per_cell=w.steps_per_cell, adaptive=w.adaptive, checkpoint_every=32)
    cfg = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, **kw)
    fwd = _fwd(M, grid, cfg)
    n = w.n_rays
    sub = np.sort(np.random.default_rng(2028).choice(n, 256, replace=False))
    cot = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    sub_t = torch.from_numpy(sub).cuda()
    cot[sub_t] = 2.0 * fwd["alpha"][sub_t]
    res = M.adjoint(grid, cfg, fwd, dL_dalpha=cot, cells=True)
    torch.cuda.synchronize()
    assert (_np(res["ray_status"]) == 0).all()
    g = _np(res["dL_dvalues"]).astype(np.float64)
    field = O.Field.grid(cells)
    p = O.params(w.obs[0], z_src=float(np.atleast_1d(w.z_src)[0]), steps_per_cell=w.steps_per_cell,
                 adaptive=w.adaptive)
    dirs = O.pix2vec_nest(w.nside, np.asarray(w.pix_first)[0] + sub)
    a = _np(fwd["alpha"])[sub].astype(np.float64)
    rng = np.random.default_rng(12)
    for trial in range(2):
        delta = rng.normal(size=(cells.n_cells, 4))
        delta[:, 0] *= 1e-5
        delta[:, 1:] *= 1e-5 / 7.8
        _, tan = O.cast_cs(field, O.cosmo(*COSMO), p, dirs, dphi=delta[:, 0], dgrad=delta[:, 1:])
        want = np.sum(2.0 * a * tan["alpha"])
        got = np.sum(g * delta)
        _print(f"full-size cell gradient, trial {trial}: adjoint {got:.9e} oracle {want:.9e} "
               f"rel {abs(got - want) / abs(want):.2e}")
        assert abs(got - want) <= 1e-5 * abs(want)
    # (b) the whole loss in one sweep and in 16 chunks of 2^16 rays
    full = M.adjoint(grid, cfg, fwd, dL_dalpha=2.0 * fwd["alpha"], cells=True)
    torch.cuda.synchronize()
    g_full = _np(full["dL_dvalues"]).astype(np.float64)
    m = 1 << 16
    g_sum = np.zeros_like(g_full)
    for c in range(n // m):
        cfg_c = M.CastConfig(w.obs, w.z_src, w.nside, [c * m], [m], **kw)
        f_c = _fwd(M, grid, cfg_c)
        r_c = M.adjoint(grid, cfg_c, f_c, dL_dalpha=2.0 * f_c["alpha"], cells=True)
        torch.cuda.synchronize()
        assert (_np(r_c["ray_status"]) == 0).all()
        g_sum += _np(r_c["dL_dvalues"]).astype(np.float64)
    scale = np.abs(g_full).max(axis=0)
    err = np.abs(g_full - g_sum).max(axis=0) / scale
    rel = np.linalg.norm(g_full - g_sum) / np.linalg.norm(g_full)
    _print(f"one sweep vs 16 chunks: max |diff| / max |g| per component {err}, relative norm {rel:.2e}")
    assert np.all(err < 1e-4) and rel < 1e-4
