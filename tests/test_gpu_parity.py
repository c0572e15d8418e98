"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs, element by element."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

COSMO = (0.3, 0.7, 0.7)


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2111_08744_amd as M
    return M


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gauss64():
    return synth.make_cells("gauss64")


@pytest.mark.parametrize("schedule", [1, 2])
def test_uniform_64_full_sky(M, gauss64, schedule):
    """64^3 uniform grid, 3072 rays (nside 16) to z = 0.5, 10 steps per cell."""
    _print("uniform 64^3, nside 16, z=0.5, schedule", schedule)
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig([250.0, 250.0, 250.0], 0.5, 16, steps_per_cell=10, schedule=schedule)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(gauss64), O.cosmo(*COSMO), [250.0, 250.0, 250.0], 0.5, 16, [0], [3072], 10, False)
    s = compare(g, o)
    _print(s)
    assert np.all(g["n_steps"] == 1692)


def test_schedules_agree(M, gauss64):
    """Every launch shape gives bit-identical results: the step arithmetic is
    written with explicit fused multiply-adds and no implicit contraction, so
    each kernel that inlines it rounds the same way."""
    grid = M.Grid(gauss64, COSMO)
    res = []
    for sched, block, batch, wpc in [(1, 256, 0, 0), (2, 256, 8, 0), (2, 0, 64, 3), (1, 0, 0, 0), (2, 0, 1, 24)]:
        cfg = M.CastConfig([250.0, 250.0, 250.0], 0.3, 8, steps_per_cell=10, schedule=sched,
                           block_size=block, batch=batch, waves_per_cu=wpc)
        res.append(run_gpu(grid, cfg))
    for r in res[1:]:
        for k in ("hash", "n_steps", "beta", "z5", "alpha", "phi_src", "status", "chi"):
            assert np.array_equal(r[k], res[0][k]), k


def test_autotuned_batched_launch(M, gauss64):
    """The autotuner picks a launch shape for a batch of cones (observers and
    source redshifts of uneven path length); results are bit-identical to the
    static schedule's and match the oracle."""
    obs, z, first, count = synth.batched_cones(500.0, 8, 8, seed=4, zlo=0.05, zhi=0.4)
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(obs, z, 8, first, count, steps_per_cell=10, schedule=1)
    tuned, ms = M.autotune(grid, cfg, sample_div=4)
    _print("autotune:", tuned.schedule, tuned.waves_per_cu, tuned.batch, f"{ms:.2f} ms")
    assert tuned.schedule in (1, 2) and ms > 0
    a = run_gpu(grid, cfg)
    b = run_gpu(grid, tuned)
    for k in ("hash", "n_steps", "beta", "z5", "alpha", "status"):
        assert np.array_equal(a[k], b[k]), k
    o = run_oracle(O.Field.grid(gauss64), O.cosmo(*COSMO), obs, z, 8, first, count, 10, False)
    _print(compare(b, o))


@pytest.mark.parametrize("name,seed", [("blobs", 5), ("blobs", 6)])
def test_amr_small_adaptive(M, name, seed):
    """Random full tree, 16^3 coarse + 3 levels, box 125 Mpc/h (periodic,
    crossed several times), adaptive steps (4 per leaf cell), nside 8 to z = 0.3."""
    cells = synth.random_amr_cells(16, 125.0, 3, seed=seed)
    _print("amr small seed", seed, "cells", cells.n_cells, cells.counts_per_level())
    grid = M.Grid(cells, COSMO)
    obs = [40.0, 70.0, 90.0]
    cfg = M.CastConfig(obs, 0.3, 8, steps_per_cell=4, adaptive=True)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(cells), O.cosmo(*COSMO), obs, 0.3, 8, [0], [768], 4, True)
    s = compare(g, o)
    _print(s)
    assert (o["n_steps"] > 400).all()          # about chi / (h0 / N) steps or more


def test_amr_halo_small(M):
    cells = synth.make_cells("amr_halo_small")
    _print("amr halo small cells", cells.n_cells, cells.counts_per_level())
    grid = M.Grid(cells, COSMO)
    obs = [125.0, 125.0, 125.0]
    cfg = M.CastConfig(obs, 0.4, 8, steps_per_cell=4, adaptive=True)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(cells), O.cosmo(*COSMO), obs, 0.4, 8, [0], [768], 4, True)
    s = compare(g, o)
    _print(s)


def test_batched_observers(M, gauss64):
    """Several observers and source redshifts in one persistent launch."""
    obs, z, first, count = synth.batched_cones(500.0, 6, 8, seed=3, zlo=0.05, zhi=0.6)
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig(obs, z, 8, first, count, steps_per_cell=10, schedule=2)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(gauss64), O.cosmo(*COSMO), obs, z, 8, first, count, 10, False)
    _print(compare(g, o))


def test_non_periodic_leaves_domain(M):
    cells = synth.random_amr_cells(16, 125.0, 2, seed=8, periodic=False)
    grid = M.Grid(cells, COSMO)
    obs = [60.0, 62.0, 58.0]
    cfg = M.CastConfig(obs, 0.2, 4, steps_per_cell=4, adaptive=True)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(cells), O.cosmo(*COSMO), obs, 0.2, 4, [0], [192], 4, True)
    assert np.all(o["status"] == O.LEFT_DOMAIN)
    s = compare(g, o)
    assert np.array_equal(g["n_steps"], o["n_steps"])
    assert np.all(np.isnan(g["z5"]))
    _print(s)


def test_max_steps(M, gauss64):
    grid = M.Grid(gauss64, COSMO)
    cfg = M.CastConfig([250.0, 250.0, 250.0], 0.5, 4, steps_per_cell=10, max_steps=100)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(gauss64), O.cosmo(*COSMO), [250.0, 250.0, 250.0], 0.5, 4, [0], [192], 10, False,
                   max_steps=100)
    assert np.all(g["status"] == M.MPATH_RAY_MAX_STEPS) and np.all(g["n_steps"] == 100)
    compare(g, o)


def test_nonfinite_cell(M):
    """A NaN in one cell's gradient stops the rays whose stencils meet it with
    status NONFINITE, in the same step as the oracle; a NaN potential in the
    observer's stencil stops every ray in its first step.  Every other ray
    agrees with the oracle at the parity bar.  (Every lookup of the cast
    masks or bounds-checks its cell indices, so the NaN positions inside the
    failing step read valid cells.)"""
    import copy
    cells = synth.make_cells("gauss32")
    obs = [125.0, 125.0, 125.0]
    for ijk, field, hit_all in (((18, 16, 16), "grad", False), ((16, 16, 16), "phi", True)):
        c = copy.deepcopy(cells)
        i = (ijk[0] * 32 + ijk[1]) * 32 + ijk[2]
        if field == "phi":
            c.phi[i] = np.nan
        else:
            c.grad[i, 1] = np.nan
        _print("NaN", field, "at cell", ijk)
        grid = M.Grid(c, COSMO)
        cfg = M.CastConfig(obs, 0.2, 4, steps_per_cell=4)
        g = run_gpu(grid, cfg)
        o = run_oracle(O.Field.grid(c), O.cosmo(*COSMO), obs, 0.2, 4, [0], [192], 4, False)
        assert np.array_equal(g["status"], o["status"])
        assert np.array_equal(g["n_steps"], o["n_steps"])
        hit = o["status"] == O.NONFINITE
        if hit_all:
            assert hit.all() and np.all(g["n_steps"] == 0)
        else:
            assert 0 < hit.sum() < len(hit) // 2
            ok = np.nonzero(~hit)[0]
            _print(compare(g, o[ok], idx=ok))


def test_static_background_chi_stop(M):
    """a = 1, a'/a = 0 (static background), stop at a comoving distance."""
    cells = synth.make_cells("gauss32")
    grid = M.Grid(cells, (0.0, 0.0, 1.0))
    cfg = M.CastConfig([10.0, 20.0, 30.0], 400.0, 4, stop_kind="chi", steps_per_cell=4)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(cells), O.STATIC, [10.0, 20.0, 30.0], 400.0, 4, [0], [192], 4, False, stop_kind="chi")
    # z5 is Phi_o - Phi_s ~ 1e-5 at first order here: compare absolutely, at
    # the level of the float32 cell values (6e-8 relative of |Phi| ~ 3e-5)
    same = g["hash"] == o["hash"]
    assert same.all()
    assert np.abs(g["z5"] - o["z5"]).max() < 5e-11
    g2 = dict(g)
    g2["z5"] = o["z5"]
    compare(g2, o)


def test_set_values_matches_rebuild(M, gauss64):
    import torch
    rng = np.random.default_rng(0)
    grid = M.Grid(gauss64, COSMO)
    scale = rng.uniform(0.5, 1.5)
    vals = np.concatenate([gauss64.phi[:, None], gauss64.grad], 1) * scale
    grid.set_values(torch.tensor(vals, dtype=torch.float32, device="cuda"))
    cfg = M.CastConfig([250.0, 250.0, 250.0], 0.2, 4, steps_per_cell=10)
    g1 = run_gpu(grid, cfg)
    c2 = synth.Cells(gauss64.box, gauss64.n0, 0, True, gauss64.level, gauss64.ijk,
                     (gauss64.phi * scale).astype(np.float32), (gauss64.grad * scale).astype(np.float32))
    g2 = run_gpu(M.Grid(c2, COSMO), cfg)
    for k in ("beta", "z5", "alpha", "phi_src", "n_steps"):
        assert np.array_equal(g1[k], g2[k]), k


def test_invalid_arguments_raise(M, gauss64):
    grid = M.Grid(gauss64, COSMO)
    with pytest.raises(M.MpathError):
        M.cast(grid, M.CastConfig([250.0, 250.0, 250.0], 25.0, 4))       # beyond the table
    with pytest.raises(M.MpathError):
        M.cast(grid, M.CastConfig([250.0, 250.0, 250.0], 0.5, 4, pix_first=[40], pix_count=[200]))
    cfg = M.CastConfig([250.0, 250.0, 250.0], 0.5, 4)
    import ctypes as C
    from paper_2111_08744_amd import _abi
    n = C.c_size_t()
    d = cfg.desc()
    d.order = 3                                  # no such interpolation order
    assert _abi.lib().mpath_cast_workspace_bytes(grid.handle, C.byref(d), C.byref(n)) == _abi.MPATH_ERR_INVALID_ARG
    d = cfg.desc()
    d.order, d.checkpoint_every = 2, 32          # TSC has no adjoint
    assert _abi.lib().mpath_cast_workspace_bytes(grid.handle, C.byref(d), C.byref(n)) == _abi.MPATH_ERR_UNSUPPORTED


def test_amr128_full_size_sampled(M):
    """The benchmark configuration itself: AMR 128^3 + 3 levels (10,035,832
    cells), all 786,432 rays (nside 256) to z = 1 in the launch the benchmark
    times; 384 seeded random rays, the 32 rays with the most steps (the
    deepest and longest paths through refined haloes) and the 32 most
    deflected, recomputed by the oracle one by one."""
    w = synth.WORKLOADS["amr"]
    cells = synth.make_cells(w.grid)
    _print("amr128 cells", cells.n_cells)
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, steps_per_cell=w.steps_per_cell,
                       adaptive=w.adaptive)
    g = run_gpu(grid, cfg)
    assert np.all(g["status"] == M.MPATH_RAY_REACHED)
    most = np.argsort(g["n_steps"], kind="stable")[-32:]
    bent = np.argsort(np.hypot(g["alpha"][:, 0], g["alpha"][:, 1]), kind="stable")[-32:]
    idx = np.unique(np.concatenate([np.random.default_rng(2024).choice(w.n_rays, 384, replace=False), most, bent]))
    _print("steps of the most-step rays", g["n_steps"][most].min(), "..", g["n_steps"].max(),
           "; median", int(np.median(g["n_steps"])))
    o = run_oracle(O.Field.grid(cells), O.cosmo(*COSMO), w.obs, w.z_src, w.nside, w.pix_first, w.pix_count,
                   w.steps_per_cell, w.adaptive, ray_index=idx)
    s = compare(g, o, idx=idx)
    _print(s)


def test_empty_and_ragged_ray_lists(M, gauss64):
    """Observers with no pixels, and one pixel, next to a full cone."""
    import torch
    grid = M.Grid(gauss64, COSMO)
    cfg0 = M.CastConfig([[250.0, 250.0, 250.0]], [0.3], 4, [0], [0], steps_per_cell=10)
    assert cfg0.n_rays() == 0
    out = M.cast(grid, cfg0)
    torch.cuda.synchronize()
    assert out["z5"].numel() == 0
    obs = [[250.0, 250.0, 250.0], [100.0, 120.0, 140.0], [400.0, 30.0, 260.0]]
    z = [0.2, 0.1, 0.3]
    first, count = [5, 0, 37], [0, 1, 16]
    for sched in (1, 2):
        cfg = M.CastConfig(obs, z, 4, first, count, steps_per_cell=10, schedule=sched)
        g = run_gpu(grid, cfg)
        o = run_oracle(O.Field.grid(gauss64), O.cosmo(*COSMO), obs, z, 4, first, count, 10, False)
        _print(compare(g, o))


def test_amr_deep_five_levels(M):
    """Five refinement levels (the depth of the largest configuration): 64^3
    coarse cells, finest 0.24 Mpc/h, adaptive steps, 768 rays (nside 8) to
    z = 0.5 against the oracle, and the level mix of the decisions."""
    cells = synth.make_cells("amr_deep")
    counts = cells.counts_per_level()
    _print("amr deep cells", cells.n_cells, counts)
    assert cells.max_level == 5 and counts[5] > 0
    grid = M.Grid(cells, COSMO)
    obs = [250.0, 250.0, 250.0]
    cfg = M.CastConfig(obs, 0.5, 8, steps_per_cell=4, adaptive=True)
    g = run_gpu(grid, cfg)
    o = run_oracle(O.Field.grid(cells), O.cosmo(*COSMO), obs, 0.5, 8, [0], [768], 4, True)
    _print(compare(g, o))
    coarse_only = 1322.038 / (500.0 / 64) * 4
    assert g["n_steps"].max() > 1.2 * coarse_only        # some rays cross the refined haloes


def test_batched_full_size_sampled(M):
    """The batched benchmark configuration itself: 64 observers, z_src in
    [0.1, 2], one NESTED base pixel at nside 128 each (1,048,576 rays of
    uneven length) in the autotuned launch the benchmark times and in the
    persistent schedule; 256 seeded random rays recomputed by the oracle."""
    w = synth.WORKLOADS["batched"]
    cells = synth.make_cells(w.grid)
    grid = M.Grid(cells, COSMO)
    cfg = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, steps_per_cell=w.steps_per_cell,
                       adaptive=w.adaptive, schedule=1)
    tuned, _ = M.autotune(grid, cfg, sample_div=8)
    _print("batched: tuned schedule", tuned.schedule, "waves/CU", tuned.waves_per_cu, "batch", tuned.batch)
    g = run_gpu(grid, tuned)
    assert np.all(g["status"] == M.MPATH_RAY_REACHED)
    p = run_gpu(grid, M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count,
                                   steps_per_cell=w.steps_per_cell, adaptive=w.adaptive, schedule=2))
    for k in ("beta", "z5", "n_steps", "hash"):
        assert np.array_equal(p[k], g[k]), k
    idx = np.sort(np.random.default_rng(2025).choice(w.n_rays, 256, replace=False))
    o = run_oracle(O.Field.grid(cells), O.cosmo(*COSMO), w.obs, w.z_src, w.nside, w.pix_first, w.pix_count,
                   w.steps_per_cell, w.adaptive, ray_index=idx)
    _print(compare(g, o, idx=idx))


def _payload(grid):
    """The packed (phi, gx, gy, gz) float32 of every cell, library order."""
    import torch
    torch.cuda.synchronize()
    return grid.ws[: 16 * grid.n_cells].view(torch.float32).reshape(-1, 4).cpu().numpy()


def _tree_central_gradient(cells):
    """The gradient rule of a grid built with grad = NULL, written out per
    cell: central differences of phi between the two same-level neighbours
    (periodic wrap), one-sided where one of them is missing, 0 where both are."""
    where = {(int(l), int(i), int(j), int(k)): c
             for c, (l, (i, j, k)) in enumerate(zip(cells.level, cells.ijk))}
    g = np.zeros((cells.n_cells, 3))
    for c in range(cells.n_cells):
        l = int(cells.level[c])
        m = cells.n0 << l
        h = cells.box / m
        for a in range(3):
            e = np.eye(3, dtype=np.int64)[a]

            def nb(sign):
                q = cells.ijk[c].astype(np.int64) + sign * e
                if cells.periodic:
                    q %= m
                elif np.any(q < 0) or np.any(q >= m):
                    return None
                return where.get((l, *map(int, q)))
            cp, cm = nb(1), nb(-1)
            if cp is not None and cm is not None:
                g[c, a] = (cells.phi[cp] - cells.phi[cm]) / (2.0 * h)
            elif cp is not None:
                g[c, a] = (cells.phi[cp] - cells.phi[c]) / h
            elif cm is not None:
                g[c, a] = (cells.phi[c] - cells.phi[cm]) / h
    return g


def test_grad_null_uniform(M, gauss64):
    """grad = NULL on a uniform periodic grid: the library's central
    differences equal synth.central_gradient bit for bit (the float32
    payload), and so do the casts."""
    import copy
    c1 = copy.deepcopy(gauss64)
    c1.grad = None
    g0, g1 = M.Grid(gauss64, COSMO), M.Grid(c1, COSMO)
    assert np.array_equal(_payload(g0), _payload(g1))
    cfg = M.CastConfig([250.0, 250.0, 250.0], 0.5, 8, steps_per_cell=10)
    r0, r1 = run_gpu(g0, cfg), run_gpu(g1, cfg)
    for k in ("beta", "z5", "alpha", "n_steps", "hash", "status"):
        assert np.array_equal(r0[k], r1[k]), k


@pytest.mark.parametrize("periodic", [True, False])
def test_grad_null_tree(M, periodic):
    """grad = NULL on a three-level tree (periodic and not): every cell's
    gradient follows the stated rule per level, and the casts equal those of
    a grid given these gradients."""
    import copy
    cells = synth.random_amr_cells(16, 125.0, 3, seed=5, periodic=periodic)
    ref = copy.deepcopy(cells)
    ref.grad = _tree_central_gradient(cells)
    c1 = copy.deepcopy(cells)
    c1.grad = None
    g0, g1 = M.Grid(ref, COSMO), M.Grid(c1, COSMO)
    p0, p1 = _payload(g0), _payload(g1)
    assert np.array_equal(p0, p1)
    obs = [60.0, 62.0, 58.0]
    cfg = M.CastConfig(obs, 0.02, 4, steps_per_cell=4, adaptive=True)
    r0, r1 = run_gpu(g0, cfg), run_gpu(g1, cfg)
    for k in ("beta", "z5", "n_steps", "hash", "status"):
        # rays that leave the non-periodic box carry NaN observables
        assert np.array_equal(r0[k], r1[k], equal_nan=k in ("beta", "z5")), k


def test_forward_only_grid(M, gauss64):
    """A grid without its auxiliary tables (aux=False: 40 B per cell less)
    casts bit for bit like the full grid and gives the same distortion
    matrices; the calls that need the tables refuse with UNSUPPORTED."""
    import torch
    from paper_2111_08744_amd import _abi
    g_full, g_fwd = M.Grid(gauss64, COSMO), M.Grid(gauss64, COSMO, aux=False)
    assert g_fwd.aux is None and g_full.aux is not None
    cfg = M.CastConfig([250.0, 250.0, 250.0], 0.3, 4, steps_per_cell=10, checkpoint_every=32)
    o_full, o_fwd = M.cast(g_full, cfg), M.cast(g_fwd, cfg)
    for k in ("beta", "z5", "n_steps", "hash"):
        assert torch.equal(o_full[k], o_fwd[k]), k
    j_full = M.adjoint(g_full, cfg, o_full, jacobian=True)["jac"]
    j_fwd = M.adjoint(g_fwd, cfg, o_fwd, jacobian=True)["jac"]
    assert torch.equal(j_full, j_fwd)
    with pytest.raises(_abi.MpathError, match="auxiliary"):
        M.adjoint(g_fwd, cfg, o_fwd, dL_dalpha=2.0 * o_fwd["alpha"], cells=True)
    with pytest.raises(_abi.MpathError, match="auxiliary"):
        g_fwd.set_values(torch.zeros((g_fwd.n_cells, 4), dtype=torch.float32, device="cuda"))
