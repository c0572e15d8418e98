#!/usr/bin/env python3
"""Benchmark: backward null-geodesic ray tracing through an AMR octree on one MI355X.

Default workload (one "step" = one full cast of every ray): the 512^3 + 5
level light cone, the largest configuration that one GPU holds: 512^3 coarse
cells + 5 refinement levels (box 2000 Mpc/h, Gaussian potential
P(k) ~ k^-3 with rms 1e-5 plus 1,900 truncated NFW-like haloes, 950 of them
within 400 Mpc/h of the observer; 407,828,120 cells, float32 Phi + grad Phi
on the GPU); observer at the box centre; the full sky at HEALPix NESTED
nside 2048 (50,331,648 rays) to z = 2; 4 RK4 steps per leaf cell.

Prints one JSON line: ray-steps/s (value), rays/s, the roofline of the cast
kernel (random-gather bound: algorithmic stencil bytes per ray-step over the
kernel time, against HBM and against the measured random-gather ceiling at
the grid image's footprint), the targets with pass/fail, secondary workloads
(AMR 128^3 + 3 levels, adjoint, batched launch, lensing products, finder,
orders, variants) and the FP64 CPU oracle's rate on a bounded sample of the
same rays.

    python bench.py [--steps K] [--warmup W] [--workload large|amr|uniform|batched]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic arithmetic of one ray-step of the method (RK4 with CIC
# interpolation of Phi and grad Phi at four sub-steps and the geodesic
# right-hand side), counted as floating-point operations with a fused
# multiply-add = 2: ~560 FP32 + ~20 FP64.
FLOPS_PER_RAY_STEP = 580.0
# Published FP32 vector peak of the MI355X (packed FP32: 256 CUs x 128
# lanes x 2 flops x 2.4 GHz) and the issue rate of unpacked FP32 and FP64
# vector FMAs, which is what this kernel uses (packed FP32 is disabled).
PEAK_FP32_TFLOPS = 157.3
ISSUE_RATE_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# Peak HBM bandwidth of the MI355X.
PEAK_HBM_GBS = 8000.0


def algo_bytes_per_ray_step(steps_per_cell):
    """Unique table bytes one ray-step needs with perfect stencil reuse: a
    new CIC stencil brings 4 new cells of 16 bytes, at most
    (|n_x|+|n_y|+|n_z|)/N <= sqrt(3)/N times per step (N steps per cell)."""
    return 64.0 * 3 ** 0.5 / steps_per_cell


WORKLOAD_TEXT = {
    "large": "512^3 coarse + 5 levels (box 2000 Mpc/h, 407,828,120 cells), full sky nside 2048 "
             "(50,331,648 rays) to z = 2, 4 steps per leaf cell",
    "amr": "AMR 128^3 coarse + 3 levels (box 500 Mpc/h, 10,035,832 cells), 786,432 rays (nside 256) to z = 1, "
           "4 steps per leaf cell",
    "uniform": "uniform 64^3, 3072 rays (nside 16) to z = 0.5, 10 steps per cell",
    "batched": "64 cones x 16384 rays on the 64^3 grid, z_src in [0.1, 2]",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import synth
    w = synth.WORKLOADS[name]
    cells = synth.make_cells(w.grid, log=lambda m: log("[bench] grid:", m))
    return w, cells


def host_cores():
    """(threads the oracle may use, nproc, CPU model): the CPUs this process
    may run on, capped by OMP_NUM_THREADS as nproc does."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, n, model


# Sources the forward integration kernel and its launch are built from (the
# adjoint's source does not change it).
CAST_SOURCES = ("cast.hip", "device.h", "internal.h", "grid.hip", "mpath_host.cpp")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2111_08744_amd", "csrc")
    for f in CAST_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(wl_name):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/), if they
    were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{wl_name}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(w, cells, sample_stride, threads):
    """The FP64 oracle on every sample_stride-th ray of the same workload."""
    import oracle as O
    t0 = time.time()
    field = O.Field.grid(cells)
    c = O.cosmo(0.3, 0.7, 0.7)
    obs = w.obs[0]
    pix = np.arange(w.pix_first[0], w.pix_first[0] + w.pix_count[0], sample_stride)
    dirs = O.pix2vec_nest(w.nside, pix)
    p = O.params(obs, z_src=float(w.z_src[0]), steps_per_cell=w.steps_per_cell, adaptive=w.adaptive)
    setup = time.time() - t0
    t0 = time.time()
    rec = O.cast(field, c, p, dirs, threads=threads)
    dt = time.time() - t0
    steps = int(rec["n_steps"].sum())
    return {"value": steps / dt, "unit": "ray-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(pix)} of {int(w.pix_count[0])} rays (every {sample_stride}th NESTED pixel), "
                      f"full paths, {steps} ray-steps in {dt:.1f} s (grid setup {setup:.1f} s untimed)",
            "rays_per_s": len(pix) / dt}


def cpu_table1():
    """The oracle's single-thread time per ray-step for the interpolation
    modes of the paper's timing table (FLRW without lookups, NGP, CIC, TSC on
    the uniform 64^3 grid; CIC on the AMR 128^3 + 3 levels grid), on a few
    rays each."""
    import oracle as O
    import synth
    c = O.cosmo(0.3, 0.7, 0.7)
    obs = [250.0, 250.0, 250.0]
    dirs = O.pix2vec_nest(4, np.arange(0, 192, 6))          # 32 rays
    g64 = synth.make_cells("gauss64")
    h0 = 500.0 / 64

    def per_step(field, p, d):
        t0 = time.perf_counter()
        rec = O.cast(field, c, p, d, threads=1)
        dt = time.perf_counter() - t0
        return dt / int(rec["n_steps"].sum()) * 1e6

    res = {"flrw": per_step(O.Field.linear([0.0, 0.0, 0.0]), O.params(obs, z_src=0.5, ds=h0 / 10), dirs)}
    for order, name in ((0, "ngp"), (1, "cic"), (2, "tsc")):
        res[f"uniform_{name}"] = per_step(O.Field.grid(g64, order=order),
                                          O.params(obs, z_src=0.5, steps_per_cell=10), dirs)
    w = synth.WORKLOADS["amr"]
    res["amr_cic"] = per_step(O.Field.grid(synth.make_cells(w.grid)),
                              O.params(w.obs[0], z_src=float(w.z_src[0]), steps_per_cell=4, adaptive=True), dirs[:8])
    return {"us_per_ray_step": res, "threads": 1,
            "paper_table1_us_per_step": {"flrw": 0.55, "ngp": 1.10, "cic": 6.0, "tsc": 14.6},
            "paper_hardware": "one core of an Intel Xeon Platinum 8168"}


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time_ms(torch, fn, reps=2):
    """Minimum over reps of fn's GPU time (HIP events on the current stream)."""
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = _events(torch)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def measure_gather_ceiling(M, torch, table, dev):
    """Random-record gather throughput (mpath_gather_probe) over a table of the
    grid image's size: records of 16, 64 and 128 bytes at uniform random
    indices, 1 or 4 reads in flight per lane, 4 to 32 waves per CU. Returns the
    best rate per record size in GB/s of records read."""
    from paper_2111_08744_amd import _abi
    L = _abi.lib()
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    stream = torch.cuda.current_stream(dev).cuda_stream
    best = {}
    for rec in (16, 64, 128):
        for wpc in (4, 8, 16, 32):
            for u in (1, 4):
                n_waves = n_cu * wpc
                iters = max(1, round((1 << 31) / (n_waves * 64 * u * rec)))
                out = torch.empty(n_waves * 64, dtype=torch.float32, device=dev)

                def run():
                    _abi.check(L.mpath_gather_probe(table.data_ptr(), table.numel(), rec, u, n_waves, iters,
                                                    12345, out.data_ptr(), stream), "mpath_gather_probe")
                ms = _time_ms(torch, run, reps=3)
                gbs = n_waves * 64 * iters * u * rec / (ms / 1e3) / 1e9
                if gbs > best.get(rec, {}).get("GB_per_s", 0.0):
                    best[rec] = {"GB_per_s": gbs, "waves_per_cu": wpc, "in_flight": u}
    log("[bench] random gathers over %.2f GB: %s" % (table.numel() / 1e9, ", ".join(
        f"{r} B records {b['GB_per_s']:.0f} GB/s ({b['waves_per_cu']} waves/CU, {b['in_flight']} in flight)"
        for r, b in best.items())))
    return best


def measure_adjoint(M, torch, dev):
    """Differentiated workload: 2^20 rays (NESTED nside 512, pixels [0, 2^20))
    to z = 1 on the uniform 64^3 grid, 10 steps per cell, checkpoints every 32
    steps; the reverse sweep gives the 2x2 distortion matrix and dz/dtheta of
    every ray and dL/d(cell values) for L = sum |alpha|^2."""
    import synth
    w = synth.WORKLOADS["differentiated"]
    grid = M.Grid(synth.make_cells(w.grid), (0.3, 0.7, 0.7), device=dev)
    kw = dict(steps_per_cell=w.steps_per_cell, adaptive=w.adaptive)
    cfg0 = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, schedule=1, **kw)
    cfgK = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, checkpoint_every=32, **kw)
    out0 = M.alloc_outputs(w.n_rays, dev)
    t_fwd = _time_ms(torch, lambda: M.cast(grid, cfg0, out0, out0.get("_ws")))
    outK = M.alloc_outputs(w.n_rays, dev)
    t_ckpt = _time_ms(torch, lambda: M.cast(grid, cfgK, outK, outK.get("_ws")))
    alpha2 = 2.0 * outK["alpha"]
    res = {}
    t_adj = _time_ms(torch, lambda: res.update(M.adjoint(grid, cfgK, outK, dL_dalpha=alpha2, jacobian=True,
                                                          cells=True, ws=res.get("_ws"))), reps=1)
    steps = int(outK["n_steps"].to(torch.int64).sum())
    bad = int((res["ray_status"] != 0).sum())
    # the loss gradient alone (one cotangent column) and the distortion matrix
    # by forward-mode tangents in the cast itself
    res1 = {}
    t_loss = _time_ms(torch, lambda: res1.update(M.adjoint(grid, cfgK, outK, dL_dalpha=alpha2, cells=True,
                                                            ws=res1.get("_ws"))), reps=1)
    outJ = M.alloc_outputs(w.n_rays, dev)
    jres = {}
    t_tan = _time_ms(torch, lambda: jres.update(M.jacobian(grid, cfg0, outJ, jres.get("_ws"))))
    log(f"[bench] adjoint: forward {t_fwd:.1f} ms, checkpointed forward {t_ckpt:.1f} ms, "
        f"reverse sweep {t_adj:.1f} ms ({t_adj / t_fwd:.2f}x), {steps} ray-steps, {bad} rays not differentiated; "
        f"loss-only reverse sweep {t_loss:.1f} ms ({t_loss / t_fwd:.2f}x); forward-mode distortion matrix "
        f"{t_tan:.1f} ms ({t_tan / t_fwd:.2f}x)")
    return {"workload": "2^20 rays (nside 512) to z = 1 on the uniform 64^3 grid, 10 steps per cell, "
                        "checkpoint every 32 steps; A, dz/dtheta per ray and dL/dcells, L = sum |alpha|^2",
            "ray_steps": steps, "forward_ms": t_fwd, "checkpointed_forward_ms": t_ckpt,
            "reverse_ms": t_adj, "adjoint_forward_ratio": t_adj / t_fwd,
            "forward_plus_adjoint_ratio": (t_ckpt + t_adj) / t_fwd, "rays_not_differentiated": bad,
            "reverse_loss_only_ms": t_loss, "reverse_loss_only_forward_ratio": t_loss / t_fwd,
            "forward_mode_jacobian_ms": t_tan, "forward_mode_jacobian_forward_ratio": t_tan / t_fwd,
            "jacobian_by_tangents_plus_loss_by_reverse_ratio": (t_tan + t_ckpt + t_loss) / t_fwd}


def measure_batched(M, torch, dev):
    """64 observers at seeded positions, z_src U[0.1, 2], one NESTED base
    pixel at nside 128 each (1,048,576 rays of uneven length) on the uniform
    64^3 grid: one autotuned launch against 64 one-cone launches."""
    import synth
    w = synth.WORKLOADS["batched"]
    grid = M.Grid(synth.make_cells(w.grid), (0.3, 0.7, 0.7), device=dev)
    kw = dict(steps_per_cell=w.steps_per_cell, adaptive=w.adaptive)
    cfg = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, schedule=1, **kw)
    tuned, tune_ms = M.autotune(grid, cfg, sample_div=8)
    out = M.alloc_outputs(w.n_rays, dev)
    t_one = _time_ms(torch, lambda: M.cast(grid, tuned, out, out.get("_ws")))
    steps = int(out["n_steps"].to(torch.int64).sum())
    t_static = _time_ms(torch, lambda: M.cast(grid, cfg, out, out.get("_ws")))
    cones = [M.CastConfig(w.obs[j], w.z_src[j], w.nside, [w.pix_first[j]], [w.pix_count[j]], schedule=1, **kw)
             for j in range(len(w.obs))]
    outs = [M.alloc_outputs(int(w.pix_count[j]), dev) for j in range(len(w.obs))]

    def per_cone():
        for c, o in zip(cones, outs):
            M.cast(grid, c, o, o.get("_ws"))
    t_cones = _time_ms(torch, per_cone, reps=1)
    log(f"[bench] batched: tuned launch (schedule {tuned.schedule}, waves/CU {tuned.waves_per_cu}, "
        f"batch {tuned.batch}) {t_one:.1f} ms, static launch {t_static:.1f} ms, "
        f"64 one-cone launches {t_cones:.1f} ms ({t_cones / t_one:.2f}x)")
    return {"workload": "64 cones x 16384 rays (nside 128 base pixels), z_src U[0.1, 2], uniform 64^3 grid",
            "ray_steps": steps, "tuned": {"schedule": tuned.schedule, "waves_per_cu": tuned.waves_per_cu,
                                          "batch": tuned.batch, "sample_ms": tune_ms},
            "one_launch_ms": t_one, "static_launch_ms": t_static, "one_cone_per_launch_ms": t_cones,
            "one_launch_ray_steps_per_s": steps / (t_one / 1e3),
            "speedup_vs_one_cone_per_launch": t_cones / t_one}


def measure_lensing(M, torch, dev):
    """Lensing products on the 64^3 uniform grid: 196,608 rays (nside 128, full
    sky) to z = 1, 10 steps per cell.  Plain cast, cast with the
    infinitesimal-beam matrix, finite beam (five rays per beam, one launch)
    and the kappa/gamma/omega/mu decomposition of the matrices."""
    import synth
    grid = M.Grid(synth.make_cells("gauss64"), (0.3, 0.7, 0.7), device=dev)
    cfg = M.CastConfig([250.0, 250.0, 250.0], 1.0, 128, steps_per_cell=10, schedule=1)
    n = cfg.n_rays()
    out = M.alloc_outputs(n, dev)
    t_plain = _time_ms(torch, lambda: M.cast(grid, cfg, out, out.get("_ws")))
    inf = {}
    t_inf = _time_ms(torch, lambda: inf.update(M.infinitesimal_beam(grid, cfg, ws=inf.get("_ws"))))
    fb = {}
    t_fb = _time_ms(torch, lambda: fb.update(M.finite_beam(grid, cfg, 1e-3, ws=fb.get("_ws"))))
    maps = {}
    t_maps = _time_ms(torch, lambda: maps.update(m=M.lensing_maps(inf["A"])))
    kap = maps["m"][:, 0]
    log(f"[bench] lensing ({n} rays): cast {t_plain:.2f} ms, infinitesimal beam {t_inf:.2f} ms, "
        f"finite beam {t_fb:.2f} ms, maps {t_maps:.3f} ms; kappa rms {float(kap.std()):.3e}")
    return {"workload": "196608 rays (nside 128) to z = 1 on the uniform 64^3 grid, 10 steps per cell",
            "rays": n, "cast_ms": t_plain, "infinitesimal_beam_ms": t_inf, "finite_beam_ms": t_fb,
            "finite_beam_eps": 1e-3, "lensing_maps_ms": t_maps,
            "infinitesimal_beam_rays_per_s": n / (t_inf / 1e3), "finite_beam_rays_per_s": n / (t_fb / 1e3)}


def measure_finder(M, torch, dev):
    """Geodesic finder on the 64^3 uniform grid: 16,384 sources at seeded
    positions around the box centre, comoving distances uniform in
    [200, 2300] Mpc/h (z up to about 1), tolerance 1e-9 rad; identity
    Newton steps first, then the exact Jacobian."""
    import synth
    grid = M.Grid(synth.make_cells("gauss64"), (0.3, 0.7, 0.7), device=dev)
    rng = np.random.default_rng(31)
    obs = np.array([250.0, 250.0, 250.0])
    v = rng.standard_normal((16384, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    src = obs + v * rng.uniform(200.0, 2300.0, len(v))[:, None]
    res = {}
    t = _time_ms(torch, lambda: res.update(M.find_geodesics(grid, obs, src, tol=1e-9, ws=res.get("_ws"))), reps=1)
    it = res["n_iter"].cpu().numpy()
    hist = np.bincount(it[it >= 0]).tolist()
    log(f"[bench] finder: {len(src)} sources in {t:.1f} ms, converged {int((it >= 0).sum())}, "
        f"iterations {hist}, max sep {float(res['sep'].max()):.2e} rad")
    # the grid-search fallback alone: two identity iterations leave the
    # first 2,048 sources unconverged, then 5 x 5 candidate rounds
    sub = src[:2048]
    g = {}
    tg = _time_ms(torch, lambda: g.update(M.find_geodesics(grid, obs, sub, tol=1e-9, max_iter=2, identity_iters=2,
                                                           grid_rounds=40, grid_n=5, ws=g.get("_ws"))), reps=1)
    itg = g["n_iter"].cpu().numpy()
    rounds = np.bincount(itg[itg >= 2] - 2).tolist()
    log(f"[bench] finder grid search: {len(sub)} sources in {tg:.1f} ms, converged {int((itg >= 0).sum())}, "
        f"rounds {rounds}")
    return {"workload": "16384 sources, chi U[200, 2300] Mpc/h, uniform 64^3 grid, tol 1e-9 rad",
            "sources": len(src), "ms": t, "sources_per_s": len(src) / (t / 1e3),
            "converged": int((it >= 0).sum()), "iterations_histogram": hist,
            "grid_search": {"workload": "the first 2048 sources: 2 identity iterations, then 5x5 grid rounds",
                            "ms": tg, "converged": int((itg >= 0).sum()), "rounds_histogram": rounds}}


def measure_variants(M, torch, dev):
    """The cast variants on the same rays, 196,608 rays (nside 128) to z = 1
    on the uniform 64^3 grid, 10 steps per cell: the plain cast; with
    dPhi/deta from the two synthetic layers (Sect. 2.2) and the ISW integral;
    the iso-chi, iso-lambda and iso-z stops (Sect. 2.4); the second form of
    the geodesic equations (dPhi/dl from step differences); three more stop
    surfaces at z = 0.25, 0.5, 0.75 in the same cast."""
    import synth
    cz = (0.3, 0.7, 0.7)
    c1 = synth.make_cells("gauss64")
    grid = M.Grid(c1, cz, device=dev)
    c2 = synth.make_cells("gauss64")
    c2.dphi_deta = M.double_layer(c1.phi, synth.make_cells("gauss64_layer2").phi, *synth.ISW_LAYER_A, cz)
    tgrid = M.Grid(c2, cz, device=dev)
    obs = [250.0, 250.0, 250.0]
    base = dict(steps_per_cell=10, schedule=1)
    cases = (("plain", grid, {}), ("time_dependent", tgrid, {}), ("iso_chi", grid, {"stop_surface": "chi"}),
             ("iso_lambda", grid, {"stop_surface": "lambda"}), ("iso_z", grid, {"stop_surface": "z"}),
             ("step_difference", grid, {"dphidl": "diff"}), ("surfaces_4", grid, {"surfaces": [0.25, 0.5, 0.75]}))
    res = {}
    for label, gr, kw in cases:
        cfg = M.CastConfig(obs, 1.0, 128, **base, **kw)
        n = cfg.n_rays()
        out = M.alloc_outputs(n * cfg.n_blocks(), dev)
        t = _time_ms(torch, lambda: M.cast(gr, cfg, out, out.get("_ws")))
        steps = int(out["n_steps"][-n:].to(torch.int64).sum())
        res[label] = {"ms": t, "ray_steps": steps, "ray_steps_per_s": steps / (t / 1e3)}
    plain = res["plain"]["ms"]
    for v in res.values():
        v["cost_vs_plain"] = v["ms"] / plain
    log("[bench] variants (uniform, nside 128, z = 1): " + ", ".join(
        f"{k} {v['ms']:.2f} ms ({v['ray_steps_per_s'] / 1e9:.2f} G ray-steps/s)" for k, v in res.items()))
    return {"workload": "196608 rays (nside 128) to z = 1 on the uniform 64^3 grid, 10 steps per cell",
            **res}


def measure_ray_order(M, torch, dev, grid, w):
    """Why rays are ordered by NESTED pixel: the AMR workload's 786,432 rays
    cast along the same directions, once in NESTED order (neighbouring rays
    in a wave share stencil lines) and once randomly permuted (seed 5)."""
    dirs = M.healpix_dirs(w.nside, int(w.pix_first[0]), int(w.pix_count[0]), device=dev)
    perm = torch.from_numpy(np.random.default_rng(5).permutation(dirs.shape[0])).to(dev)
    res = {}
    for label, td in (("nested", dirs), ("shuffled", dirs[perm].contiguous())):
        cfg = M.CastConfig(w.obs, w.z_src, w.nside, pix_count=[td.shape[0]], dirs=td, steps_per_cell=w.steps_per_cell,
                           adaptive=w.adaptive, schedule=1)
        out = M.alloc_outputs(td.shape[0], dev)
        res[label] = {"ms": _time_ms(torch, lambda: M.cast(grid, cfg, out, out.get("_ws")))}
    res["shuffled_over_nested"] = res["shuffled"]["ms"] / res["nested"]["ms"]
    log(f"[bench] ray order (AMR cast): NESTED {res['nested']['ms']:.1f} ms, shuffled {res['shuffled']['ms']:.1f} ms "
        f"({res['shuffled_over_nested']:.2f}x)")
    return {"workload": "the AMR workload's rays as caller directions, NESTED order vs a random permutation", **res}


def measure_orders(M, torch, dev):
    """The three interpolation orders (Sect. 2.2) on the same rays: 196,608
    rays (nside 128) to z = 1 on the uniform 64^3 grid and 49,152 rays
    (nside 64) to z = 1 on the AMR 128^3 + 3 levels grid; time per ray-step."""
    import synth
    res = {}
    for name, grid_name, nside, spc, adaptive in (("uniform", "gauss64", 128, 10, False),
                                                  ("amr", "amr128", 64, 4, True)):
        grid = M.Grid(synth.make_cells(grid_name), (0.3, 0.7, 0.7), device=dev)
        obs = [250.0, 250.0, 250.0]
        row = {}
        for order, label in ((0, "ngp"), (1, "cic"), (2, "tsc")):
            cfg = M.CastConfig(obs, 1.0, nside, steps_per_cell=spc, adaptive=adaptive, schedule=1, order=order)
            out = M.alloc_outputs(cfg.n_rays(), dev)
            t = _time_ms(torch, lambda: M.cast(grid, cfg, out, out.get("_ws")))
            steps = int(out["n_steps"].to(torch.int64).sum())
            row[label] = {"ms": t, "ray_steps": steps, "ray_steps_per_s": steps / (t / 1e3)}
        res[name] = row
        del grid
        log(f"[bench] orders ({name}): " + ", ".join(
            f"{k} {v['ms']:.2f} ms ({v['ray_steps_per_s'] / 1e9:.2f} G ray-steps/s)" for k, v in row.items()))
    return res


def time_casts(M, torch, grid, cfg, out, steps, warmup, label):
    """warmup untimed casts, then steps casts each bracketed by HIP events on
    the stream the library launches on (torch's current stream); returns
    (wall seconds of the timed region, per-launch event milliseconds)."""
    dev = grid.device
    ws = None
    for _ in range(warmup):
        ws = M.cast(grid, cfg, out, ws)["_ws"]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(stream)
        ws = M.cast(grid, cfg, out, ws)["_ws"]
        evs[i][1].record(stream)
        if steps > 4 and (i + 1) % 5 == 0:
            log(f"[bench] {label}: {i + 1} of {steps} timed casts queued")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in evs]


def roofline(w, ray_steps, launch_ms, traffic, ceiling_gbs=None):
    """Random-gather roofline of the cast kernel: algorithmic stencil bytes
    per launch over the mean launch time, against peak HBM bandwidth and
    against the measured random-gather ceiling; the ALU view beside it."""
    kern_s = float(np.mean(launch_ms)) / 1e3
    algo = algo_bytes_per_ray_step(w.steps_per_cell)
    achieved = algo * ray_steps / kern_s / 1e9
    flops = FLOPS_PER_RAY_STEP * ray_steps / kern_s / 1e12
    r = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
         "traffic": traffic, "kernel": "cast_static_kernel", "launch_ms_mean": float(np.mean(launch_ms)),
         "algorithmic_bytes_per_ray_step": algo, "ray_steps_per_launch": ray_steps,
         "algorithmic_bytes_per_launch": algo * ray_steps,
         "alu_view": {"achieved_TFLOP_s": flops, "flops_per_ray_step": FLOPS_PER_RAY_STEP,
                      "peak_fp32_TFLOP_s": PEAK_FP32_TFLOPS, "frac_of_peak_fp32": flops / PEAK_FP32_TFLOPS,
                      "unpacked_issue_rate_TFLOP_s": ISSUE_RATE_TFLOPS,
                      "frac_of_unpacked_issue_rate": flops / ISSUE_RATE_TFLOPS}}
    if traffic is not None:
        r["hbm_bytes_per_ray_step"] = traffic / ray_steps
        r["hbm_GB_per_s"] = traffic / kern_s / 1e9
    if ceiling_gbs is not None:
        r["measured_gather_ceiling_GB_per_s"] = ceiling_gbs
        r["frac_of_measured_gather_ceiling"] = achieved / ceiling_gbs
    return r


def measure_secondary_amr(M, torch, dev, steps):
    """The AMR 128^3 + 3 levels workload (786,432 rays to z = 1) as a
    secondary line, with its own gather roofline."""
    w, cells = workload("amr")
    grid = M.Grid(cells, (0.3, 0.7, 0.7), device=dev, aux=False)
    cfg = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, steps_per_cell=w.steps_per_cell,
                       adaptive=w.adaptive)
    out = M.alloc_outputs(cfg.n_rays(), dev)
    wall, ms = time_casts(M, torch, grid, cfg, out, steps, 1, "amr")
    ray_steps = int(out["n_steps"].to(torch.int64).sum())
    res = {"workload": WORKLOAD_TEXT["amr"], "cells": int(cells.n_cells), "rays": cfg.n_rays(),
           "ray_steps_per_cast": ray_steps, "ray_steps_per_s": ray_steps * steps / wall,
           "rays_per_s": cfg.n_rays() * steps / wall, "ms_per_cast": wall * 1e3 / steps,
           "roofline": roofline(w, ray_steps, ms, traffic_from_profiles("amr"))}
    res["ray_order"] = measure_ray_order(M, torch, dev, grid, w)
    log(f"[bench] amr: {res['ray_steps_per_s'] / 1e9:.2f} G ray-steps/s, {res['ms_per_cast']:.2f} ms per cast")
    return res


LARGE_NEED_GIB = 120


def host_available_gib():
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) / 2 ** 20
    except OSError:
        pass
    return float("inf")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=None,
                    help="large (default: the 512^3 + 5 level light cone) or amr")
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workloads (AMR 128^3, adjoint, batched launch, products)")
    ap.add_argument("--no-gather-probe", action="store_true",
                    help="skip the random-gather ceiling measurement")
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="oracle on every n-th NESTED pixel (default: 16,384 rays of the workload)")
    ap.add_argument("--only", default=None,
                    choices=("amr", "adjoint", "batched", "lensing", "finder", "orders", "variants"),
                    help="run one secondary measurement alone (no headline cast; for profiling) and print it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the casts, copy MIB mebibytes once with a plain device copy "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(rays would be sharded by sky pixel with the grid replicated on every GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2111_08744_amd as M

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda:0")
    if args.only:
        fn = {"amr": lambda: measure_secondary_amr(M, torch, dev, 5), "adjoint": lambda: measure_adjoint(M, torch, dev),
              "batched": lambda: measure_batched(M, torch, dev), "lensing": lambda: measure_lensing(M, torch, dev),
              "finder": lambda: measure_finder(M, torch, dev), "orders": lambda: measure_orders(M, torch, dev),
              "variants": lambda: measure_variants(M, torch, dev)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    fallback = None
    if args.workload is None:
        # the light cone's tree takes about 60 GB of host memory and the
        # oracle's copy of it (CPU baseline) about 40 GB more
        avail = host_available_gib()
        args.workload = "large"
        if avail < LARGE_NEED_GIB:
            args.workload = "amr"
            fallback = (f"{avail:.0f} GiB of host memory available, below the {LARGE_NEED_GIB} GiB the 512^3 + 5 "
                        f"level light cone needs: the AMR 128^3 workload instead")
            log(f"[bench] {fallback}")
    t0 = time.time()
    w, cells = workload(args.workload)
    t_gen = time.time() - t0
    log(f"[bench] workload {w.name}: grid {w.grid} with {cells.n_cells} cells, {w.n_rays} rays, "
        f"generated in {t_gen:.1f} s")
    torch.cuda.synchronize()
    t0 = time.time()
    grid = M.Grid(cells, (0.3, 0.7, 0.7), device=dev, aux=False)
    torch.cuda.synchronize()
    t_build = time.time() - t0
    log(f"[bench] grid build {t_build:.2f} s ({grid.ws.numel() / 1e9:.1f} GB), cells per level "
        f"{grid.cells_per_level}")
    cfg = M.CastConfig(w.obs, w.z_src, w.nside, w.pix_first, w.pix_count, steps_per_cell=w.steps_per_cell,
                       adaptive=w.adaptive, schedule=args.schedule, block_size=args.block,
                       waves_per_cu=args.waves_per_cu, batch=args.batch)
    n_rays = cfg.n_rays()
    out = M.alloc_outputs(n_rays, dev)
    wall, launch_ms = time_casts(M, torch, grid, cfg, out, args.steps, args.warmup, w.name)
    # every cast integrates the same rays: count the work from the last one
    n_steps = out["n_steps"].to(torch.int64)
    ray_steps = int(n_steps.sum().item())
    status = torch.bincount(out["status"].to(torch.int64), minlength=4).tolist()
    log(f"[bench] {ray_steps} ray-steps per cast; statuses {status}; steps/ray "
        f"min {int(n_steps.min())} mean {ray_steps / n_rays:.1f} max {int(n_steps.max())}")
    ms_per_step = wall * 1e3 / args.steps
    value = ray_steps * args.steps / wall
    log(f"[bench] {args.steps} casts in {wall:.3f} s: {value / 1e9:.2f} G ray-steps/s, "
        f"launch mean {np.mean(launch_ms):.2f} ms (min {np.min(launch_ms):.2f}, max {np.max(launch_ms):.2f})")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {nbytes} bytes copied")
        del src, dst

    # the distortion matrix of every ray by forward-mode tangents, one pass
    jac_line = None
    if not args.no_secondary and w.adaptive:
        jw = {}
        torch.cuda.synchronize()
        ev = _events(torch)
        ev[0].record()
        jw.update(M.jacobian(grid, cfg))
        ev[1].record()
        torch.cuda.synchronize()
        t_j = ev[0].elapsed_time(ev[1])
        jac_line = {"ms": t_j, "forward_ms": float(np.mean(launch_ms)), "ratio_to_forward": t_j / float(np.mean(launch_ms)),
                    "rays_per_s": n_rays / (t_j / 1e3), "all_finite": bool(torch.isfinite(jw["jac"]).all())}
        log(f"[bench] forward-mode distortion matrix of all {n_rays} rays: {t_j:.0f} ms "
            f"({jac_line['ratio_to_forward']:.2f}x the cast)")
        del jw
    ceiling = None
    probe = None
    if not args.no_gather_probe:
        probe = measure_gather_ceiling(M, torch, grid.ws, dev)
        ceiling = max(b["GB_per_s"] for b in probe.values())
    roof = roofline(w, ray_steps, launch_ms, traffic_from_profiles(w.name), ceiling)
    if probe is not None:
        roof["gather_probe"] = {"table_bytes": int(grid.ws.numel()), "best_per_record_bytes":
                                {str(r): b for r, b in probe.items()},
                                "kind": "uniform random record gathers over a table the size of the grid image"}
    res = {
        "metric": "ray-steps/sec + rays/sec to z_src at 1 GPU; adjoint/forward cost ratio",
        "value": value,
        "unit": "ray-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT.get(w.name, w.name),
            "cells": int(cells.n_cells), "rays": n_rays, "ray_steps_per_cast": ray_steps,
            "steps_per_cell": w.steps_per_cell, "adaptive": bool(w.adaptive),
            **({"fallback": fallback} if fallback else {}),
        },
        "rays_per_s": n_rays * args.steps / wall,
        "adjoint_forward_ratio": None,
        "grid_generate_s": t_gen,
        "grid_build_s": t_build,
        "grid_device_bytes": int(grid.ws.numel()),
        "roofline": roof,
    }
    if jac_line is not None:
        res["distortion_matrix_forward_mode"] = jac_line
    del grid, out
    torch.cuda.empty_cache()
    if not args.no_secondary:
        sec = {"amr": measure_secondary_amr(M, torch, dev, 5)}
        sec.update({"adjoint": measure_adjoint(M, torch, dev), "batched": measure_batched(M, torch, dev),
                    "lensing": measure_lensing(M, torch, dev), "finder": measure_finder(M, torch, dev),
                    "orders": measure_orders(M, torch, dev), "variants": measure_variants(M, torch, dev)})
        res["secondary"] = sec
        res["adjoint_forward_ratio"] = sec["adjoint"]["adjoint_forward_ratio"]
    targets = {}
    if ceiling is not None:
        f = roof["frac_of_measured_gather_ceiling"]
        targets["forward_ge_0.6_of_measured_gather_ceiling"] = {"value": f, "pass": f >= 0.6}
    if "secondary" in res:
        r = res["adjoint_forward_ratio"]
        targets["adjoint_le_3x_forward"] = {"value": r, "pass": r <= 3.0,
                                            "what": "reverse sweep (distortion matrix and cell gradient) / cast"}
        r = res["secondary"]["adjoint"]["forward_mode_jacobian_forward_ratio"]
        targets["distortion_matrix_le_3x_forward"] = {"value": r, "pass": r <= 3.0,
                                                      "what": "forward-mode distortion matrix / cast"}
        b = res["secondary"]["batched"]["speedup_vs_one_cone_per_launch"]
        targets["batched_ge_2x_one_cone_per_launch"] = {"value": b, "pass": b >= 2.0}
        o = res["secondary"]["orders"]
        for grid in ("uniform", "amr"):
            r = o[grid]["tsc"]["ms"] / o[grid]["cic"]["ms"]
            targets[f"tsc_le_3x_cic_{grid}"] = {"value": r, "pass": r <= 3.0, "what": "TSC cast time / CIC cast time"}
    res["targets"] = targets
    if not args.no_cpu_baseline:
        threads, nproc, model = host_cores()
        stride = args.cpu_stride or max(1, n_rays // 16384)
        log(f"[bench] CPU baseline: oracle on every {stride}th ray with {threads} threads ({model})")
        res["cpu_baseline"] = cpu_baseline(w, cells, stride, threads)
        res["cpu_baseline"].update({"nproc": nproc, "cpu_model": model})
        log(f"[bench] CPU baseline: {res['cpu_baseline']['value'] / 1e6:.2f} M ray-steps/s")
        if not args.no_secondary:
            res["cpu_baseline"]["single_thread"] = cpu_table1()
            log(f"[bench] oracle single-thread us/step: {res['cpu_baseline']['single_thread']['us_per_ray_step']}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
