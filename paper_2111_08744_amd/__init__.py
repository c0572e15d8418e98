"""MI355X (gfx950) weak-field null-geodesic ray tracer: Python binding.

Thin marshalling over the C ABI of ``include/mpath.h`` (``libmpath.so`` in
this directory).  PyTorch provides device memory and the current HIP stream;
every step of the ray tracing runs in the library's kernels.  The names follow
the C entry points:

    grid = Grid(cells, cosmo=(0.3, 0.7, 0.7))      # mpath_grid_build
    out  = cast(grid, CastConfig(obs, z_src, nside, ...))            # mpath_cast
    res  = adjoint(grid, cfg, out, dL_dalpha=..., jacobian=True)     # mpath_adjoint
    alpha, z5 = cast_differentiable(values, grid, cfg)  # torch.autograd.Function

Method: Breton & Reverdy, Magrathea-Pathfinder, Sect. 2 (geodesic
integration with AMR interpolation, lens equation, redshifts).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import (MPATH_RAY_LEFT_DOMAIN, MPATH_RAY_MAX_STEPS, MPATH_RAY_NONFINITE,  # noqa: F401
                   MPATH_RAY_REACHED, MPATH_SCHED_AUTO, MPATH_SCHED_PERSISTENT,
                   MPATH_SCHED_STATIC, MPATH_STOP_CHI, MPATH_STOP_REDSHIFT, MpathError)

__all__ = ["Grid", "cast", "CastConfig", "jacobian", "adjoint", "autotune", "cast_differentiable", "library_path",
           "lensing_maps", "finite_beam", "infinitesimal_beam", "born_beam", "find_geodesics",
           "MpathError"]


def library_path() -> str:
    return _abi.LIB_PATH


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Grid:
    """An octree of Phi and grad Phi resident on the GPU (mpath_grid_build).

    cells: an object with box, n0, max_level, periodic, level[n] (uint8),
    ijk[n,3] (int32), phi[n], grad[n,3] (float64 or float32 numpy arrays;
    grad None: the library's central differences of phi) and optionally
    dphi_deta[n] (a time-dependent potential, Sect. 2.2).
    cosmo: (omega_m, omega_l, h); (0, 0, h) is a static background.
    aux: also build the auxiliary tables (40 B per cell) that set_values and
    the cell cotangents of the adjoint need; a forward-only grid
    (aux=False) casts and differentiates per ray all the same.
    """

    def __init__(self, cells, cosmo=(0.3, 0.7, 0.7), device="cuda", aux=True):
        torch = _torch()
        L = _abi.lib()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the grid lives in GPU memory")
        level = np.ascontiguousarray(cells.level, np.uint8)
        ijk = np.ascontiguousarray(cells.ijk, np.int32)
        f32 = np.asarray(cells.phi).dtype == np.float32
        vt = np.float32 if f32 else np.float64
        phi = np.ascontiguousarray(cells.phi, vt)
        grad = None if cells.grad is None else np.ascontiguousarray(cells.grad, vt)
        td = getattr(cells, "dphi_deta", None)
        td = None if td is None else np.ascontiguousarray(td, vt)
        if td is not None and td.shape != phi.shape:
            raise ValueError("dphi_deta must have one value per cell")
        self.time_dependent = td is not None
        self._keep = (level, ijk, phi, grad, td)
        d = _abi.mpath_grid_desc()
        d.box = float(cells.box)
        d.n0 = int(cells.n0)
        d.max_level = int(cells.max_level)
        d.periodic = int(bool(cells.periodic))
        d.value_dtype = _abi.MPATH_F32 if f32 else _abi.MPATH_F64
        d.n_cells = len(level)
        d.level = level.ctypes.data
        d.ijk = ijk.ctypes.data
        d.phi = phi.ctypes.data
        d.grad = None if grad is None else grad.ctypes.data
        d.dphi_deta = None if td is None else td.ctypes.data
        nbytes = C.c_size_t()
        _abi.check(L.mpath_grid_workspace_bytes(C.byref(d), C.byref(nbytes)), "mpath_grid_workspace_bytes")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.aux = None
        if aux:
            abytes = C.c_size_t()
            _abi.check(L.mpath_grid_aux_bytes(C.byref(d), C.byref(abytes)), "mpath_grid_aux_bytes")
            self.aux = torch.empty(abytes.value, dtype=torch.uint8, device=self.device)
        cz = _abi.mpath_cosmo(*map(float, cosmo))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _abi.check(L.mpath_grid_build_with_aux(C.byref(d), C.byref(cz), _ptr(self.ws), nbytes.value,
                                                   None if self.aux is None else _ptr(self.aux),
                                                   0 if self.aux is None else self.aux.numel(),
                                                   _stream_ptr(self.device), C.byref(h)), "mpath_grid_build_with_aux")
        self._h = h
        self._keep = None
        self.values_version = 0      # counts set_values calls
        self.cosmo = tuple(map(float, cosmo))
        info = _abi.mpath_grid_info()
        _abi.check(L.mpath_grid_get_info(self._h, C.byref(info)), "mpath_grid_get_info")
        self.n_cells = info.n_cells
        self.max_level = info.max_level
        self.n0 = info.n0
        self.box = info.box
        self.eta0 = info.eta0
        self.cells_per_level = list(info.cells_per_level[: info.max_level + 1])
        self.payload_ptr = info.payload
        self.perm_ptr = info.perm

    @property
    def handle(self):
        return self._h

    def set_values(self, values):
        """values: float32 CUDA tensor [n_cells, 4] = (phi, gx, gy, gz) in the
        caller's cell order (mpath_grid_set_values)."""
        torch = _torch()
        assert values.is_cuda and values.dtype == torch.float32 and values.shape == (self.n_cells, 4)
        values = values.contiguous()
        _abi.check(_abi.lib().mpath_grid_set_values(self._h, _ptr(values), _stream_ptr(self.device)),
                   "mpath_grid_set_values")
        self.values_version += 1
        self._values_ref = values     # keep alive until the stream is done with it

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _abi.lib().mpath_grid_free(h)
            except Exception:   # interpreter shutdown: module globals already gone
                pass
            self._h = None


class CastConfig:
    """Everything mpath_cast_desc holds besides the grid (host side)."""

    def __init__(self, obs, stop, nside, pix_first=None, pix_count=None, stop_kind="z",
                 steps_per_cell=10, adaptive=False, max_steps=1 << 40, schedule=0,
                 block_size=0, waves_per_cu=0, batch=0, checkpoint_every=0, dirs=None, order=1, surfaces=None,
                 stop_surface="eta", dphidl="chain"):
        self.obs = np.ascontiguousarray(np.atleast_2d(obs), np.float64)
        self.stop = np.ascontiguousarray(np.atleast_1d(stop), np.float64)
        self.nside = int(nside)
        self.pix_first = None if pix_first is None else np.ascontiguousarray(np.atleast_1d(pix_first), np.int64)
        self.pix_count = None if pix_count is None else np.ascontiguousarray(np.atleast_1d(pix_count), np.int64)
        self.stop_kind = {"z": MPATH_STOP_REDSHIFT, "chi": MPATH_STOP_CHI}[stop_kind] \
            if isinstance(stop_kind, str) else int(stop_kind)
        self.steps_per_cell = int(steps_per_cell)
        self.adaptive = bool(adaptive)
        self.max_steps = int(max_steps)
        self.schedule = int(schedule)
        self.block_size = int(block_size)
        self.waves_per_cu = int(waves_per_cu)
        self.batch = int(batch)
        self.checkpoint_every = int(checkpoint_every)
        self.order = int(order)          # 0 NGP, 1 CIC, 2 TSC
        # the parameter the stop surface holds (mpath_cast_desc.stop_surface)
        self.stop_surface = {"eta": 0, "chi": 1, "lambda": 2, "z": 3}[stop_surface] \
            if isinstance(stop_surface, str) else int(stop_surface)
        # dPhi/dlambda: "chain" (chain rule) or "diff" (difference between step starts)
        self.dphidl = {"chain": 0, "diff": 1}[dphidl] if isinstance(dphidl, str) else int(dphidl)
        # intermediate stop surfaces [n_obs, n_s] (or [n_s] for every observer),
        # nearest first, each nearer than the observer's stop
        if surfaces is not None:
            sf = np.atleast_1d(np.asarray(surfaces, np.float64))
            if sf.ndim == 1:
                sf = np.tile(sf, (self.obs.shape[0], 1))
            surfaces = np.ascontiguousarray(sf)
        self.surfaces = surfaces
        # initial directions: None = NESTED pixel centres; else a float64 CUDA
        # tensor [n_rays, 3] of unit vectors (pix_count gives the rays per observer)
        if dirs is not None:
            if not (dirs.is_cuda and dirs.dtype == _torch().float64 and dirs.dim() == 2 and dirs.shape[1] == 3):
                raise ValueError("dirs must be a float64 CUDA tensor of shape [n_rays, 3]")
            dirs = dirs.contiguous()
        self.dirs = dirs

    def desc(self) -> _abi.mpath_cast_desc:
        d = _abi.mpath_cast_desc()
        d.n_obs = self.obs.shape[0]
        d.obs_pos = self.obs.ctypes.data
        d.stop_value = self.stop.ctypes.data
        d.stop_kind = self.stop_kind
        d.nside = self.nside
        d.pix_first = self.pix_first.ctypes.data if self.pix_first is not None else None
        d.pix_count = self.pix_count.ctypes.data if self.pix_count is not None else None
        d.order = self.order
        d.steps_per_cell = self.steps_per_cell
        d.adaptive = int(self.adaptive)
        d.max_steps = self.max_steps
        d.schedule = self.schedule
        d.block_size = self.block_size
        d.waves_per_cu = self.waves_per_cu
        d.batch = self.batch
        d.checkpoint_every = self.checkpoint_every
        d.dirs = self.dirs.data_ptr() if self.dirs is not None else None
        d.n_surfaces = 0 if self.surfaces is None else self.surfaces.shape[1]
        d.surface_stops = None if self.surfaces is None else self.surfaces.ctypes.data
        d.stop_surface = self.stop_surface
        d.dphidl = self.dphidl
        return d

    def n_blocks(self) -> int:
        """Output blocks of n_rays: one per stop surface."""
        return 1 if self.surfaces is None else self.surfaces.shape[1] + 1

    def n_rays(self) -> int:
        n = C.c_int64()
        d = self.desc()
        _abi.check(_abi.lib().mpath_cast_count_rays(C.byref(d), C.byref(n)), "mpath_cast_count_rays")
        return n.value


_OUT_FIELDS = {
    "beta": ("float64", 2), "alpha": ("float32", 2), "z5": ("float64", 1), "z0": ("float64", 1),
    "phi_src": ("float32", 1), "n_steps": ("int32", 1), "status": ("int32", 1), "hash": ("int32", 1),
    "chi": ("float64", 1), "z1": ("float64", 1), "z4": ("float64", 1), "isw": ("float64", 1),
}


def alloc_outputs(n_rays: int, device="cuda", fields=None):
    torch = _torch()
    out = {}
    for k, (dt, w) in _OUT_FIELDS.items():
        if fields is not None and k not in fields:
            continue
        shape = (n_rays, w) if w > 1 else (n_rays,)
        out[k] = torch.empty(shape, dtype=getattr(torch, dt), device=device)
    return out


def observables_struct(out) -> _abi.mpath_observables:
    o = _abi.mpath_observables()
    for k in _OUT_FIELDS:
        setattr(o, k, out[k].data_ptr() if k in out else None)
    return o


def cast(grid: Grid, cfg: CastConfig, out=None, ws=None):
    """mpath_cast: cast every ray of cfg on the current stream of the grid's
    device; returns the dict of output tensors (see mpath_observables)."""
    torch = _torch()
    L = _abi.lib()
    d = cfg.desc()
    n = cfg.n_rays()
    if cfg.dirs is not None and cfg.dirs.shape[0] != n:
        raise ValueError(f"dirs has {cfg.dirs.shape[0]} rows for {n} rays")
    if out is None:
        out = alloc_outputs(n * cfg.n_blocks(), grid.device)
    nbytes = C.c_size_t()
    _abi.check(L.mpath_cast_workspace_bytes(grid.handle, C.byref(d), C.byref(nbytes)), "mpath_cast_workspace_bytes")
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=grid.device)
    obs = observables_struct(out)
    with torch.cuda.device(grid.device):
        _abi.check(L.mpath_cast(grid.handle, C.byref(d), C.byref(obs), _ptr(ws), ws.numel(),
                                _stream_ptr(grid.device)), "mpath_cast")
    out["_ws"] = ws
    return out


def jacobian(grid: Grid, cfg: CastConfig, out=None, ws=None):
    """mpath_cast_jacobian: the cast of every ray of cfg (the outputs of
    ``cast``, bit for bit) with the distortion matrix ``jac`` [n_rays, 2, 2]
    (A_ab = d beta_a / d theta_b) and ``dz_dtheta`` [n_rays, 2] by
    forward-mode differentiation in the same pass."""
    torch = _torch()
    L = _abi.lib()
    d = cfg.desc()
    n = cfg.n_rays()
    if cfg.dirs is not None and cfg.dirs.shape[0] != n:
        raise ValueError(f"dirs has {cfg.dirs.shape[0]} rows for {n} rays")
    if out is None:
        out = alloc_outputs(n, grid.device)
    for k in ("jac", "dz_dtheta"):
        if k not in out:
            out[k] = torch.empty((n, 2, 2) if k == "jac" else (n, 2), dtype=torch.float32, device=grid.device)
    nbytes = C.c_size_t()
    _abi.check(L.mpath_cast_jacobian_workspace_bytes(grid.handle, C.byref(d), C.byref(nbytes)),
               "mpath_cast_jacobian_workspace_bytes")
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=grid.device)
    obs = observables_struct(out)
    with torch.cuda.device(grid.device):
        _abi.check(L.mpath_cast_jacobian(grid.handle, C.byref(d), C.byref(obs), _ptr(out["jac"]),
                                         _ptr(out["dz_dtheta"]), _ptr(ws), ws.numel(), _stream_ptr(grid.device)),
                   "mpath_cast_jacobian")
    out["_ws"] = ws
    return out


def adjoint(grid: Grid, cfg: CastConfig, fwd, dL_dalpha=None, dL_dz=None, jacobian=False, cells=False,
            phi_total=False, ws=None):
    """mpath_adjoint: reverse sweep over the checkpointed cast ``fwd`` (the
    dict returned by ``cast`` with cfg.checkpoint_every > 0, on the same grid
    values).

    jacobian: return ``jac`` [n_rays, 2, 2] (A_ab = d beta_a / d theta_b) and
    ``dz_dtheta`` [n_rays, 2].  cells: return ``dL_dvalues`` [n_cells, 4],
    the derivative of the loss with per-ray cotangents dL_dalpha [n_rays, 2]
    (float32) and dL_dz [n_rays] (float64) with respect to the cell values
    (phi, gx, gy, gz) in the caller's order.  phi_total (uniform periodic
    grids): also ``dL_dphi_total`` [n_cells] for a gradient defined as the
    central difference of phi.  ``ray_status`` [n_rays]: 0 derivative
    computed, 1 ray not reached (no derivative), 2 replay mismatch."""
    torch = _torch()
    L = _abi.lib()
    d = cfg.desc()
    if cfg.checkpoint_every <= 0:
        raise ValueError("the adjoint needs a cast with checkpoint_every > 0")
    n = cfg.n_rays()
    dev = grid.device
    res = {}
    ad = _abi.mpath_adjoint_desc()
    keep = []
    if dL_dalpha is not None:
        dL_dalpha = dL_dalpha.to(device=dev, dtype=torch.float32).contiguous()
        assert dL_dalpha.shape == (n, 2)
        keep.append(dL_dalpha)
        ad.dL_dalpha = dL_dalpha.data_ptr()
    if dL_dz is not None:
        dL_dz = dL_dz.to(device=dev, dtype=torch.float64).contiguous()
        assert dL_dz.shape == (n,)
        keep.append(dL_dz)
        ad.dL_dz = dL_dz.data_ptr()
    if jacobian:
        res["jac"] = torch.empty((n, 2, 2), dtype=torch.float32, device=dev)
        res["dz_dtheta"] = torch.empty((n, 2), dtype=torch.float32, device=dev)
        ad.jac = res["jac"].data_ptr()
        ad.dz_dtheta = res["dz_dtheta"].data_ptr()
    if cells:
        res["dL_dvalues"] = torch.empty((grid.n_cells, 4), dtype=torch.float32, device=dev)
        ad.dL_dvalues = res["dL_dvalues"].data_ptr()
    if phi_total:
        res["dL_dphi_total"] = torch.empty((grid.n_cells,), dtype=torch.float32, device=dev)
        ad.dL_dphi_total = res["dL_dphi_total"].data_ptr()
    res["ray_status"] = torch.empty((n,), dtype=torch.int32, device=dev)
    ad.ray_status = res["ray_status"].data_ptr()
    nbytes = C.c_size_t()
    _abi.check(L.mpath_adjoint_workspace_bytes(grid.handle, C.byref(d), C.byref(nbytes)),
               "mpath_adjoint_workspace_bytes")
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
    obs = observables_struct(fwd)
    cast_ws = fwd["_ws"]
    with torch.cuda.device(dev):
        _abi.check(L.mpath_adjoint(grid.handle, C.byref(d), C.byref(obs), _ptr(cast_ws), cast_ws.numel(),
                                   C.byref(ad), _ptr(ws), ws.numel(), _stream_ptr(dev)), "mpath_adjoint")
    res["_ws"] = ws
    res["_keep"] = keep
    return res


def _autograd_function():
    torch = _torch()

    class CastFunction(torch.autograd.Function):
        """(alpha [n_rays, 2], z5 [n_rays]) as functions of the cell values
        [n_cells, 4] = (phi, gx, gy, gz) in the caller's order; backward runs
        mpath_adjoint, which replays the forward path on the grid's values:
        the grid must keep these values until the backward (a set_values or
        another cast_differentiable on the same Grid in between raises
        there), and a ray whose replay does not retrace its forward path bit
        for bit raises too instead of contributing nothing."""

        @staticmethod
        def forward(ctx, values, grid, cfg):
            if cfg.checkpoint_every <= 0:
                raise ValueError("cast_differentiable needs cfg.checkpoint_every > 0")
            grid.set_values(values.detach().to(torch.float32))
            out = cast(grid, cfg)
            ctx.grid, ctx.cfg, ctx.out = grid, cfg, out
            ctx.values_version = grid.values_version
            return out["alpha"].clone(), out["z5"].clone()

        @staticmethod
        def backward(ctx, g_alpha, g_z5):
            if ctx.grid.values_version != ctx.values_version:
                raise RuntimeError("cast_differentiable: the grid's cell values changed between the forward "
                                   "and the backward (set_values or another cast_differentiable on this Grid)")
            res = adjoint(ctx.grid, ctx.cfg, ctx.out, dL_dalpha=g_alpha, dL_dz=g_z5, cells=True)
            bad = int((res["ray_status"] == 2).sum())
            if bad:
                raise RuntimeError(f"cast_differentiable: {bad} rays did not retrace their forward path in the "
                                   "reverse sweep (the cell values differ from the forward's)")
            return res["dL_dvalues"], None, None

    return CastFunction


_CAST_FN = None


def cast_differentiable(values, grid: Grid, cfg: CastConfig):
    """torch.autograd entry: sets the grid's cell values (float32 [n_cells,
    4], caller order), casts with checkpoints and returns (alpha, z5); their
    gradients flow back to ``values`` through mpath_adjoint."""
    global _CAST_FN
    if _CAST_FN is None:
        _CAST_FN = _autograd_function()
    return _CAST_FN.apply(values, grid, cfg)


def autotune(grid: Grid, cfg: CastConfig, sample_div: int = 8):
    """mpath_autotune: time candidate launch shapes on a sample of cfg's rays
    (1/sample_div of every observer's pixels) and return (a copy of cfg with
    the fastest schedule, waves_per_cu and batch, the sample's time in ms)."""
    import copy
    torch = _torch()
    L = _abi.lib()
    d = cfg.desc()
    nbytes = C.c_size_t()
    _abi.check(L.mpath_autotune_workspace_bytes(grid.handle, C.byref(d), int(sample_div), C.byref(nbytes)),
               "mpath_autotune_workspace_bytes")
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=grid.device)
    tuned = _abi.mpath_cast_desc()
    ms = C.c_float()
    with torch.cuda.device(grid.device):
        _abi.check(L.mpath_autotune(grid.handle, C.byref(d), int(sample_div), _ptr(ws), ws.numel(),
                                    _stream_ptr(grid.device), C.byref(tuned), C.byref(ms)), "mpath_autotune")
    out = copy.copy(cfg)
    out.schedule = tuned.schedule
    out.waves_per_cu = tuned.waves_per_cu
    out.batch = tuned.batch
    return out, ms.value


def lensing_maps(A):
    """mpath_lensing_maps: (kappa, gamma1, gamma2, omega, mu) [n, 5] float32 of
    distortion matrices A [n, 2, 2] (float32 CUDA tensor)."""
    torch = _torch()
    if not (A.is_cuda and A.dtype == torch.float32 and A.dim() == 3 and tuple(A.shape[1:]) == (2, 2)):
        raise ValueError("A must be a float32 CUDA tensor of shape [n, 2, 2]")
    A = A.contiguous()
    out = torch.empty((A.shape[0], 5), dtype=torch.float32, device=A.device)
    with torch.cuda.device(A.device):
        _abi.check(_abi.lib().mpath_lensing_maps(_ptr(A), A.shape[0], _ptr(out), _stream_ptr(A.device)),
                   "mpath_lensing_maps")
    return out


def finite_beam(grid: Grid, cfg: CastConfig, eps: float, ws=None):
    """mpath_finite_beam: finite-beam distortion matrices [n_rays, 2, 2] and the
    beam status [n_rays] of every ray of cfg, beams of semi-aperture eps (rad)."""
    torch = _torch()
    L = _abi.lib()
    d = cfg.desc()
    n = cfg.n_rays()
    if cfg.dirs is not None and cfg.dirs.shape[0] != n:
        raise ValueError(f"dirs has {cfg.dirs.shape[0]} rows for {n} rays")
    nbytes = C.c_size_t()
    _abi.check(L.mpath_finite_beam_workspace_bytes(grid.handle, C.byref(d), C.byref(nbytes)),
               "mpath_finite_beam_workspace_bytes")
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=grid.device)
    A = torch.empty((n, 2, 2), dtype=torch.float32, device=grid.device)
    st = torch.empty((n,), dtype=torch.int32, device=grid.device)
    with torch.cuda.device(grid.device):
        _abi.check(L.mpath_finite_beam(grid.handle, C.byref(d), float(eps), _ptr(A), _ptr(st), _ptr(ws),
                                       ws.numel(), _stream_ptr(grid.device)), "mpath_finite_beam")
    return {"A": A, "status": st, "_ws": ws}


def infinitesimal_beam(grid: Grid, cfg: CastConfig, out=None, ws=None):
    """mpath_infinitesimal_beam: cast every ray of cfg (outputs as ``cast``) and
    integrate its infinitesimal-beam distortion matrix, returned as ``A``
    [n_rays, 2, 2] float32 (NaN for rays that did not reach the source)."""
    torch = _torch()
    L = _abi.lib()
    d = cfg.desc()
    n = cfg.n_rays()
    if cfg.dirs is not None and cfg.dirs.shape[0] != n:
        raise ValueError(f"dirs has {cfg.dirs.shape[0]} rows for {n} rays")
    if out is None:
        out = alloc_outputs(n, grid.device)
    nbytes = C.c_size_t()
    _abi.check(L.mpath_cast_workspace_bytes(grid.handle, C.byref(d), C.byref(nbytes)), "mpath_cast_workspace_bytes")
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=grid.device)
    A = torch.empty((n, 2, 2), dtype=torch.float32, device=grid.device)
    obs = observables_struct(out)
    with torch.cuda.device(grid.device):
        _abi.check(L.mpath_infinitesimal_beam(grid.handle, C.byref(d), C.byref(obs), _ptr(A), _ptr(ws), ws.numel(),
                                              _stream_ptr(grid.device)), "mpath_infinitesimal_beam")
    out["A"] = A
    out["_ws"] = ws
    return out


def find_geodesics(grid: Grid, obs, src, steps_per_cell=10, adaptive=False, tol=1e-10, max_iter=10,
                   identity_iters=3, checkpoint_every=32, max_steps=1 << 40, ws=None, grid_rounds=0, grid_n=5,
                   grid_max=0):
    """mpath_find_geodesics: initial directions theta [n, 3] connecting the
    observer obs [3] to sources at comoving positions src [n, 3] (host
    arrays), with the exact distortion matrix A [n, 2, 2], dz5/dtheta [n, 2],
    z5, z0, phi_src, the final angle sep to beta, n_iter and the status.
    grid_rounds > 0 adds the grid-search fallback (grid_n x grid_n
    candidates, at most grid_max sources, 0 = all)."""
    torch = _torch()
    L = _abi.lib()
    obs = np.ascontiguousarray(obs, np.float64).reshape(3)
    src = np.ascontiguousarray(src, np.float64).reshape(-1, 3)
    n = src.shape[0]
    d = _abi.mpath_finder_desc()
    d.obs_pos = obs.ctypes.data
    d.n_src = n
    d.src_pos = src.ctypes.data if n else None
    d.order = 1
    d.steps_per_cell = int(steps_per_cell)
    d.adaptive = int(bool(adaptive))
    d.max_steps = int(max_steps)
    d.tol = float(tol)
    d.max_iter = int(max_iter)
    d.identity_iters = int(identity_iters)
    d.checkpoint_every = int(checkpoint_every)
    d.grid_rounds = int(grid_rounds)
    d.grid_n = int(grid_n)
    d.grid_max = int(grid_max)
    nbytes = C.c_size_t()
    _abi.check(L.mpath_find_geodesics_workspace_bytes(grid.handle, C.byref(d), C.byref(nbytes)),
               "mpath_find_geodesics_workspace_bytes")
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=grid.device)
    dev = grid.device
    res = {"theta": torch.empty((n, 3), dtype=torch.float64, device=dev),
           "A": torch.empty((n, 2, 2), dtype=torch.float32, device=dev),
           "dz_dtheta": torch.empty((n, 2), dtype=torch.float32, device=dev),
           "z5": torch.empty((n,), dtype=torch.float64, device=dev),
           "z0": torch.empty((n,), dtype=torch.float64, device=dev),
           "z1": torch.empty((n,), dtype=torch.float64, device=dev),
           "phi_src": torch.empty((n,), dtype=torch.float32, device=dev),
           "sep": torch.empty((n,), dtype=torch.float64, device=dev),
           "n_iter": torch.empty((n,), dtype=torch.int32, device=dev),
           "status": torch.empty((n,), dtype=torch.int32, device=dev)}
    o = _abi.mpath_finder_out()
    for k, v in res.items():
        setattr(o, k, v.data_ptr() if n else None)
    with torch.cuda.device(dev):
        _abi.check(L.mpath_find_geodesics(grid.handle, C.byref(d), C.byref(o), _ptr(ws), ws.numel(),
                                          _stream_ptr(dev)), "mpath_find_geodesics")
    res["_ws"] = ws
    return res


def born_beam(grid: Grid, cfg: CastConfig, ws=None):
    """mpath_born_beam: Born-approximation distortion matrices [n_rays, 2, 2]
    along the straight lines of cfg's initial directions, and the status."""
    torch = _torch()
    L = _abi.lib()
    d = cfg.desc()
    n = cfg.n_rays()
    if cfg.dirs is not None and cfg.dirs.shape[0] != n:
        raise ValueError(f"dirs has {cfg.dirs.shape[0]} rows for {n} rays")
    nbytes = C.c_size_t()
    _abi.check(L.mpath_cast_workspace_bytes(grid.handle, C.byref(d), C.byref(nbytes)), "mpath_cast_workspace_bytes")
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=grid.device)
    A = torch.empty((n, 2, 2), dtype=torch.float32, device=grid.device)
    st = torch.empty((n,), dtype=torch.int32, device=grid.device)
    with torch.cuda.device(grid.device):
        _abi.check(L.mpath_born_beam(grid.handle, C.byref(d), _ptr(A), _ptr(st), _ptr(ws), ws.numel(),
                                     _stream_ptr(grid.device)), "mpath_born_beam")
    return {"A": A, "status": st, "_ws": ws}


def double_layer(phi1, phi2, a1, a2, cosmo=(0.3, 0.7, 0.7)):
    """mpath_double_layer: dPhi/deta of every cell from the potential on two
    light cones slightly shifted in time (Sect. 2.2), phi1 at scale factors
    a1 and phi2 at a2 (arrays, or scalars for the whole grid); returns a
    float64 numpy array, for the dphi_deta field of a grid's cells."""
    phi1 = np.ascontiguousarray(phi1, np.float64)
    phi2 = np.ascontiguousarray(phi2, np.float64)
    if phi1.shape != phi2.shape or phi1.ndim != 1:
        raise ValueError("phi1 and phi2 must be 1-d arrays of equal length")
    n = phi1.shape[0]
    a1 = np.ascontiguousarray(np.broadcast_to(np.asarray(a1, np.float64), (n,)))
    a2 = np.ascontiguousarray(np.broadcast_to(np.asarray(a2, np.float64), (n,)))
    out = np.empty(n, np.float64)
    cz = _abi.mpath_cosmo(*map(float, cosmo))
    _abi.check(_abi.lib().mpath_double_layer(n, phi1.ctypes.data, phi2.ctypes.data, a1.ctypes.data, a2.ctypes.data,
                                             C.byref(cz), out.ctypes.data), "mpath_double_layer")
    return out


def healpix_dirs(nside: int, pix_first: int = 0, count=None, device="cuda"):
    """mpath_healpix_dirs: NESTED pixel-centre directions [count, 3] (float64
    CUDA tensor) of pixels pix_first .. pix_first + count - 1."""
    torch = _torch()
    count = 12 * nside * nside - pix_first if count is None else int(count)
    out = torch.empty((count, 3), dtype=torch.float64, device=device)
    with torch.cuda.device(out.device):
        _abi.check(_abi.lib().mpath_healpix_dirs(int(nside), int(pix_first), count, _ptr(out) if count else None,
                                                 _stream_ptr(out.device)), "mpath_healpix_dirs")
    return out
