"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *draws* inputs: cell lists of an octree carrying a potential
and its gradient, observer positions, source redshifts and sky-pixel ranges.
It contains none of the ray-tracing arithmetic (no geodesics, field
evaluation along rays, cosmology or HEALPix geometry); both implementations
of the method receive what is built here as plain arrays.  The one
interpolation it does, a periodic trilinear sampling of the coarse
potential, only sets the values of refined cells when a tree is drawn.

Every generator takes an explicit seed and uses numpy's PCG64 stream, so the
same call gives bit-identical arrays on every machine with this image.

The paper ran on RayGal light cones (Sect. 3), which are not available here;
the recipes below stand in for them at the scales the paper quotes: coarse
cells of a few Mpc/h, refinement of +3 to +5 levels in haloes, |Phi| of order
1e-5 and potential wells reaching a few 1e-5 (Sect. 3.2).

Units: lengths in Mpc/h, Phi dimensionless (Phi/c^2).
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

__all__ = [
    "sphere_and_uniform_centres", "LARGE_OBS",
    "Cells", "gaussian_potential", "central_gradient", "uniform_cells",
    "fourier_field", "random_amr_cells", "amr_halo_cells", "Workload",
    "WORKLOADS", "make_cells", "batched_cones", "second_layer", "ISW_LAYER_A",
]


@dataclasses.dataclass
class Cells:
    """A flat cell list of a full octree (every cell, internal or leaf).

    level[i]  refinement level of cell i (0 = coarse)
    ijk[i]    integer coordinates of cell i at its own level, in
              [0, n0 * 2**level)
    phi[i]    potential sampled at the centre of cell i
    grad[i]   gradient of the potential at the centre of cell i
    dphi_deta optional time derivative of the potential per cell (None: a
              static potential)
    """
    box: float
    n0: int
    max_level: int
    periodic: bool
    level: np.ndarray   # uint8 [n]
    ijk: np.ndarray     # int32 [n, 3]
    phi: np.ndarray     # float64 [n]
    grad: np.ndarray    # float64 [n, 3]
    dphi_deta: Optional[np.ndarray] = None

    @property
    def n_cells(self) -> int:
        return int(self.level.shape[0])

    def counts_per_level(self):
        return np.bincount(self.level, minlength=self.max_level + 1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Gaussian random potential with P(k) ~ k^slope on a periodic grid
# ---------------------------------------------------------------------------
def gaussian_potential(n: int, box: float, seed: int, rms: float = 1e-5,
                       slope: float = -3.0) -> np.ndarray:
    """Periodic Gaussian field with power spectrum ~ k^slope, rescaled so the
    grid rms is exactly `rms`.  Real white noise -> rfftn -> * k^(slope/2)
    (k = 0 mode removed) -> irfftn."""
    rng = _rng(seed)
    white = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(white)
    kx = np.fft.fftfreq(n, d=box / n)
    kz = np.fft.rfftfreq(n, d=box / n)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)          # |k|^(slope/2)
    field = np.fft.irfftn(wk * amp, s=(n, n, n), axes=(0, 1, 2))
    field -= field.mean()
    field *= rms / np.sqrt(np.mean(field ** 2))
    return field


def central_gradient(phi: np.ndarray, box: float) -> np.ndarray:
    """Second-order periodic central differences of a cubic grid -> [n,n,n,3]."""
    n = phi.shape[0]
    h = box / n
    g = np.empty(phi.shape + (3,), dtype=np.float64)
    for d in range(3):
        g[..., d] = (np.roll(phi, -1, axis=d) - np.roll(phi, 1, axis=d)) / (2.0 * h)
    return g


def uniform_cells(phi: np.ndarray, grad: np.ndarray, box: float,
                  periodic: bool = True) -> Cells:
    """Cell list of a uniform grid (a tree with only the coarse level).
    Array index order is [i, j, k] = [x, y, z]."""
    n = phi.shape[0]
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.int32)
    return Cells(box=float(box), n0=n, max_level=0, periodic=periodic,
                 level=np.zeros(n ** 3, dtype=np.uint8), ijk=ijk,
                 phi=phi.reshape(-1).astype(np.float64).copy(),
                 grad=grad.reshape(-1, 3).astype(np.float64).copy())


# ---------------------------------------------------------------------------
# Smooth periodic analytic field (sum of Fourier modes), sampled at cell centres
# ---------------------------------------------------------------------------
class FourierField:
    """Phi(x) = sum_m a_m cos(2 pi n_m . x / L + p_m): periodic, smooth, with an
    exact gradient, so every AMR level can carry its own sample."""

    def __init__(self, box: float, seed: int, n_modes: int = 24, kmax: int = 6,
                 rms: float = 1e-5):
        rng = _rng(seed)
        self.box = float(box)
        self.nvec = rng.integers(-kmax, kmax + 1, size=(n_modes, 3))
        self.nvec[np.all(self.nvec == 0, axis=1)] = (1, 0, 0)
        kn = np.linalg.norm(self.nvec, axis=1)
        self.amp = rng.standard_normal(n_modes) * kn ** -1.5
        self.phase = rng.uniform(0, 2 * np.pi, size=n_modes)
        # normalise so the field rms over the box is `rms` (modes may repeat,
        # so estimate the rms on a sample grid)
        g = (np.arange(16) + 0.5) * self.box / 16
        pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        p, _ = self(pts, _raw=True)
        self.amp *= rms / np.sqrt(np.mean(p ** 2))

    def __call__(self, x: np.ndarray, _raw: bool = False):
        kvec = 2 * np.pi * self.nvec / self.box                # [m,3]
        arg = x @ kvec.T + self.phase                           # [n,m]
        phi = np.cos(arg) @ self.amp
        grad = -(np.sin(arg) * self.amp) @ kvec
        return phi, grad


def fourier_field(box: float, seed: int, **kw) -> FourierField:
    return FourierField(box, seed, **kw)


def _cell_centres(level: np.ndarray, ijk: np.ndarray, box: float, n0: int) -> np.ndarray:
    h = box / (n0 * (2.0 ** level.astype(np.float64)))
    return (ijk.astype(np.float64) + 0.5) * h[:, None]


def _children(ijk: np.ndarray) -> np.ndarray:
    """All 8 children (at the next level) of the given cells, octant-major."""
    out = []
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                out.append(2 * ijk + np.array([ox, oy, oz], dtype=ijk.dtype))
    return np.concatenate(out, axis=0)


def random_amr_cells(n0: int, box: float, max_level: int, seed: int,
                     p_refine=(0.25, 0.35, 0.45), blobs: int = 4,
                     periodic: bool = True, field_seed: int | None = None) -> Cells:
    """Small random full tree (0 or 8 children per cell) for brute-force
    octree checks and parity tests.  Refinement is drawn near a few random
    blob centres (so refined regions are contiguous and level transitions are
    common), with probability p_refine[l] inside a blob at level l."""
    rng = _rng(seed)
    field = FourierField(box, seed if field_seed is None else field_seed)
    centres = rng.uniform(0, box, size=(blobs, 3))
    radius = rng.uniform(0.12, 0.3, size=blobs) * box
    ii, jj, kk = np.meshgrid(np.arange(n0), np.arange(n0), np.arange(n0), indexing="ij")
    lev_ijk = [np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int32)]
    for lev in range(max_level):
        cur = lev_ijk[-1]
        xc = _cell_centres(np.full(len(cur), lev, np.uint8), cur, box, n0)
        d = xc[:, None, :] - centres[None, :, :]
        if periodic:
            d -= box * np.round(d / box)
        inside = np.any(np.linalg.norm(d, axis=2) < radius[None, :], axis=1)
        p = p_refine[min(lev, len(p_refine) - 1)]
        refine = inside & (rng.uniform(size=len(cur)) < p)
        if not refine.any():
            break
        lev_ijk.append(_children(cur[refine]))
    level = np.concatenate([np.full(len(a), l, np.uint8) for l, a in enumerate(lev_ijk)])
    ijk = np.concatenate(lev_ijk, axis=0)
    x = _cell_centres(level, ijk, box, n0)
    phi, grad = field(x)
    return Cells(box=float(box), n0=n0, max_level=len(lev_ijk) - 1, periodic=periodic,
                 level=level, ijk=ijk, phi=phi, grad=grad)


# ---------------------------------------------------------------------------
# AMR grid with haloes: Gaussian background + truncated NFW-like haloes,
# refined where a lognormal-plus-halo density exceeds 8x the mean
# ---------------------------------------------------------------------------
def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _in_chunks(fn, n: int, chunk: int = 1 << 22) -> None:
    """fn(a, b) over consecutive ranges of [0, n) on a thread pool (numpy
    releases the GIL in its array operations; every range writes only its own
    slice of the outputs, so the result does not depend on the pool)."""
    spans = [(a, min(n, a + chunk)) for a in range(0, n, chunk)]
    if len(spans) <= 1:
        for a, b in spans:
            fn(a, b)
        return
    with ThreadPoolExecutor(_workers()) as ex:
        for _ in ex.map(lambda ab: fn(*ab), spans):
            pass


def _cic_sample_periodic(grid: np.ndarray, x: np.ndarray, box: float, chunk: int = 1 << 21) -> np.ndarray:
    """Trilinear (cloud-in-cell) sample of a periodic cell-centred grid.
    Used only to give refined cells a background value (input synthesis).
    Points are taken in chunks; corner weights are the products
    (w_x w_y) w_z and corners are summed in octant order."""
    n = grid.shape[0]
    flat = grid.reshape((n ** 3,) + grid.shape[3:])
    out = np.zeros(x.shape[:1] + grid.shape[3:], dtype=np.float64)

    def run(s0, s1):
        u = x[s0:s1] / (box / n) - 0.5
        b = np.floor(u).astype(np.int64)
        t = u - b
        lo = [(b[:, d] % n, 1.0 - t[:, d]) for d in range(3)]
        hi = [((b[:, d] + 1) % n, t[:, d]) for d in range(3)]
        acc = out[s0:s1]
        for o in range(8):
            (i, wi), (j, wj), (k, wk) = [(hi if (o >> d) & 1 else lo)[d] for d in range(3)]
            w = wi * wj * wk
            v = flat[(i * n + j) * n + k]
            acc += (w[:, None] * v) if v.ndim > 1 else w * v
    _in_chunks(run, len(x), chunk)
    return out


class HaloSet:
    """Truncated NFW-like haloes: Phi_h(r) = -P0 [f(r/rs) - f(R/rs)] for r < R,
    0 beyond, f(y) = ln(1+y)/y, so Phi is continuous; density
    rho/rhobar = D0 / (y (1+y)^2) inside R."""

    def __init__(self, box, seed, n_halo, phi_range=(1e-6, 3e-5), rs_range=(0.2, 1.5),
                 trunc=25.0, dens_norm=1.0, centres=None):
        rng = _rng(seed)
        self.box = float(box)
        self.pos = (rng.uniform(0, box, size=(n_halo, 3)) if centres is None
                    else np.asarray(centres, np.float64))
        lo, hi = np.log(phi_range[0]), np.log(phi_range[1])
        self.p0 = np.exp(rng.uniform(lo, hi, size=len(self.pos)))
        lo, hi = np.log(rs_range[0]), np.log(rs_range[1])
        self.rs = np.exp(rng.uniform(lo, hi, size=len(self.pos)))
        self.R = trunc * self.rs
        # density amplitude scales with the potential depth over rs^2
        # (Poisson: Phi ~ rho rs^2); dens_norm tunes the refined volume
        self.d0 = dens_norm * self.p0 / self.rs ** 2 * 1e5

    def _iter_near(self, x, R):
        """Yield (halo index, indices of x within radius R[h] of halo h,
        minimum-image separations, distances).  Points are bucketed on a
        periodic grid of cells a quarter of the largest radius wide; each
        halo inspects the buckets within its own radius (plus one)."""
        box = self.box
        nb = max(1, int(box // max(0.25 * R.max(), 1e-9)))
        bsz = box / nb
        bidx = np.floor(np.mod(x, box) / bsz).astype(np.int64) % nb
        key = (bidx[:, 0] * nb + bidx[:, 1]) * nb + bidx[:, 2]
        del bidx
        order = np.argsort(key, kind="stable")
        starts = np.searchsorted(key[order], np.arange(nb ** 3 + 1))
        del key
        for h in range(len(self.pos)):
            hb = np.floor(np.mod(self.pos[h], box) / bsz).astype(np.int64) % nb
            m = int(np.ceil(R[h] / bsz)) + 1
            r = np.arange(-m, m + 1) if 2 * m + 1 < nb else np.arange(nb)
            bi, bj, bk = [np.unique((hb[d] + r) % nb) for d in range(3)]
            nbk = ((bi[:, None, None] * nb + bj[None, :, None]) * nb + bk[None, None, :]).ravel()
            s0, ln = starts[nbk], starts[nbk + 1] - starts[nbk]
            tot = int(ln.sum())
            if tot == 0:
                continue
            # the bucket ranges back to back, in bucket order
            cand = order[np.repeat(s0 - (np.cumsum(ln) - ln), ln) + np.arange(tot)]
            d = x[cand] - self.pos[h]
            d -= box * np.round(d / box)
            r2 = np.einsum("ij,ij->i", d, d)
            m = r2 < R[h] ** 2
            if m.any():
                yield h, cand[m], d[m], np.sqrt(r2[m])

    def potential(self, x):
        phi = np.zeros(len(x))
        grad = np.zeros((len(x), 3))

        def run(a, b):
            ph, gr = phi[a:b], grad[a:b]
            for h, sel, d, r in self._iter_near(x[a:b], self.R):
                rs, R, p0 = self.rs[h], self.R[h], self.p0[h]
                y = np.maximum(r / rs, 1e-12)
                f = np.log1p(y) / y
                fR = np.log1p(R / rs) / (R / rs)
                ph[sel] += -p0 * (f - fR)
                # d f/dy = 1/(y(1+y)) - ln(1+y)/y^2 ; dPhi/dr = -p0 f'(y)/rs
                fp = 1.0 / (y * (1.0 + y)) - np.log1p(y) / y ** 2
                dphidr = -p0 * fp / rs
                gr[sel] += (dphidr / np.maximum(r, 1e-12))[:, None] * d
        _in_chunks(run, len(x))
        return phi, grad

    def density(self, x, half=0.0):
        """Halo density at the point of the cube of half-width `half` around
        each x that is closest to the halo centre (so a cell is refined when
        any part of it is dense enough)."""
        rho = np.zeros(len(x))
        Rext = self.R + np.sqrt(3.0) * half

        def run(a, b):
            out = rho[a:b]
            for h, sel, d, r in self._iter_near(x[a:b], Rext):
                dd = np.maximum(np.abs(d) - half, 0.0)
                rr = np.sqrt(np.einsum("ij,ij->i", dd, dd))
                inside = rr < self.R[h]
                y = np.maximum(rr / self.rs[h], 1e-3)
                out[sel] += np.where(inside, self.d0[h] / (y * (1.0 + y) ** 2), 0.0)
        _in_chunks(run, len(x))
        return rho


def amr_halo_cells(n0: int, box: float, max_level: int, seed: int, n_halo: int = 200,
                   threshold: float = 8.0, dens_norm: float = 1.0, rms: float = 1e-5,
                   halo_centres=None, max_cells: int | None = None, log=None) -> Cells:
    """AMR tree: Gaussian potential on the coarse grid (P(k) ~ k^-3, rms `rms`),
    plus `n_halo` truncated NFW-like haloes.  Density 1 + delta =
    exp(g - 1/2) (g: the unit Gaussian paired with Phi) + halo densities; a
    cell is refined when the density at its centre exceeds `threshold`,
    at every level up to max_level.  Refined cells take the background
    potential by trilinear sampling of the coarse grid plus the exact halo
    potential at their own centre.  log: optional callable taking a progress
    message (very large trees take minutes)."""
    say = log if log is not None else (lambda msg: None)
    rng_seed = seed
    phi0 = gaussian_potential(n0, box, rng_seed, rms=rms)
    grad0 = central_gradient(phi0, box)
    g = phi0 / np.std(phi0)          # unit Gaussian for the lognormal density
    halos = HaloSet(box, seed + 7919, n_halo, dens_norm=dens_norm, centres=halo_centres)

    ii, jj, kk = np.meshgrid(np.arange(n0), np.arange(n0), np.arange(n0), indexing="ij")
    lev_ijk = [np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int32)]
    for lev in range(max_level):
        cur = lev_ijk[-1]
        x = _cell_centres(np.full(len(cur), lev, np.uint8), cur, box, n0)
        if lev == 0:
            gb = g.reshape(-1)
        else:
            gb = _cic_sample_periodic(g, x, box)
        half = 0.5 * box / (n0 * 2 ** lev)
        rho = np.exp(-gb - 0.5) + halos.density(x, half)   # wells (Phi < 0) are overdense
        refine = rho > threshold
        if not refine.any():
            break
        kids = _children(cur[refine])
        say(f"level {lev}: {len(cur)} cells, {int(refine.sum())} refined")
        if max_cells is not None and sum(len(a) for a in lev_ijk) + len(kids) > max_cells:
            break
        lev_ijk.append(kids)

    level = np.concatenate([np.full(len(a), l, np.uint8) for l, a in enumerate(lev_ijk)])
    ijk = np.concatenate(lev_ijk, axis=0)
    phi = np.empty(len(level))
    grad = np.empty((len(level), 3))
    n_coarse = n0 ** 3
    phi[:n_coarse] = phi0.reshape(-1)
    grad[:n_coarse] = grad0.reshape(-1, 3)
    if len(level) > n_coarse:
        xr = _cell_centres(level[n_coarse:], ijk[n_coarse:], box, n0)
        phi[n_coarse:] = _cic_sample_periodic(phi0, xr, box)
        say("background potential sampled on the refined cells")
        grad[n_coarse:] = _cic_sample_periodic(grad0, xr, box)
        say("background gradient sampled on the refined cells")
        del xr
    xall = _cell_centres(level, ijk, box, n0)
    hp, hg = halos.potential(xall)
    say("halo potentials added")
    phi += hp
    grad += hg
    return Cells(box=float(box), n0=n0, max_level=len(lev_ijk) - 1, periodic=True,
                 level=level, ijk=ijk, phi=phi, grad=grad)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    """One ray-tracing workload: a grid recipe plus observers and sky pixels."""
    name: str
    grid: str                  # "gauss64" | "amr128" | ...
    nside: int
    obs: np.ndarray            # [n_obs, 3]
    z_src: np.ndarray          # [n_obs]
    pix_first: np.ndarray      # [n_obs] int64 (NESTED)
    pix_count: np.ndarray      # [n_obs] int64
    steps_per_cell: int
    adaptive: bool

    @property
    def n_rays(self) -> int:
        return int(self.pix_count.sum())


# Two light-cone layers of the uniform 64^3 potential, slightly shifted in
# time: the second is the first decayed as in linear LCDM near z = 0.5
# (d ln Phi / d ln a = -0.3) plus an independent Gaussian field of the same
# spectrum at a fifth of that change (a non-linear, uncorrelated part).
ISW_LAYER_A = (0.66, 0.68)


def second_layer(phi1: np.ndarray, n: int, box: float, seed: int, a1: float, a2: float,
                 slope: float = -0.3, noise: float = 0.2) -> np.ndarray:
    """Potential of the second layer at a2 of a uniform n^3 grid whose first
    layer (at a1, cell order of uniform_cells) is phi1."""
    d = slope * (a2 - a1) / a1
    g2 = gaussian_potential(n, box, seed=seed).ravel()
    return phi1 * (1.0 + d) + noise * d * g2


def make_cells(grid: str, log=None) -> Cells:
    """Build a named grid (deterministic); log as in amr_halo_cells."""
    if grid == "gauss64":
        # uniform 64^3 grid, box 500 Mpc/h, P(k) ~ k^-3, rms 1e-5, seed 1
        phi = gaussian_potential(64, 500.0, seed=1)
        return uniform_cells(phi, central_gradient(phi, 500.0), 500.0)
    if grid == "gauss64_layer2":
        # the second layer of gauss64 at ISW_LAYER_A[1] (phi only; seed 21)
        c = make_cells("gauss64")
        c.phi = second_layer(c.phi, 64, 500.0, 21, *ISW_LAYER_A)
        return c
    if grid == "gauss32":
        phi = gaussian_potential(32, 250.0, seed=11)
        return uniform_cells(phi, central_gradient(phi, 250.0), 250.0)
    if grid == "amr_small":
        # 16^3 coarse, box 125 Mpc/h, up to 3 levels around random blobs
        return random_amr_cells(16, 125.0, 3, seed=5)
    if grid == "amr_halo_small":
        return amr_halo_cells(32, 250.0, 3, seed=12, n_halo=40, dens_norm=1.0)
    if grid == "amr_deep":
        # 64^3 coarse, box 500 Mpc/h, 5 levels (finest 0.24 Mpc/h) in 60
        # haloes: the depth of the 512^3 + 5 levels configuration on a grid
        # small enough for full oracle comparisons (about 1.2e6 cells)
        return amr_halo_cells(64, 500.0, 5, seed=5, n_halo=60, dens_norm=3000.0, threshold=30.0)
    if grid == "amr128":
        # 128^3 coarse, box 500 Mpc/h, 3 levels, 200 haloes, ~1e7 cells
        return amr_halo_cells(128, 500.0, 3, seed=2, n_halo=200, dens_norm=AMR128_DENS_NORM)
    if grid == "amr512":
        # 512^3 coarse, box 2000 Mpc/h (coarse cells 3.9 Mpc/h), 5 levels
        # (finest 0.12 Mpc/h): 950 haloes uniform in a sphere of 400 Mpc/h
        # around the observer plus 950 uniform in the box; refinement as in
        # amr_deep (threshold 30, density normalisation 3000): about 4e8 cells
        cen = sphere_and_uniform_centres(2000.0, LARGE_OBS, 400.0, 950, 950, seed=108)
        return amr_halo_cells(512, 2000.0, 5, seed=7, n_halo=len(cen), threshold=30.0, dens_norm=3000.0,
                              halo_centres=cen, log=log)
    raise KeyError(grid)


# observer of the 512^3 + 5 level light cone (the box centre)
LARGE_OBS = (1000.0, 1000.0, 1000.0)


def sphere_and_uniform_centres(box: float, centre, radius: float, n_in: int, n_out: int, seed: int) -> np.ndarray:
    """n_in points uniform in the ball of `radius` around `centre` (periodic)
    followed by n_out points uniform in the box."""
    rng = _rng(seed)
    u = rng.standard_normal((n_in, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, n_in) ** (1.0 / 3.0)
    inner = np.asarray(centre, np.float64) + u * r[:, None]
    return np.concatenate([inner, rng.uniform(0.0, box, (n_out, 3))]) % box


# density normalisation of the 128^3 AMR grid's haloes, chosen so the tree holds
# about 1e7 cells (the count is recorded by the tests)
AMR128_DENS_NORM = 10000.0


def _full_sky(nside):
    return np.array([0], np.int64), np.array([12 * nside * nside], np.int64)


def batched_cones(box: float, n_obs: int, nside: int, seed: int,
                  zlo: float = 0.1, zhi: float = 2.0):
    """n_obs observers at uniform positions, source redshift U[zlo, zhi], each
    cone one NESTED base-resolution patch (nside^2 pixels of a random base
    pixel)."""
    rng = _rng(seed)
    obs = rng.uniform(0, box, size=(n_obs, 3))
    z = rng.uniform(zlo, zhi, size=n_obs)
    base = rng.integers(0, 12, size=n_obs)
    first = (base * nside * nside).astype(np.int64)
    count = np.full(n_obs, nside * nside, np.int64)
    return obs, z, first, count


def _wl(name):
    c = np.array([[250.0, 250.0, 250.0]])
    if name == "uniform":        # 64^3, 3072 rays to z = 0.5, 10 steps per cell
        f, n = _full_sky(16)
        return Workload(name, "gauss64", 16, c, np.array([0.5]), f, n, 10, False)
    if name == "amr":            # 128^3 + 3 levels, 786432 rays to z = 1, 4 steps per leaf cell
        f, n = _full_sky(256)
        return Workload(name, "amr128", 256, c, np.array([1.0]), f, n, 4, True)
    if name == "batched":        # 64 cones of 16384 rays on the 64^3 grid
        obs, z, first, count = batched_cones(500.0, 64, 128, seed=3)
        return Workload(name, "gauss64", 128, obs, z, first, count, 10, False)
    if name == "large":          # 512^3 + 5 levels, full sky at nside 2048 (50,331,648 rays) to z = 2
        f, n = _full_sky(2048)
        return Workload(name, "amr512", 2048, np.array([LARGE_OBS]), np.array([2.0]), f, n, 4, True)
    if name == "differentiated":  # 2^20 rays to z = 1 on the 64^3 grid
        return Workload(name, "gauss64", 512, c, np.array([1.0]),
                        np.array([0], np.int64), np.array([1 << 20], np.int64), 10, False)
    raise KeyError(name)


class _Workloads(dict):
    def __missing__(self, key):
        v = _wl(key)
        self[key] = v
        return v


WORKLOADS = _Workloads()
