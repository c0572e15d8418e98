"""Pins of the oracle's second form of the geodesic equations (Sect. 2.2):
the equations written with dPhi/dlambda only (dPhi/deta eliminated through
the chain rule) and dPhi/dlambda estimated per step from Phi at the last two
step starts (Eq. dPhi/dl, second form)."""
import numpy as np

import synth

COSMO = (0.3, 0.7, 0.7)


def _rel(a, b, L):
    return np.abs(a["r"] - b["r"]).max() / L


def test_linear_potential_first_order_convergence(O):
    """Phi = g . x: the difference quotient is g . (mean k over the previous
    step), so the two forms differ only by the change of k over one step
    (the Hubble term, the bending): the gap halves with the step."""
    f = O.Field.linear([2e-6, -1e-6, 3e-6], phi0=1e-5)
    dirs = O.pix2vec_nest(1, np.arange(12))
    for cz, kw, L in ((O.cosmo(0.0, 0.0, 0.7), {"chi": 800.0}, 800.0), (O.cosmo(*COSMO), {"z_src": 0.5}, 1300.0)):
        gaps = []
        for ds in (4.0, 2.0, 1.0):
            a = O.cast(f, cz, O.params([0.0, 0.0, 0.0], ds=ds, dphidl=O.DPHIDL_CHAIN, **kw), dirs)
            b = O.cast(f, cz, O.params([0.0, 0.0, 0.0], ds=ds, dphidl=O.DPHIDL_DIFF, **kw), dirs)
            assert (a["status"] == O.REACHED).all() and (b["status"] == O.REACHED).all()
            gaps.append(_rel(a, b, L))
        assert gaps[0] > 1e-9
        for g0, g1 in zip(gaps, gaps[1:]):
            assert 1.95 < g0 / g1 < 2.05, gaps


def test_constant_potential_identical(O):
    """Phi constant: every difference and gradient vanishes, both forms are
    the FLRW equations."""
    cells = synth.uniform_cells(np.full((8, 8, 8), 3e-5), np.zeros((8, 8, 8, 3)), 64.0)
    f = O.Field.grid(cells)
    c = O.cosmo(*COSMO)
    dirs = O.pix2vec_nest(1, np.arange(12))
    a = O.cast(f, c, O.params([1.0, 2.0, 3.0], z_src=0.4, steps_per_cell=4, dphidl=O.DPHIDL_CHAIN), dirs)
    b = O.cast(f, c, O.params([1.0, 2.0, 3.0], z_src=0.4, steps_per_cell=4, dphidl=O.DPHIDL_DIFF), dirs)
    for k in ("r", "k", "eta", "z5", "n_steps", "hash"):
        assert np.array_equal(a[k], b[k]), k


def test_light_cone_potential_carries_the_time_derivative(O):
    """The reason for the second form: on a light cone the potential a photon
    meets changes with time through its position.  A cone whose cells hold
    Phi = phi0 - T r (r from the observer, zero spatial gradient) cast with
    the difference estimate reproduces the dPhi/deta = T grid cast with the
    chain rule: the estimate sees Phi change at -T |k| instead of -T |k0|,
    and |k|/|k0| grows from 1 to ~1.05 over the path, so the dPhi/deta effect
    on chi (2.7 %) is reproduced to ~2.7 % of itself (7e-4); the static
    potential misses it."""
    n, box = 64, 4000.0
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int32)
    centres = (ijk + 0.5) * (box / n)
    obs = np.array([2000.3, 1999.6, 2000.9])
    T, phi0 = 2e-5, 1e-5
    r = np.linalg.norm(centres - obs, axis=1)

    def cells(phi, tdot=None):
        return synth.Cells(box=box, n0=n, max_level=0, periodic=False, level=np.zeros(len(ijk), np.uint8), ijk=ijk,
                           phi=phi, grad=np.zeros((len(ijk), 3)), dphi_deta=tdot)

    c = O.cosmo(*COSMO)
    dirs = O.pix2vec_nest(2, np.arange(48))
    p = lambda mode: O.params(obs, z_src=0.5, steps_per_cell=8, dphidl=mode)
    cone = O.cast(O.Field.grid(cells(phi0 - T * r)), c, p(O.DPHIDL_DIFF), dirs)
    tdot = O.cast(O.Field.grid(cells(np.full(len(r), phi0), np.full(len(r), T))), c, p(O.DPHIDL_CHAIN), dirs)
    stat = O.cast(O.Field.grid(cells(np.full(len(r), phi0))), c, p(O.DPHIDL_CHAIN), dirs)
    assert (cone["status"] == O.REACHED).all() and (tdot["status"] == O.REACHED).all()
    assert np.abs(cone["chi"] / tdot["chi"] - 1).max() < 2e-3
    assert np.abs(stat["chi"] / tdot["chi"] - 1).min() > 2e-2
    assert np.abs(cone["alpha"]).max() < 1e-12
