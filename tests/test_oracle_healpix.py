"""Pins of the oracle's HEALPix NESTED pixel centres (Sect. 2.4 initialises
photon directions at HEALPix pixel centres; Gorski et al. 2005).

The reference set of centres is built here independently from the RING-scheme
definition (rings of constant z, evenly spaced azimuths); the NESTED centres
must be exactly a permutation of it."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "healpix_base_pixels.txt")


def ring_centres(nside):
    """Pixel centres of the RING scheme (Gorski et al. 2005, Sect. 4)."""
    zs, phis = [], []
    ns = nside
    for i in range(1, 4 * ns):
        if i < ns:                     # north polar cap
            z = 1.0 - i * i / (3.0 * ns * ns)
            ph = (np.arange(1, 4 * i + 1) - 0.5) * np.pi / (2 * i)
        elif i <= 3 * ns:              # equatorial belt
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            s = (i - ns + 1) % 2
            ph = (np.arange(1, 4 * ns + 1) - 0.5 * s) * np.pi / (2 * ns)
        else:                          # south polar cap
            ii = 4 * ns - i
            z = -(1.0 - ii * ii / (3.0 * ns * ns))
            ph = (np.arange(1, 4 * ii + 1) - 0.5) * np.pi / (2 * ii)
        zs.append(np.full(len(ph), z))
        phis.append(ph)
    z = np.concatenate(zs)
    ph = np.concatenate(phis)
    st = np.sqrt((1 - z) * (1 + z))
    return np.stack([st * np.cos(ph), st * np.sin(ph), z], 1)


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16, 64])
def test_nested_is_permutation_of_ring(O, nside):
    v = O.pix2vec_nest(nside, np.arange(12 * nside * nside))
    r = ring_centres(nside)
    assert len(v) == len(r) == 12 * nside * nside
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    # nearest ring centre of every nested centre; must be a bijection
    from scipy.spatial import cKDTree
    d, idx = cKDTree(r).query(v)
    assert d.max() < 1e-12
    assert len(np.unique(idx)) == len(v)
    # the pixel centres are balanced over the sphere
    assert np.abs(v.sum(axis=0)).max() < 1e-9


def test_base_pixels_golden(O):
    rows = np.loadtxt(GOLDEN)
    v = O.pix2vec_nest(1, rows[:, 0].astype(int))
    assert np.allclose(v[:, 2], rows[:, 1], atol=1e-15)
    ph = np.arctan2(v[:, 1], v[:, 0]) % (2 * np.pi)
    assert np.allclose(ph, rows[:, 2] * np.pi, atol=1e-14)


@pytest.mark.parametrize("nside", [2, 8, 32])
def test_nested_hierarchy(O, nside):
    """Nested pixel p at nside has its four children 4p..4p+3 at 2 nside:
    their centres surround the parent centre (mean direction ~ parent)."""
    par = O.pix2vec_nest(nside, np.arange(12 * nside * nside))
    kids = O.pix2vec_nest(2 * nside, np.arange(48 * nside * nside)).reshape(-1, 4, 3)
    m = kids.mean(axis=1)
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    pix_size = np.sqrt(4 * np.pi / (12 * nside * nside))
    sep = np.arccos(np.clip(np.sum(m * par, 1), -1, 1))
    assert sep.max() < 0.3 * pix_size
    # children of one parent are nearer to their own parent than one pixel size
    d = np.arccos(np.clip(np.einsum("pkc,pc->pk", kids, par), -1, 1))
    assert d.max() < pix_size


def test_face_axes_point_north_east(O):
    """Within a base face the nested x index (even bits) runs towards the
    north-east and y (odd bits) towards the north-west (Gorski et al. 2005)."""
    v = O.pix2vec_nest(2, [0, 1, 2])   # face 0: (x,y) = (0,0), (1,0), (0,1)
    ph = np.arctan2(v[:, 1], v[:, 0])
    assert v[1, 2] > v[0, 2] and ph[1] > ph[0]      # x: north and east
    assert v[2, 2] > v[0, 2] and ph[2] < ph[0]      # y: north and west
