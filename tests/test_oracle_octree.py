"""Pins of the oracle's octree lookups and CIC interpolation with AMR level
fallback (Sect. 2.2, the five-step procedure and Fig. 1) against brute force
over the cell list."""
import numpy as np
import pytest

import synth


def brute(cells, x):
    """Leaf level, stencil level and CIC values by linear scans of the cell
    list: the deepest cell containing x; then, from that level down, the
    first level where all 8 cells around x exist."""
    n0, box, per = cells.n0, cells.box, cells.periodic
    u = np.asarray(x, float) / (box / n0)
    present = {(int(l), *map(int, c)): i for i, (l, c) in enumerate(zip(cells.level, cells.ijk))}

    def find(l, I):
        m = n0 << l
        if per:
            I = [int(v) % m for v in I]
        elif any(v < 0 or v >= m for v in I):
            return None
        return present.get((l, *map(int, I)))

    # linear scan (vectorised): every cell containing x, keep the deepest
    m = (n0 << cells.level.astype(np.int64))[:, None]
    I = np.floor(u[None, :] * (2.0 ** cells.level.astype(float))[:, None]).astype(np.int64)
    if per:
        I %= m
    hit = np.all(I == cells.ijk, axis=1)
    leaf = int(cells.level[hit].max()) if hit.any() else -1
    if leaf < 0:
        return None
    for l in range(leaf, -1, -1):
        y = u * 2.0 ** l
        b = np.floor(y - 0.5).astype(np.int64)
        ids = []
        for o in range(8):
            off = np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1])
            ids.append(find(l, b + off))
        if any(v is None for v in ids):
            continue
        phi, grad = 0.0, np.zeros(3)
        for o, cid in enumerate(ids):
            off = np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1])
            r = y - (b + off + 0.5)                      # separation in cell units
            w = np.prod(1.0 - np.abs(r))                # W_CIC
            phi += w * cells.phi[cid]
            grad += w * cells.grad[cid]
        return leaf, l, phi, grad
    return (leaf, None, None, None)


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("seed", [5, 6])
def test_lookup_and_cic_match_brute_force(O, periodic, seed):
    cells = synth.random_amr_cells(8, 80.0, 3, seed=seed, p_refine=(0.3, 0.4, 0.5), periodic=periodic)
    assert cells.max_level == 3
    f = O.Field.grid(cells)
    rng = np.random.default_rng(seed)
    lo, hi = (-20.0, 100.0) if periodic else (0.0, 80.0)
    pts = rng.uniform(lo, hi, size=(400, 3))
    # also points exactly on cell faces and centres of the finest level
    hf = 80.0 / (8 * 8)
    pts[:50] = np.round(pts[:50] / hf) * hf
    pts[50:100] = (np.floor(pts[50:100] / hf) + 0.5) * hf
    n_fallback = 0
    for x in pts:
        st, phi, g, leaf, lvl = f.probe(x)
        ref = brute(cells, x)
        if ref is None:             # outside a non-periodic box
            assert st == 1 and leaf == -1
            continue
        assert leaf == ref[0]
        if ref[1] is None:
            assert st == 1          # no complete stencil even at the coarse level
            continue
        assert st == 0 and lvl == ref[1]
        n_fallback += lvl < leaf
        assert phi == pytest.approx(ref[2], rel=1e-12, abs=1e-22)
        assert np.allclose(g, ref[3], rtol=1e-12, atol=1e-24)
    assert n_fallback > 3           # the fallback branch is exercised


def test_cic_reproduces_linear_fields(O):
    """CIC weights sum to one and reproduce a linear field exactly (any level)."""
    cells = synth.random_amr_cells(8, 80.0, 2, seed=9, periodic=False)
    g = np.array([1e-6, -2e-6, 3e-7])
    x = (cells.ijk + 0.5) * (80.0 / (8 * 2.0 ** cells.level))[:, None]
    cells.phi = 1e-5 + x @ g
    cells.grad = np.tile(g, (cells.n_cells, 1))
    f = O.Field.grid(cells)
    rng = np.random.default_rng(0)
    for p in rng.uniform(5.5, 74.5, size=(300, 3)):
        st, phi, gg, leaf, lvl = f.probe(p)
        assert st == 0
        assert phi == pytest.approx(1e-5 + p @ g, rel=1e-13)
        assert np.allclose(gg, g, rtol=1e-13)


def test_non_periodic_edge_leaves_domain(O):
    cells = synth.random_amr_cells(8, 80.0, 1, seed=3, periodic=False)
    f = O.Field.grid(cells)
    # within half a coarse cell of the boundary no coarse stencil exists
    assert f.probe([2.0, 40.0, 40.0])[0] == 1
    assert f.probe([40.0, 40.0, 79.0])[0] == 1
    assert f.probe([40.0, 40.0, 40.0])[0] == 0


def test_rejects_non_full_tree(O):
    cells = synth.random_amr_cells(8, 80.0, 2, seed=4)
    fine = np.nonzero(cells.level == 1)[0]
    keep = np.ones(cells.n_cells, bool)
    keep[fine[3]] = False
    bad = synth.Cells(cells.box, cells.n0, cells.max_level, cells.periodic, cells.level[keep],
                      cells.ijk[keep], cells.phi[keep], cells.grad[keep])
    with pytest.raises(ValueError):
        O.Field.grid(bad)
    # a family of leaves missing any one of its 8 cells (the first one included)
    deep = np.nonzero(cells.level == 2)[0]
    par = cells.ijk[deep] >> 1
    fam = deep[np.all(par == par[0], axis=1)]
    assert len(fam) == 8
    for c in fam:
        keep = np.ones(cells.n_cells, bool)
        keep[c] = False
        bad = synth.Cells(cells.box, cells.n0, cells.max_level, cells.periodic, cells.level[keep],
                          cells.ijk[keep], cells.phi[keep], cells.grad[keep])
        with pytest.raises(ValueError, match="full tree"):
            O.Field.grid(bad)
    # and a missing coarse cell
    keep = np.ones(cells.n_cells, bool)
    keep[0] = False
    bad = synth.Cells(cells.box, cells.n0, cells.max_level, cells.periodic, cells.level[keep],
                      cells.ijk[keep], cells.phi[keep], cells.grad[keep])
    with pytest.raises(ValueError):
        O.Field.grid(bad)
