"""Pins of the oracle's NGP and TSC interpolation (Sect. 2.2, weights W_NGP,
W_TSC and the level-fallback procedure) by values the weight formulas fix:
the response to a single unit cell, exact reproduction of linear fields, and
which level the fallback takes on small refined trees."""
import numpy as np
import pytest

import synth

N0, BOX = 8, 8.0           # h0 = 1


def _tree(coarse_fn, refined=(), fine_fn=None, periodic=True):
    """Coarse 8^3 grid plus the 8 children of each coarse cell in `refined`;
    values (phi, grad) from coarse_fn / fine_fn of the cell centres."""
    ii, jj, kk = np.meshgrid(np.arange(N0), np.arange(N0), np.arange(N0), indexing="ij")
    ijk0 = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)
    lv, ijk, centres = [np.zeros(len(ijk0), int)], [ijk0], [ijk0 + 0.5]
    for c in refined:
        kids = np.array([[2 * c[0] + (o & 1), 2 * c[1] + ((o >> 1) & 1), 2 * c[2] + (o >> 2)] for o in range(8)])
        lv.append(np.ones(8, int))
        ijk.append(kids)
        centres.append((kids + 0.5) / 2.0)
    lv, ijk, centres = np.concatenate(lv), np.concatenate(ijk), np.concatenate(centres)
    phi = np.empty(len(lv))
    grad = np.empty((len(lv), 3))
    for i in range(len(lv)):
        fn = coarse_fn if lv[i] == 0 else fine_fn
        phi[i], grad[i] = fn(centres[i])
    return synth.Cells(box=BOX, n0=N0, max_level=1 if len(refined) else 0, periodic=periodic,
                       level=lv.astype(np.uint8), ijk=ijk.astype(np.int32), phi=phi, grad=grad)


def _unit_cell(c0):
    c0 = np.asarray(c0)

    def fn(x):
        hit = np.all(np.floor(x) == c0)
        return (1.0, np.array([1.0, 2.0, 3.0])) if hit else (0.0, np.zeros(3))
    return fn


@pytest.mark.parametrize("order,cases", [
    # TSC: 3/4 at a cell's own centre, 1/8 one cell away, 1/2 on the shared
    # face (both branches of W_TSC give 1/2 at |r| = 1/2)
    (2, [((3.5, 4.5, 2.5), 0.75 ** 3), ((4.5, 4.5, 2.5), 0.125 * 0.75 ** 2),
         ((4.5, 5.5, 3.5), 0.125 ** 3), ((4.0, 4.5, 2.5), 0.5 * 0.75 ** 2), ((5.5, 4.5, 2.5), 0.0)]),
    # CIC: 1 at its centre, 0 at the next centre, 1/2 on the face
    (1, [((3.5, 4.5, 2.5), 1.0), ((4.5, 4.5, 2.5), 0.0), ((4.0, 4.5, 2.5), 0.5), ((3.75, 4.5, 2.5), 0.75)]),
    # NGP: the cell's value anywhere inside it, nothing outside
    (0, [((3.01, 4.99, 2.5), 1.0), ((3.99, 4.01, 2.01), 1.0), ((4.01, 4.5, 2.5), 0.0)]),
])
def test_unit_cell_response(O, order, cases):
    cells = _tree(_unit_cell((3, 4, 2)))
    f = O.Field.grid(cells, order=order)
    for x, w in cases:
        st, phi, grad, leaf, lvl = f.probe(np.array(x))
        assert st == 0 and leaf == 0 and lvl == 0
        assert phi == pytest.approx(w, abs=1e-15), (order, x)
        assert np.allclose(grad, w * np.array([1.0, 2.0, 3.0]), atol=1e-15)


def _linear(a, g):
    g = np.asarray(g, float)
    return lambda x: (a + g @ x, g.copy())


@pytest.mark.parametrize("order", [1, 2])
def test_linear_fields_reproduced(O, order):
    """CIC and TSC weights have unit sum and zero first moment, so a field
    linear in the cell centres is interpolated exactly (non-periodic grid,
    points whose stencils stay inside)."""
    fn = _linear(0.3, [0.01, -0.02, 0.05])
    cells = _tree(fn, periodic=False)
    f = O.Field.grid(cells, order=order)
    rng = np.random.default_rng(1)
    for x in rng.uniform(2.0, 6.0, (40, 3)):
        st, phi, grad, leaf, lvl = f.probe(x)
        assert st == 0
        want, g = fn(x)
        assert phi == pytest.approx(want, abs=1e-14)
        assert np.allclose(grad, g, atol=1e-15)


def test_ngp_piecewise_constant(O):
    fn = _linear(0.3, [0.01, -0.02, 0.05])
    f = O.Field.grid(_tree(fn, periodic=False), order=0)
    rng = np.random.default_rng(2)
    for x in rng.uniform(0.0, 8.0, (40, 3)):
        st, phi, grad, leaf, lvl = f.probe(x)
        assert st == 0
        assert phi == pytest.approx(fn(np.floor(x) + 0.5)[0], abs=1e-15)


def test_tsc_level_fallback(O):
    """One refined coarse cell: its children have no complete 27-cell
    neighbourhood at level 1, so TSC falls back to level 0 (the coarse
    linear field comes out).  A refined 3x3x3 block: inside its central cell
    the level-1 neighbourhood is complete (the fine linear field comes out).
    NGP takes the child's own value in both."""
    coarse = _linear(0.1, [0.01, 0.0, 0.0])
    fine = _linear(-0.2, [0.0, 0.03, 0.0])
    one = O.Field.grid(_tree(coarse, refined=[(4, 4, 4)], fine_fn=fine), order=2)
    x = np.array([4.3, 4.6, 4.2])
    st, phi, grad, leaf, lvl = one.probe(x)
    assert (st, leaf, lvl) == (0, 1, 0)
    assert phi == pytest.approx(coarse(x)[0], abs=1e-14)
    block = [(i, j, k) for i in (3, 4, 5) for j in (3, 4, 5) for k in (3, 4, 5)]
    blk = O.Field.grid(_tree(coarse, refined=block, fine_fn=fine), order=2)
    st, phi, grad, leaf, lvl = blk.probe(x)
    assert (st, leaf, lvl) == (0, 1, 1)
    assert phi == pytest.approx(fine(x)[0], abs=1e-14)
    # near the block's edge the level-1 neighbourhood runs out again
    st, phi, grad, leaf, lvl = blk.probe(np.array([3.2, 4.5, 4.5]))
    assert (st, leaf, lvl) == (0, 1, 0)
    ngp = O.Field.grid(_tree(coarse, refined=[(4, 4, 4)], fine_fn=fine), order=0)
    st, phi, grad, leaf, lvl = ngp.probe(x)
    assert (leaf, lvl) == (1, 1)
    assert phi == pytest.approx(fine(np.floor(2 * x) / 2 + 0.25)[0], abs=1e-15)


def test_tsc_stops_at_the_edge_of_a_non_periodic_box(O):
    f = O.Field.grid(_tree(_linear(0.0, [0.0, 0.0, 0.0]), periodic=False), order=2)
    assert f.probe(np.array([0.5, 4.0, 4.0]))[0] == 1       # the -x neighbour is missing
    assert f.probe(np.array([1.5, 4.0, 4.0]))[0] == 0
