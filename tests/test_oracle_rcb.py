"""Pins of the oracle's locality relabelling (Section 3.3: recursive
bisection of 2D coordinates, alternately by x and y) and renumbering,
against hand-worked cases and the properties of the definitions."""
import numpy as np
import pytest

import oracle as O
from oracle.rcb import rcb_order, relabel
from workloads import grid2d, random_graph, rgg, rgg_points


def test_rcb_hand_worked():
    # depth 0 by x: p1 (0.1), p3 (0.3) | p2 (0.5), p0 (0.9);
    # depth 1 by y: p3 (0.2), p1 (0.8) and p0 (0.1), p2 (0.5)
    pts = np.array([[0.9, 0.1], [0.1, 0.8], [0.5, 0.5], [0.3, 0.2]])
    assert rcb_order(pts, leaf=1).tolist() == [3, 1, 0, 2]
    # a leaf of two keeps each half as sorted at depth 0
    assert rcb_order(pts, leaf=2).tolist() == [1, 3, 2, 0]
    # one box: the input order
    assert rcb_order(pts, leaf=4).tolist() == [0, 1, 2, 3]


def test_rcb_ties_keep_input_order_and_zero_signs():
    pts = np.zeros((100, 2))
    assert rcb_order(pts, leaf=1).tolist() == list(range(100))
    pts[::2, 0] = -0.0
    assert rcb_order(pts, leaf=3).tolist() == list(range(100))


def _check_bisection(pts, order, a, b, depth, leaf):
    """Every box of more than `leaf` points splits at len // 2 with all
    coordinates of the first half <= those of the second on its axis."""
    if b - a <= leaf:
        return
    mid = a + (b - a) // 2
    axis = depth % 2
    lo, hi = pts[order[a:mid], axis], pts[order[mid:b], axis]
    assert lo.max() <= hi.min(), (a, b, depth)
    _check_bisection(pts, order, a, mid, depth + 1, leaf)
    _check_bisection(pts, order, mid, b, depth + 1, leaf)


@pytest.mark.parametrize("n,leaf", [(1, 32), (37, 4), (1000, 1), (5000, 32), (4099, 100)])
def test_rcb_is_a_permutation_with_the_bisection_property(n, leaf):
    pts = rgg_points(n, 9)
    o = rcb_order(pts, leaf)
    assert sorted(o.tolist()) == list(range(n))
    _check_bisection(pts, o, 0, n, 0, leaf)


def test_rcb_lattice_equals_sorted_boxes():
    # a 4 x 4 lattice with leaf 1, worked by hand: x halves {0,1} | {2,3},
    # then y halves, then x, then y
    xs, ys = np.meshgrid(np.arange(4.0), np.arange(4.0), indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1)   # point i = (i // 4, i % 4)
    o = rcb_order(pts, leaf=1)
    got = [tuple(pts[i].astype(int)) for i in o]
    assert got == [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (0, 3), (1, 2), (1, 3),
                   (2, 0), (2, 1), (3, 0), (3, 1), (2, 2), (2, 3), (3, 2), (3, 3)]


def test_relabel_hand_worked():
    # path 0 -5- 1 -7- 2, new node x = old order[x] with order = [2, 0, 1]
    from workloads import csr_from_edges
    g = csr_from_edges(3, np.array([0, 1]), np.array([1, 2]), np.array([5, 7], dtype=np.uint32),
                       np.array([10, 20, 30], dtype=np.uint32))
    h = relabel(g, [2, 0, 1])
    assert h.xadj.tolist() == [0, 1, 2, 4]
    assert h.adj.tolist() == [2, 2, 0, 1]
    assert h.ew.tolist() == [7, 5, 7, 5]
    assert h.vw.tolist() == [30, 10, 20]


@pytest.mark.parametrize("make", [lambda: grid2d(9, 7), lambda: random_graph(300, 900, 3, 9, 5),
                                  lambda: rgg(2000, 5)])
def test_relabel_identity_inverse_and_invariants(make):
    g = O.Graph.of(make())
    same = relabel(g, np.arange(g.n))
    for f in ("xadj", "adj", "ew", "vw"):
        assert np.array_equal(getattr(same, f), getattr(g, f)), f
    perm = np.random.default_rng(4).permutation(g.n)
    h = relabel(g, perm)
    assert O.validate(h) == 0
    assert sorted(np.diff(h.xadj).tolist()) == sorted(np.diff(g.xadj).tolist())
    assert int(h.ew.astype(np.int64).sum()) == int(g.ew.astype(np.int64).sum())
    back = relabel(h, np.argsort(perm))
    for f in ("xadj", "adj", "ew", "vw"):
        assert np.array_equal(getattr(back, f), getattr(g, f)), f


def test_rcb_relabelled_rgg_has_locality():
    """The renamed random geometric graph keeps its edges (node i renamed
    inv[i]) and its neighbours' ids lie far closer together."""
    n = 1 << 14
    g = O.Graph.of(rgg(n, seed=9))
    o = rcb_order(rgg_points(n, 9))
    h = relabel(g, o)
    inv = np.empty(n, dtype=np.int64)
    inv[o] = np.arange(n)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.xadj))
    eg = np.sort(inv[src] * n + inv[g.adj])
    eh = np.sort(np.repeat(np.arange(n, dtype=np.int64), np.diff(h.xadj)) * n + h.adj)
    assert np.array_equal(eg, eh)
    gap_h = np.abs(np.repeat(np.arange(n), np.diff(h.xadj)) - h.adj).mean()
    gap_g = np.abs(src - g.adj).mean()
    assert gap_h * 20 < gap_g
