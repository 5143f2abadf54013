"""Generators: shapes, symmetry, determinism (no method arithmetic here)."""
import math

import numpy as np

import oracle as O
from workloads import batch_graphs, grid2d, random_graph, rgg, rmat


def _symmetric(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj))
    a = src * g.n + g.adj
    b = g.adj.astype(np.int64) * g.n + src
    ia, ib = np.argsort(a), np.argsort(b)
    return np.array_equal(a[ia], b[ib]) and np.array_equal(g.ew[ia], g.ew[ib])


def test_grid_counts():
    g = grid2d(64, 64)
    assert (g.n, g.m, g.nnz) == (4096, 8064, 16128)
    assert O.validate(g) == O.OK
    deg = g.degrees()
    assert deg.min() == 2 and deg.max() == 4 and (deg == 2).sum() == 4


def test_rgg_mean_degree_and_determinism():
    n = 1 << 15
    g = rgg(n, seed=2)
    assert O.validate(g) == O.OK and _symmetric(g)
    assert abs(g.nnz / n - 8.0) < 0.4
    h = rgg(n, seed=2)
    assert np.array_equal(g.adj, h.adj) and np.array_equal(g.xadj, h.xadj)
    assert not np.array_equal(g.adj[:1000], rgg(n, seed=5).adj[:1000])


def test_rmat_simple_symmetric_weighted():
    g = rmat(12, 16, seed=3, wseed=33)
    assert g.n == 4096 and O.validate(g) == O.OK and _symmetric(g)
    assert g.ew.min() >= 1 and g.ew.max() <= 100
    deg = g.degrees()
    assert deg.max() > 20 * deg.mean()          # power-law skew
    h = rmat(12, 16, seed=3, wseed=33)
    assert np.array_equal(g.adj, h.adj) and np.array_equal(g.ew, h.ew)


def test_random_graph_and_batch():
    g = random_graph(100, 300, seed=1, wmax=5, cmax=4, cmin=0)
    assert O.validate(g) == O.OK and g.m == 300
    gs = batch_graphs(count=6, seed=4, nmin=1e3, nmax=4e3)
    for i, b in enumerate(gs):
        assert O.validate(b) == O.OK
        assert 1 <= b.ew.min() and b.ew.max() <= 16 and 1 <= b.vw.min() and b.vw.max() <= 16
        assert 700 <= b.n <= 4500


def test_rcb_order_is_a_relabelling_with_locality():
    from workloads.graphs import rcb_order, rgg_points
    n = 1 << 14
    pts = rgg_points(n, 9)
    o = rcb_order(pts, leaf=32)
    assert np.array_equal(np.sort(o), np.arange(n))
    # every bisection: the lower half of a box lies at or below the upper
    # half along x at even depths, along y at odd depths
    q = pts[o]
    size, depth = n, 0
    while size > 32:
        for a in range(0, n, size):
            lo, hi = q[a:a + size // 2], q[a + size // 2:a + size]
            assert lo[:, depth % 2].max() <= hi[:, depth % 2].min()
        size, depth = size // 2, depth + 1
    # the rcb graph is the generation-order graph with node i renamed inv[i]
    g, h = rgg(n, seed=9), rgg(n, seed=9, order="rcb")
    assert O.validate(h) == O.OK and _symmetric(h) and h.m == g.m
    inv = np.empty(n, dtype=np.int64)
    inv[o] = np.arange(n)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.xadj))
    eg = np.sort(inv[src] * n + inv[g.adj])
    eh = np.sort(np.repeat(np.arange(n, dtype=np.int64), np.diff(h.xadj)) * n + h.adj)
    assert np.array_equal(eg, eh)
    # ids of neighbours are close in rcb order, far in generation order
    gap = lambda x, s: np.abs(s - x.adj).mean()
    assert gap(h, np.repeat(np.arange(n), np.diff(h.xadj))) * 20 < gap(g, src)


def test_relabel_reference():
    from workloads import rcb_order, relabel, rgg_points
    n = 1 << 13
    pts = rgg_points(n, 4)
    o = rcb_order(pts)
    h = relabel(rgg(n, seed=4), o)
    r = rgg(n, seed=4, order="rcb")
    assert np.array_equal(h.xadj, r.xadj) and np.array_equal(h.adj, r.adj)
    assert np.array_equal(h.ew, r.ew) and np.array_equal(h.vw, r.vw)
    g = rmat(10, 8, seed=1, wseed=2)
    perm = np.random.default_rng(3).permutation(g.n)
    back = relabel(relabel(g, perm), np.argsort(perm))
    assert np.array_equal(back.xadj, g.xadj) and np.array_equal(back.adj, g.adj)
    assert np.array_equal(back.ew, g.ew) and np.array_equal(back.vw, g.vw)
