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
