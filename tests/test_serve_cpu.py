"""Host logic of the served form: how the dispatcher forms a batch out of the
requests that have arrived (no GPU)."""
import numpy as np

from paper_0910_2004_amd.serve import WEIGHT_CAP, Request, footprint, take_batch, weight_sums
from workloads import CSR, grid2d, path_graph


def _heavy(n, w):
    """A path on n nodes with every edge weight w and every node weight 1."""
    g = path_graph([1] * (n - 1))
    return CSR(g.n, g.xadj, g.adj, np.full(len(g.adj), w, np.uint32), g.vw)


def test_weight_sums():
    g = grid2d(3, 4)   # 17 edges of weight 1, 12 nodes of weight 1
    assert weight_sums(g) == (17, 12)
    h = _heavy(5, 7)
    assert weight_sums(h) == (4 * 7, 5)


def test_batch_keeps_rating_seed_and_order():
    g = grid2d(4, 4)
    reqs = [Request(0, g, 0, 2), Request(1, g, 1, 2), Request(2, g, 0, 2), Request(3, g, 0, 2, seed=7),
            Request(4, g, 0, 8)]
    batch, rest = take_batch(reqs, 1 << 40, 512, {})
    assert [r.rid for r in batch] == [0, 2, 4]
    assert [r.rid for r in rest] == [1, 3]


def test_batch_limits():
    g = grid2d(10, 10)
    reqs = [Request(i, g, 0, 2) for i in range(6)]
    fp = footprint(g)
    batch, rest = take_batch(reqs, 3 * fp, 512, {})
    assert len(batch) == 3 and len(rest) == 3
    batch, rest = take_batch(reqs, 1, 512, {})          # a tiny budget: one at a time
    assert [r.rid for r in batch] == [0]
    batch, rest = take_batch(reqs, 1 << 40, 4, {})
    assert len(batch) == 4


def test_batch_union_weight_sums_fit_32_bits():
    w = (WEIGHT_CAP // 3) // 9 + 1        # 9 edges: each graph holds a bit over a third of the cap
    g = _heavy(10, w)
    assert 3 * weight_sums(g)[0] > WEIGHT_CAP >= 2 * weight_sums(g)[0]
    reqs = [Request(i, g, 0, 2) for i in range(5)]
    batch, rest = take_batch(reqs, 1 << 40, 512, {})
    assert [r.rid for r in batch] == [0, 1]
    assert sum(weight_sums(r.graph)[0] for r in batch) <= WEIGHT_CAP
