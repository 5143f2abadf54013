"""Test infrastructure: the reference for the locality relabelling (the
preliminary partition of Section 3.3 by recursive bisection of the nodes'
2D coordinates, alternately by x and by y) and for renumbering a graph.
Only the tests and the bench's CPU baseline use this module.

rcb_order follows the definition recursively: a box of more than `leaf`
points is ordered stably by x (at even depths) or y (at odd depths), cut
after its first len // 2 points, and each half is ordered the same way one
depth deeper, the lower half first; a box of at most `leaf` points keeps its
order.

relabel follows its definition: node x of the result is node order[x] of
the input, every CSR entry (v, u, w) becomes (inv[v], inv[u], w), and the
entries are sorted by (row, neighbour) with a library sort.
"""
import sys

import numpy as np

from . import Graph


def rcb_order(pts, leaf: int = 32) -> np.ndarray:
    pts = np.asarray(pts, dtype=np.float64) + 0.0   # -0.0 reads as +0.0
    sys.setrecursionlimit(max(sys.getrecursionlimit(), 10000))

    def order(idx, depth):
        if len(idx) <= leaf:
            return [idx]
        srt = idx[np.argsort(pts[idx, depth % 2], kind="stable")]   # equal keys keep their order
        mid = len(srt) // 2
        return order(srt[:mid], depth + 1) + order(srt[mid:], depth + 1)

    n = len(pts)
    return np.concatenate(order(np.arange(n, dtype=np.int64), 0)) if n else np.zeros(0, np.int64)


def relabel(g, order) -> Graph:
    order = np.asarray(order, dtype=np.int64)
    n = g.n
    assert np.array_equal(np.sort(order), np.arange(n)), "order must be a permutation"
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(g.xadj, dtype=np.int64)))
    rows, nbrs = inv[src], inv[np.asarray(g.adj, dtype=np.int64)]
    perm = np.lexsort((nbrs, rows))
    xadj = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=xadj[1:])
    return Graph(n, xadj, nbrs[perm].astype(np.int32), np.asarray(g.ew, dtype=np.uint32)[perm],
                 np.asarray(g.vw, dtype=np.uint32)[order])
