"""Graph generators (numpy).  Every generator is deterministic for its seed.

Recipes (the workload families of the partitioner's experiments, Section 6):
  * ``grid2d``     -- rows x cols 4-neighbour mesh, id = row*cols + col.
  * ``rgg``        -- random geometric graph: n points uniform in the unit
                      square (numpy PCG64), edge iff Euclidean distance < r.
                      The paper's instances use r = 0.55 sqrt(ln n / n); the
                      default here picks r for a mean degree of 8,
                      r = sqrt(8 / (pi n)).
  * ``rmat``       -- R-MAT power-law graph: each of edge_factor * 2^scale
                      samples descends ``scale`` quadrant levels with
                      probabilities (a, b, c, 1-a-b-c); self loops dropped,
                      symmetrised, duplicates removed; edge weights uniform
                      integers in [1, wmax] drawn per undirected edge in
                      ascending (min, max) order.
  * ``batch_graphs`` -- the uneven batch: n log-uniform, half degraded grids
                      (10 % of edges removed), half RGGs of mean degree 8,
                      node and edge weights uniform in [1, 16].
  * ``serve_requests`` -- the served mix: |E| log-uniform, graph type uniform
                      over {grid of side sqrt(|E|/2); random geometric graph
                      with n = |E|/4; R-MAT of scale log2(|E|/16) clamped to
                      [6, 20], edge factor 16, weights in [1, 100]}, rating
                      uniform over {expansion*2, innerOuter}, k uniform over
                      {2, 8, 32, 64}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class CSR:
    n: int
    xadj: np.ndarray   # int64[n+1]
    adj: np.ndarray    # int32[nnz]
    ew: np.ndarray     # uint32[nnz]
    vw: np.ndarray     # uint32[n]

    @property
    def nnz(self) -> int:
        return int(self.xadj[-1]) if len(self.xadj) else 0

    @property
    def m(self) -> int:
        """Undirected edge count |E| = nnz / 2."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.xadj)


def csr_from_edges(n: int, a: np.ndarray, b: np.ndarray, w: Optional[np.ndarray] = None,
                   vw: Optional[np.ndarray] = None) -> CSR:
    """Symmetric CSR with ascending rows from undirected edges {a_i, b_i}.

    The edge list must hold no self loop and no duplicate pair.
    """
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    m = len(a)
    if w is None:
        w = np.ones(m, dtype=np.uint32)
    w = np.asarray(w, dtype=np.uint32)
    if vw is None:
        vw = np.ones(n, dtype=np.uint32)
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    key = src * np.int64(max(n, 1)) + dst
    order = np.argsort(key, kind="stable")
    src, dst, ww = src[order], dst[order], ww[order]
    counts = np.bincount(src, minlength=n) if m else np.zeros(n, dtype=np.int64)
    xadj = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=xadj[1:])
    return CSR(n, xadj, dst.astype(np.int32), ww.astype(np.uint32),
               np.asarray(vw, dtype=np.uint32).copy())


def _canonical_pairs(a: np.ndarray, b: np.ndarray, n: int):
    """Drop self loops, orient min<max, remove duplicates; sorted by (min,max)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = np.unique(lo * np.int64(n) + hi)
    return key // n, key % n


# ---------------------------------------------------------------------------
def grid2d(rows: int, cols: int, ew: Optional[np.ndarray] = None,
           vw: Optional[np.ndarray] = None) -> CSR:
    """4-neighbour mesh; edge list order: horizontal edges then vertical."""
    n = rows * cols
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    idx = (r * cols + c).astype(np.int64)
    ha, hb = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    va, vb = idx[:-1, :].ravel(), idx[1:, :].ravel()
    a = np.concatenate([ha, va])
    b = np.concatenate([hb, vb])
    return csr_from_edges(n, a, b, ew, vw)


def degrade_grid(rows: int, cols: int, frac: float, rng: np.random.Generator,
                 wmax: int = 16) -> CSR:
    """Grid minus floor(frac * m) edges drawn without replacement; weights in [1, wmax]."""
    n = rows * cols
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    idx = (r * cols + c).astype(np.int64)
    a = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    b = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    m = len(a)
    drop = rng.choice(m, size=int(math.floor(frac * m)), replace=False)
    keep = np.ones(m, dtype=bool)
    keep[drop] = False
    a, b = a[keep], b[keep]
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    w = rng.integers(1, wmax + 1, size=len(a), dtype=np.int64).astype(np.uint32)
    vw = rng.integers(1, wmax + 1, size=n, dtype=np.int64).astype(np.uint32)
    return csr_from_edges(n, a, b, w, vw)


def rgg_points(n: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).random((n, 2))


def rgg(n: int, seed: int, radius: Optional[float] = None, mean_degree: float = 8.0,
        ew: Optional[np.ndarray] = None, vw: Optional[np.ndarray] = None,
        points: Optional[np.ndarray] = None) -> CSR:
    """Random geometric graph in the unit square; edge iff distance < radius;
    node ids in the points' generation order."""
    from scipy.spatial import cKDTree
    if radius is None:
        radius = math.sqrt(mean_degree / (math.pi * n))
    pts = rgg_points(n, seed) if points is None else points
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    if len(pairs):
        d = pts[pairs[:, 0]] - pts[pairs[:, 1]]
        pairs = pairs[(d * d).sum(axis=1) < radius * radius]
    a = np.minimum(pairs[:, 0], pairs[:, 1]).astype(np.int64) if len(pairs) else np.zeros(0, np.int64)
    b = np.maximum(pairs[:, 0], pairs[:, 1]).astype(np.int64) if len(pairs) else np.zeros(0, np.int64)
    order = np.lexsort((b, a))
    return csr_from_edges(n, a[order], b[order], ew, vw)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 3, wseed: int = 33, wmax: int = 100, chunk: int = 1 << 24) -> CSR:
    """R-MAT graph: 2^scale nodes, edge_factor * 2^scale samples (see module doc)."""
    n = 1 << scale
    total = edge_factor * n
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = []
    ab, abc = a + b, a + b + c
    for start in range(0, total, chunk):
        cnt = min(chunk, total - start)
        src = np.zeros(cnt, dtype=np.int64)
        dst = np.zeros(cnt, dtype=np.int64)
        for lev in range(scale):
            r = rng.random(cnt)
            sbit = r >= ab
            dbit = ((r >= a) & (r < ab)) | (r >= abc)
            bit = np.int64(1) << np.int64(scale - 1 - lev)
            src |= sbit.astype(np.int64) * bit
            dst |= dbit.astype(np.int64) * bit
        keep = src != dst
        src, dst = src[keep], dst[keep]
        lo = np.minimum(src, dst)
        hi = np.maximum(src, dst)
        keys.append(np.unique(lo * np.int64(n) + hi))
        del src, dst, lo, hi
    key = np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.int64)
    del keys
    lo = key // n
    hi = key % n
    del key
    wr = np.random.Generator(np.random.PCG64(wseed))
    w = wr.integers(1, wmax + 1, size=len(lo), dtype=np.int64).astype(np.uint32)
    return csr_from_edges(n, lo, hi, w, np.ones(n, dtype=np.uint32))


def random_graph(n: int, m: int, seed: int, wmax: int = 1, cmax: int = 1, cmin: int = 1) -> CSR:
    """Uniform random simple graph with about m edges; weights in [1,wmax], c in [cmin,cmax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n < 2:
        return csr_from_edges(n, np.zeros(0), np.zeros(0), None,
                              rng.integers(cmin, cmax + 1, size=n).astype(np.uint32))
    aa = rng.integers(0, n, size=2 * m + 4)
    bb = rng.integers(0, n, size=2 * m + 4)
    lo, hi = _canonical_pairs(aa, bb, n)
    if len(lo) > m:
        pick = np.sort(rng.choice(len(lo), size=m, replace=False))
        lo, hi = lo[pick], hi[pick]
    w = rng.integers(1, wmax + 1, size=len(lo)).astype(np.uint32)
    vw = rng.integers(cmin, cmax + 1, size=n).astype(np.uint32)
    return csr_from_edges(n, lo, hi, w, vw)


def path_graph(weights, vw=None) -> CSR:
    n = len(weights) + 1
    a = np.arange(n - 1)
    return csr_from_edges(n, a, a + 1, np.asarray(weights, dtype=np.uint32), vw)


def cycle_graph(n: int, w=None) -> CSR:
    a = np.arange(n)
    b = (a + 1) % n
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    order = np.lexsort((hi, lo))
    ww = None if w is None else np.asarray(w, dtype=np.uint32)[order]
    return csr_from_edges(n, lo[order], hi[order], ww)


def star_graph(leaves: int) -> CSR:
    a = np.zeros(leaves, dtype=np.int64)
    b = np.arange(1, leaves + 1)
    return csr_from_edges(leaves + 1, a, b)


def complete_graph(n: int, w=None) -> CSR:
    a, b = np.triu_indices(n, 1)
    return csr_from_edges(n, a, b, None if w is None else np.asarray(w, dtype=np.uint32))


def _batch_member(seed: int, g: int, ng: int, wmax: int) -> CSR:
    rng = np.random.Generator(np.random.PCG64([seed, g]))
    if g % 2 == 0:
        rows = max(2, int(round(math.sqrt(ng))))
        cols = max(2, int(round(ng / rows)))
        return degrade_grid(rows, cols, 0.1, rng, wmax)
    pts = rng.random((ng, 2))
    tmp = rgg(ng, 0, points=pts)
    w = rng.integers(1, wmax + 1, size=tmp.m, dtype=np.int64).astype(np.uint32)
    vw = rng.integers(1, wmax + 1, size=ng, dtype=np.int64).astype(np.uint32)
    # re-weight: the edge list of tmp in (min,max) order
    src = np.repeat(np.arange(ng, dtype=np.int64), np.diff(tmp.xadj))
    sel = tmp.adj > src
    return csr_from_edges(ng, src[sel], tmp.adj[sel].astype(np.int64), w, vw)


def batch_graphs(count: int = 4096, seed: int = 4, nmin: float = 1e3, nmax: float = 6.4e4,
                 wmax: int = 16, workers: int = 1) -> List[CSR]:
    """The uneven batch (see module doc).  Graph g uses sub-seed (seed, g), so
    the result does not depend on `workers` (processes generating it)."""
    top = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(top.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)
    args = [(seed, g, int(sizes[g]), wmax) for g in range(count)]
    if workers <= 1:
        return [_batch_member(*a) for a in args]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_batch_member, *zip(*args), chunksize=16))


def _serve_member(seed: int, i: int, emin: float, emax: float) -> Tuple[CSR, int, int]:
    rng = np.random.Generator(np.random.PCG64([seed, i]))
    e = float(np.exp(rng.uniform(math.log(emin), math.log(emax))))
    kind = int(rng.integers(0, 3))
    rating = int(rng.integers(0, 2))
    k = int((2, 8, 32, 64)[int(rng.integers(0, 4))])
    sub = int(rng.integers(0, 2**31 - 1))
    if kind == 0:
        side = max(2, int(round(math.sqrt(e / 2))))
        g = grid2d(side, side)
    elif kind == 1:
        g = rgg(max(2, int(round(e / 4))), seed=sub)
    else:
        scale = min(20, max(6, int(round(math.log2(e / 16)))))
        g = rmat(scale, 16, seed=sub, wseed=sub + 1)
    return g, rating, k


def serve_requests(count: int = 2000, seed: int = 5, emin: float = 1e3, emax: float = 4e6,
                   workers: int = 1) -> List[Tuple[CSR, int, int]]:
    """The served mix (see module doc): (graph, rating, k) per request.
    Request i uses sub-seed (seed, i), independent of `workers`."""
    args = [(seed, i, emin, emax) for i in range(count)]
    if workers <= 1:
        return [_serve_member(*a) for a in args]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_serve_member, *zip(*args), chunksize=4))
