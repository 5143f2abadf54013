"""Oracle runs for the parity tests that compare many graphs: each returns
SHA-256 digests of the oracle's hierarchy and way back up, so that worker
processes (which import neither torch nor the HIP library) can run them in
parallel with the GPU."""
import hashlib

import numpy as np

import oracle as O
from workloads.graphs import _batch_member


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def hierarchy_digest(levels, parts, res):
    """Per level: n, nnz, digests of the four CSR arrays and of cmap (None on
    the coarsest level), |M|, stop reason; the level-0 partition's digest and
    every level's cut/balance tuple."""
    out = []
    for lv in levels:
        G = lv.graph
        out.append((int(G.n), int(G.xadj[-1]) if G.n else 0, digest(G.xadj, np.int64),
                    digest(G.adj, np.int32), digest(G.ew, np.uint32), digest(G.vw, np.uint32),
                    None if lv.cmap is None else digest(lv.cmap, np.int32), int(lv.matched),
                    int(lv.stop_reason)))
    return out, digest(parts[0], np.int32), [tuple(int(x) for x in r.as_tuple()) for r in res]


def batch_member_digest(args):
    """Graph g of the uneven batch (sub-seed (seed, g), ng nodes, weights in
    [1, wmax]) coarsened by the oracle alone (rating, seed, stop_n, stall
    1/20, 64 levels at most), then its way back up with the stand-in
    partition (k, part seed 1, eps 3/100)."""
    seed, g, ng, wmax, rating, cseed, stop_n, k = args
    gr = _batch_member(seed, g, ng, wmax)
    H = O.coarsen(gr, rating, cseed, stop_n, 1, 20, 64)
    parts, res = O.uncoarsen(H, k, 1, 3, 100)
    return hierarchy_digest(H.levels, parts, res)


def served_graph(spec):
    """A graph of the served tests by its recipe: ("mix", seed, i, emin, emax)
    is member i of the served mix, ("grid", side), ("rgg", n, seed) and
    ("rmat", scale, seed, wseed) the generators' own graphs."""
    from workloads import grid2d, rgg, rmat
    from workloads.graphs import _serve_member
    kind = spec[0]
    if kind == "mix":
        return _serve_member(*spec[1:])[0]
    if kind == "grid":
        return grid2d(spec[1], spec[1])
    if kind == "rgg":
        return rgg(spec[1], seed=spec[2])
    return rmat(spec[1], 16, seed=spec[2], wseed=spec[3])


def served_digest(args):
    """A served request run by the oracle alone: the graph of `spec`
    coarsened with (rating, seed, stop_n, stall 1/20, max_levels), then its
    way back up with the stand-in partition (k, part seed 1, eps 3/100)."""
    spec, rating, cseed, stop_n, max_levels, k = args
    g = served_graph(spec)
    H = O.coarsen(g, rating, cseed, stop_n, 1, 20, max_levels)
    parts, res = O.uncoarsen(H, k, 1, 3, 100)
    return hierarchy_digest(H.levels, parts, res)
