"""Pure-Python brute-force checks for tiny graphs, written independently of the
C oracle: ratings as ``fractions.Fraction``, matchings by exhaustive search,
contraction with dictionaries.  Used only to pin the oracle."""
from __future__ import annotations

import itertools
from fractions import Fraction

M64 = (1 << 64) - 1


def mix64(z: int) -> int:
    """SplitMix64 output function (pinned by the published stream values)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def edges_of(g):
    """Undirected edges (a, b, w) with a < b, from a CSR."""
    out = []
    for v in range(g.n):
        for j in range(int(g.xadj[v]), int(g.xadj[v + 1])):
            u = int(g.adj[j])
            if u > v:
                out.append((v, u, int(g.ew[j])))
    return out


def out_of(g):
    return [sum(int(g.ew[j]) for j in range(int(g.xadj[v]), int(g.xadj[v + 1]))) for v in range(g.n)]


INF = None  # marker for a zero denominator


def rating_value(kind: str, w: int, cu: int, cv: int, ou: int, ov: int):
    """Section 3.1 ratings as Fractions; a zero denominator gives +infinity
    (returned as (1, 0) so that it sorts above every finite value)."""
    if kind == "weight":
        num, den = w, 1
    elif kind == "expansion":
        num, den = w, cu + cv
    elif kind == "expansion*":
        num, den = w, cu * cv
    elif kind == "expansion*2":
        num, den = w * w, cu * cv
    elif kind == "innerOuter":
        num, den = w, ou + ov - 2 * w
    else:
        raise ValueError(kind)
    if den == 0:
        return (1, Fraction(0))
    return (0, Fraction(num, den))


def order_key(kind, g, seed, a, b, w, outs):
    """Sort key: larger key = higher in the strict edge order."""
    cu, cv = int(g.vw[a]), int(g.vw[b])
    r = rating_value(kind, w, cu, cv, outs[a], outs[b])
    eid = (min(a, b) << 32) | max(a, b)
    return (r, mix64(seed ^ eid), -eid)


def greedy(g, kind, seed):
    """Greedy of Section 3.2 under the strict order."""
    outs = out_of(g)
    es = edges_of(g)
    es.sort(key=lambda e: order_key(kind, g, seed, e[0], e[1], e[2], outs), reverse=True)
    mate = [-1] * g.n
    for a, b, _ in es:
        if mate[a] < 0 and mate[b] < 0:
            mate[a], mate[b] = b, a
    return mate


def all_matchings(n, es):
    """Every matching of the edge list (exponential; tiny graphs only)."""
    res = []

    def rec(i, used, cur):
        if i == len(es):
            res.append(list(cur))
            return
        rec(i + 1, used, cur)
        a, b = es[i][0], es[i][1]
        if a not in used and b not in used:
            used.add(a); used.add(b); cur.append(es[i])
            rec(i + 1, used, cur)
            cur.pop(); used.discard(a); used.discard(b)

    rec(0, set(), [])
    return res


def finite_value(kind, g, e, outs):
    inf, val = rating_value(kind, e[2], int(g.vw[e[0]]), int(g.vw[e[1]]), outs[e[0]], outs[e[1]])
    return val if not inf else None


def contract_dict(g, mate):
    """Contraction of Section 2 with dictionaries and min-representative ids."""
    reps = [v for v in range(g.n) if mate[v] < 0 or v < mate[v]]
    cid = {v: i for i, v in enumerate(reps)}
    cmap = [cid[v] if (mate[v] < 0 or v < mate[v]) else cid[mate[v]] for v in range(g.n)]
    nc = len(reps)
    cvw = [0] * nc
    for v in range(g.n):
        cvw[cmap[v]] += int(g.vw[v])
    rows = [dict() for _ in range(nc)]
    for a, b, w in edges_of(g):
        x, y = cmap[a], cmap[b]
        if x == y:
            continue
        rows[x][y] = rows[x].get(y, 0) + w
        rows[y][x] = rows[y].get(x, 0) + w
    xadj = [0]
    adj, ew = [], []
    for x in range(nc):
        for y in sorted(rows[x]):
            adj.append(y)
            ew.append(rows[x][y])
        xadj.append(len(adj))
    return cmap, nc, xadj, adj, ew, cvw


def local_max_rounds(n, es, key):
    """Synchronous rounds: every free node points at its best edge (by
    `key`) to a free neighbour; edges chosen at both ends are matched."""
    mate = [-1] * n
    adj = [[] for _ in range(n)]
    for e in es:
        adj[e[0]].append(e)
        adj[e[1]].append(e)
    while True:
        best = {}
        for v in range(n):
            if mate[v] >= 0:
                continue
            cand = [e for e in adj[v] if mate[e[0] if e[1] == v else e[1]] < 0]
            if cand:
                best[v] = max(cand, key=key)
        if not best:
            return mate
        for v, e in best.items():
            u = e[0] if e[1] == v else e[1]
            if best.get(u) is e and mate[v] < 0:
                mate[v], mate[u] = u, v


def two_phase_rounds(g, kind, seed, block_bits):
    """Section 3.3's two-phase matching in its round form: local-max rounds on
    the block-internal edges (blocks of 2^block_bits consecutive ids), then
    local-max rounds on the edges between blocks that beat the block edge
    matched at each end; those replace the block edges at their ends."""
    outs = out_of(g)
    key = lambda e: order_key(kind, g, seed, e[0], e[1], e[2], outs)
    es = edges_of(g)
    inner = [e for e in es if e[0] >> block_bits == e[1] >> block_bits]
    loc = local_max_rounds(g.n, inner, key)
    wloc = {}
    for a, b, w in inner:
        if loc[a] == b:
            wloc[a] = wloc[b] = key((a, b, w))
    gap = [e for e in es if e[0] >> block_bits != e[1] >> block_bits
           and all(x not in wloc or key(e) > wloc[x] for x in e[:2])]
    gm = local_max_rounds(g.n, gap, key)
    return [gm[v] if gm[v] >= 0 else (loc[v] if loc[v] >= 0 and gm[loc[v]] < 0 else -1)
            for v in range(g.n)]


def fm_pair_ref(g, part, k, a, b, run_seed, alpha, depth, eps):
    """A second, dictionary-based writing of one two-block local search
    (Section 5.2) with the same readings as the oracle: gains over the two
    blocks, bounded BFS area, TopGain with the MaxLoad exception, patience
    alpha * min(|A|, |B|), rollback to the smallest (imbalance, cut).
    Returns (moves, kept).  For tiny graphs only."""
    nbr = {v: {} for v in range(g.n)}
    for v in range(g.n):
        for j in range(int(g.xadj[v]), int(g.xadj[v + 1])):
            nbr[v][int(g.adj[j])] = int(g.ew[j])
    c = [int(x) for x in g.vw]
    where = {v: (0 if part[v] == a else 1) for v in range(g.n) if part[v] in (a, b)}
    total, maxc = sum(c), max(c) if c else 0
    S = k * eps.denominator
    L = (eps.denominator + eps.numerator) * total + S * maxc
    w = [sum(c[v] for v in where if where[v] == s) for s in (0, 1)]
    size = [sum(1 for v in where if where[v] == s) for s in (0, 1)]

    def imb():
        return max(0, S * max(w) - L)

    def gain(v):
        return sum(x if where[u] != where[v] else -x for u, x in nbr[v].items() if u in where)

    def cut():
        return sum(x for v in where for u, x in nbr[v].items()
                   if u in where and where[v] == 0 and where[u] == 1)

    # bounded BFS inside each block from the boundary
    dist = {v: 0 for v in where if any(u in where and where[u] != where[v] for u in nbr[v])}
    frontier = sorted(dist)
    for d in range(1, depth + 1):
        nxt = []
        for v in frontier:
            for u in nbr[v]:
                if u in where and where[u] == where[v] and u not in dist:
                    dist[u] = d
                    nxt.append(u)
        frontier = nxt
    queued = {v for v in dist if dist[v] == 0}
    moved = []
    best, kept, since = (imb(), cut()), 0, 0
    while True:
        tops = []
        for s in (0, 1):
            cand = [v for v in queued if where[v] == s]
            tops.append(max(cand, key=lambda v: (gain(v), mix64(run_seed ^ v), -v)) if cand else None)
        if tops[0] is None and tops[1] is None:
            break
        key = lambda v: (gain(v), mix64(run_seed ^ v), -v)
        if (S * w[0] > L or S * w[1] > L) and w[0] != w[1]:
            s = 0 if w[0] > w[1] else 1
            if tops[s] is None:
                s = 1 - s
        elif tops[0] is None or tops[1] is None:
            s = 0 if tops[1] is None else 1
        else:
            s = 0 if key(tops[0]) > key(tops[1]) else 1
        v = tops[s]
        queued.discard(v)
        where[v] = 1 - s
        w[s] -= c[v]
        w[1 - s] += c[v]
        moved.append(v)
        for u in nbr[v]:
            if u in dist and u not in queued and u not in moved:
                queued.add(u)
        now = (imb(), cut())
        if now < best:
            best, kept, since = now, len(moved), 0
        else:
            since += 1
        if since > alpha * min(size):
            break
    return moved, kept
