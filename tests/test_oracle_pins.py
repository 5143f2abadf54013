"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: hand-worked
graphs (tests/golden), published generator values, closed forms, brute-force
enumeration, an independent pure-Python implementation (tests/refpy.py) and
invariants of the definitions.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import refpy
from workloads import (complete_graph, csr_from_edges, cycle_graph, grid2d, path_graph,
                       random_graph, star_graph)

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RATING_NAMES = ["expansion*2", "innerOuter", "weight", "expansion", "expansion*"]


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def graph_from(spec):
    e = np.array(spec["edges"], dtype=np.int64).reshape(-1, 3)
    return csr_from_edges(spec["n"], e[:, 0], e[:, 1], e[:, 2].astype(np.uint32),
                          np.array(spec["vw"], dtype=np.uint32))


# --------------------------------------------------------------------------
# tie-break hash
# --------------------------------------------------------------------------
def test_splitmix64_published_stream():
    g = gold("splitmix64.json")
    want = [int(x, 16) for x in g["outputs"]]
    assert O.splitmix64_stream(g["state"], len(want)) == want
    # the pure-Python copy used by the brute-force checks is pinned by the same values
    s, got = g["state"], []
    for _ in want:
        s = (s + 0x9E3779B97F4A7C15) & refpy.M64
        got.append(refpy.mix64(s))
    assert got == want


def test_mix64_is_a_bijection_sample():
    xs = list(range(0, 1 << 16)) + [(1 << 64) - 1 - i for i in range(1000)]
    hs = {O.mix64(x) for x in xs}
    assert len(hs) == len(xs)


# The stand-in coarsest partition: part(x) = mix64(seed + x) mod k.  The
# published SplitMix64 stream with state 0 outputs mix64(i * gamma) at step i,
# so a seed of i * gamma - x puts that output at node x.  A seed mixed by XOR,
# a missing mix, or a reduction other than the remainder fails here.
GAMMA = 0x9E3779B97F4A7C15


@pytest.mark.parametrize("k", [1, 2, 3, 7, 64, 100, 255, 256])
def test_initial_partition_published_stream(k):
    g = gold("splitmix64.json")
    assert g["state"] == 0
    for i, h in enumerate(g["outputs"], start=1):
        for x in (0, 1, 2, 5, 1000):
            seed = (i * GAMMA - x) % (1 << 64)
            part = O.initial_partition(x + 1, k, seed)
            assert int(part[x]) == int(h, 16) % k, (i, x, k)
    # seed = gamma: node 0 takes the first output
    assert int(O.initial_partition(1, k, GAMMA)[0]) == 0xE220A8397B1DCDAF % k


def test_initial_partition_matches_python_mix64():
    rng = np.random.default_rng(11)
    for _ in range(20):
        seed = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        k = int(rng.integers(1, 257))
        n = int(rng.integers(0, 300))
        part = O.initial_partition(n, k, seed)
        want = [refpy.mix64((seed + x) % (1 << 64)) % k for x in range(n)]
        assert part.tolist() == want


# --------------------------------------------------------------------------
# W1: P4 with weights 3, 4, 2 -- ratings, every level, projection, L_max
# --------------------------------------------------------------------------
def test_w1_csr_and_ratings():
    w = gold("w1_p4.json")
    g = graph_from(w["graph"])
    assert g.xadj.tolist() == w["csr"]["xadj"]
    assert g.adj.tolist() == w["csr"]["adj"]
    assert g.ew.tolist() == w["csr"]["ew"]
    assert O.out_weights(g).tolist() == w["out"]
    for name, want in w["rate"].items():
        num, den = O.rate(g, O.RATINGS[name])
        assert num.tolist() == want["num"] and den.tolist() == want["den"], name


@pytest.mark.parametrize("rating", RATING_NAMES)
def test_w1_hierarchy(rating):
    w = gold("w1_p4.json")
    g = graph_from(w["graph"])
    H = O.coarsen(g, O.RATINGS[rating], seed=42, stop_n=1, cross_check=True)
    assert len(H.levels) == 4 and H.levels[-1].graph.n == 1
    for lv, want in zip(H.levels, w["levels"]):
        G = lv.graph
        assert G.n == want["n"]
        assert G.xadj.tolist() == want["xadj"] and G.adj.tolist() == want["adj"]
        assert G.ew.tolist() == want["ew"] and G.vw.tolist() == want["vw"]
        if "mate" in want:
            assert lv.mate.tolist() == want["mate"]
            assert lv.rounds == want["rounds"]
            assert lv.cmap.tolist() == want["cmap"]
    num, den = O.rate(H.levels[1].graph, O.RATINGS[rating])
    assert num.tolist() == w["level1_rate"][rating]["num"]
    assert den.tolist() == w["level1_rate"][rating]["den"]
    if rating == "innerOuter":
        _, den2 = O.rate(H.levels[2].graph, O.INNER_OUTER)
        assert den2.tolist() == [w["level2_innerOuter_den"]] * 2


def test_w1_projection_and_lmax():
    w = gold("w1_p4.json")
    g = graph_from(w["graph"])
    H = O.coarsen(g, O.EXPANSION_STAR2, seed=42, stop_n=1)
    p1 = np.array(w["projection"]["part1"], dtype=np.int32)
    p0 = O.project(H.levels[0].cmap, p1)
    assert p0.tolist() == w["projection"]["part0"]
    r1 = O.cut_balance(H.levels[1].graph, p1, 2, 3, 100)
    r0 = O.cut_balance(g, p0, 2, 3, 100)
    assert r1.cut == r0.cut == w["projection"]["cut"]
    assert r1.block_w.tolist() == r0.block_w.tolist() == w["projection"]["block_w"]
    assert [r0.lmax_num, r0.lmax_den] == w["lmax_k2_eps3_100"]["level0"]
    assert [r1.lmax_num, r1.lmax_den] == w["lmax_k2_eps3_100"]["level1"]
    # L_max = (1 + eps) c(V)/k + max c(v) (Section 2) written out with Fractions
    assert Fraction(r0.lmax_num, r0.lmax_den) == Fraction(103, 100) * 4 / 2 + 1


def test_w2_monotone_path_rounds():
    w = gold("w2_p5.json")
    g = graph_from(w["graph"])
    mate, m, rounds, act, deg = O.match_rounds(g, O.EXPANSION_STAR2, O.level_seed(42, 0))
    assert mate.tolist() == w["mate"] and rounds == w["rounds"] and m == 2
    assert act.tolist() == w["round_active"]      # pointing nodes per round
    assert deg.tolist() == w["round_degree"]      # their degree sums (full degrees)
    gm, gmm = O.match_greedy(g, O.EXPANSION_STAR2, O.level_seed(42, 0))
    assert gm.tolist() == w["mate"]
    cmap, cg = O.contract(g, mate)
    assert cmap.tolist() == w["cmap"]
    c = w["coarse"]
    assert (cg.n, cg.xadj.tolist(), cg.adj.tolist(), cg.ew.tolist(), cg.vw.tolist()) == \
        (c["n"], c["xadj"], c["adj"], c["ew"], c["vw"])


@pytest.mark.parametrize("L", [2, 5, 9, 16, 31])
def test_monotone_path_needs_half_length_rounds(L):
    g = path_graph(list(range(1, L + 1)))
    _, _, rounds, _, _ = O.match_rounds(g, O.EXPANSION_STAR2, 7)
    assert rounds == (L + 1) // 2


@pytest.mark.parametrize("seed", range(20))
def test_w3_triangle_hash_decides(seed):
    g = complete_graph(3)
    mate, m = O.match_greedy(g, O.EXPANSION_STAR2, O.level_seed(seed, 0))
    assert m == 1
    cmap, cg = O.contract(g, mate)
    assert cg.n == 2 and cg.ew.tolist() == [2, 2]          # parallel edges merged
    assert sorted(cg.vw.tolist()) == [1, 2]
    assert mate.tolist() == refpy.greedy(g, "expansion*2", O.level_seed(seed, 0))


@pytest.mark.parametrize("seed", range(20))
def test_w4_four_cycle_shape_is_hash_independent(seed):
    g = cycle_graph(4)
    mate, m = O.match_greedy(g, O.EXPANSION_STAR2, O.level_seed(seed, 0))
    assert m == 2
    cmap, cg = O.contract(g, mate)
    assert cg.n == 2 and cg.vw.tolist() == [2, 2] and cg.ew.tolist() == [2, 2]


def test_w5_star_stalls():
    g = star_graph(3)
    H = O.coarsen(g, O.EXPANSION_STAR2, seed=1, stop_n=1, stall_num=1, stall_den=20)
    ns = [lv.graph.n for lv in H.levels]
    assert ns[:3] == [4, 3, 2]
    assert H.levels[1].graph.vw.max() == 2
    # a big star: one leaf per level, so the stall rule ends the hierarchy
    g = star_graph(100)
    H = O.coarsen(g, O.EXPANSION_STAR2, seed=1, stop_n=5)
    assert [lv.graph.n for lv in H.levels] == [101, 100]
    assert H.stop_reason == O.STOP_STALL


def test_w6_greedy_half_approximation():
    w = gold("w6_p4.json")
    g = graph_from(w["graph"])
    mate, m = O.match_greedy(g, O.EXPANSION_STAR2, 3)
    assert mate.tolist() == w["greedy_mate"]
    num, den = O.rate(g, O.EXPANSION_STAR2)
    val = sum(Fraction(int(num[j]), int(den[j])) for v in range(g.n)
              for j in range(g.xadj[v], g.xadj[v + 1]) if mate[v] == g.adj[j] and v < g.adj[j])
    assert val == Fraction(*w["greedy_value"])
    best = max(sum(Fraction(e[2] ** 2) for e in M) for M in refpy.all_matchings(g.n, refpy.edges_of(g)))
    assert best == Fraction(*w["optimum_value"])
    assert 2 * val >= best


# --------------------------------------------------------------------------
# Matching on random small graphs: Greedy == rounds == pure-Python greedy,
# maximal, >= 1/2 optimum, certificate
# --------------------------------------------------------------------------
def _small_graphs():
    cases = []
    for s in range(24):
        n = 4 + s % 9
        m = min(n * (n - 1) // 2, 3 + (s * 7) % 16)
        wmax = [1, 3, 100][s % 3]
        cmax = [1, 4, 9][(s // 3) % 3]
        cmin = 0 if s % 5 == 0 else 1
        cases.append((s, random_graph(n, m, seed=1000 + s, wmax=wmax, cmax=cmax, cmin=cmin)))
    return cases


@pytest.mark.parametrize("rating", RATING_NAMES)
def test_greedy_equals_rounds_and_python(rating):
    for s, g in _small_graphs():
        seed = O.level_seed(s, 3)
        a, ma = O.match_greedy(g, O.RATINGS[rating], seed)
        b, mb, _, _, _ = O.match_rounds(g, O.RATINGS[rating], seed)
        assert np.array_equal(a, b) and ma == mb
        assert a.tolist() == refpy.greedy(g, rating, seed)
        assert O.greedy_certificate(g, O.RATINGS[rating], seed, a) == 0


@pytest.mark.parametrize("rating", RATING_NAMES)
def test_maximal_and_half_of_optimum(rating):
    for s, g in _small_graphs():
        es = refpy.edges_of(g)
        if len(es) > 16:
            continue
        seed = O.level_seed(s, 0)
        mate, _ = O.match_greedy(g, O.RATINGS[rating], seed)
        # a matching: symmetric, node disjoint, made of edges
        for v in range(g.n):
            if mate[v] >= 0:
                assert mate[mate[v]] == v
        # maximal: no edge with two free ends (Section 3.3: rounds go on while an edge can be matched)
        for a, b, _ in es:
            assert mate[a] >= 0 or mate[b] >= 0
        outs = refpy.out_of(g)
        vals = {(a, b): refpy.finite_value(rating, g, (a, b, w), outs) for a, b, w in es}
        if any(v is None for v in vals.values()):
            continue     # infinite ratings: the weight bound is meaningless
        got = sum(vals[(a, b)] for a, b, _ in es if mate[a] == b)
        best = max(sum(vals[(e[0], e[1])] for e in M) for M in refpy.all_matchings(g.n, es))
        assert 2 * got >= best


def test_half_of_optimum_networkx_medium():
    nx = pytest.importorskip("networkx")
    for s in range(6):
        g = random_graph(40, 90, seed=77 + s, wmax=20, cmax=5)
        num, den = O.rate(g, O.EXPANSION_STAR2)
        # integer-scaled ratings: exact for networkx's integer mode
        L = 1
        for d in set(int(x) for x in den):
            L = L * d // np.gcd(L, d)
        G = nx.Graph()
        vals = {}
        for v in range(g.n):
            for j in range(g.xadj[v], g.xadj[v + 1]):
                u = int(g.adj[j])
                if u > v:
                    vals[(v, u)] = int(num[j]) * (L // int(den[j]))
                    G.add_edge(v, u, weight=vals[(v, u)])
        opt = nx.max_weight_matching(G)
        best = sum(vals[(min(a, b), max(a, b))] for a, b in opt)
        mate, _ = O.match_greedy(g, O.EXPANSION_STAR2, 5)
        got = sum(vals[(v, int(mate[v]))] for v in range(g.n) if mate[v] > v)
        assert 2 * got >= best


def test_certificate_detects_wrong_matchings():
    g = random_graph(30, 70, seed=5, wmax=9, cmax=3)
    seed = 11
    mate, _ = O.match_greedy(g, O.EXPANSION_STAR2, seed)
    assert O.greedy_certificate(g, O.EXPANSION_STAR2, seed, mate) == 0
    # another seed gives another valid maximal matching, not this greedy one
    other, _ = O.match_greedy(g, O.EXPANSION_STAR2, seed + 1)
    if not np.array_equal(other, mate):
        assert O.greedy_certificate(g, O.EXPANSION_STAR2, seed, other) > 0
    # drop one matched pair: not maximal any more
    bad = mate.copy()
    v = int(np.flatnonzero(bad >= 0)[0])
    bad[bad[v]] = -1
    bad[v] = -1
    assert O.greedy_certificate(g, O.EXPANSION_STAR2, seed, bad) > 0
    # a non-symmetric mate array
    bad = mate.copy()
    bad[v] = (bad[v] + 1) % g.n
    assert O.greedy_certificate(g, O.EXPANSION_STAR2, seed, bad) > 0


# --------------------------------------------------------------------------
# Contraction: definition written with dicts, invariants
# --------------------------------------------------------------------------
def test_contract_matches_dict_definition_and_invariants():
    for s, g in _small_graphs() + [(99, grid2d(7, 9)), (98, random_graph(200, 700, 9, wmax=50, cmax=7))]:
        mate, m = O.match_greedy(g, O.EXPANSION_STAR2, O.level_seed(s, 1))
        cmap, cg = O.contract(g, mate)
        rc, nc, xadj, adj, ew, cvw = refpy.contract_dict(g, mate.tolist())
        assert cmap.tolist() == rc and cg.n == nc
        assert cg.xadj.tolist() == xadj and cg.adj.tolist() == adj and cg.ew.tolist() == ew
        assert cg.vw.tolist() == cvw
        # c(V) preserved, w(E') = w(E) - w(M)
        assert int(cg.vw.sum()) == int(g.vw.sum())
        wM = sum(w for a, b, w in refpy.edges_of(g) if mate[a] == b)
        assert int(cg.ew.sum()) // 2 == int(g.ew.sum()) // 2 - wM
        assert cg.n == g.n - m
        assert O.validate(cg) == O.OK


# --------------------------------------------------------------------------
# Cut / balance: closed forms on the 64x64 grid, projection invariance
# --------------------------------------------------------------------------
def test_cut_closed_forms_on_grid():
    g = grid2d(64, 64)
    ids = np.arange(4096)
    col, row = ids % 64, ids // 64
    halves = (col >= 32).astype(np.int32)
    r = O.cut_balance(g, halves, 2, 3, 100)
    assert r.cut == 64 and r.block_w.tolist() == [2048, 2048] and r.feasible
    checker = ((row + col) % 2).astype(np.int32)
    assert O.cut_balance(g, checker, 2, 3, 100).cut == 8064
    one = np.zeros(4096, dtype=np.int32)
    r = O.cut_balance(g, one, 2, 3, 100)
    assert r.cut == 0 and r.block_w.tolist() == [4096, 0] and not r.feasible
    # L_max on the 64x64 grid, k=2, eps=3%: 1.03 * 4096 / 2 + 1 = 2110.44
    assert Fraction(r.lmax_num, r.lmax_den) == Fraction(211044, 100)
    assert r.imb_num == 200 * 4096 - 422088
    quarters = (2 * (row >= 32) + (col >= 32)).astype(np.int32)
    r = O.cut_balance(g, quarters, 4, 3, 100)
    assert r.cut == 128 and r.block_w.tolist() == [1024] * 4
    assert (r.bal_num, r.bal_den) == (4 * 1024, 4096)


def test_projection_preserves_cut_and_blocks():
    g = random_graph(3000, 9000, seed=3, wmax=7, cmax=3)
    H = O.coarsen(g, O.INNER_OUTER, seed=9, stop_n=40)
    assert len(H.levels) > 3
    parts, res = O.uncoarsen(H, 8, part_seed=1)
    for l in range(len(H.levels) - 1):
        assert res[l].cut == res[l + 1].cut
        assert res[l].block_w.tolist() == res[l + 1].block_w.tolist()
    # direct recount of the level-0 cut from the edge list
    cut = sum(w for a, b, w in refpy.edges_of(g) if parts[0][a] != parts[0][b])
    assert cut == res[0].cut


def test_cut_balance_argument_errors():
    g = grid2d(3, 3)
    p = np.zeros(9, dtype=np.int32)
    assert O.cut_balance_status(g, p, 0, 3, 100) == O.E_ARG
    assert O.cut_balance_status(g, p, 4097, 3, 100) == O.E_ARG
    assert O.cut_balance_status(g, p, 2, 3, 0) == O.E_ARG
    p[3] = 2
    assert O.cut_balance_status(g, p, 2, 3, 100) == O.E_RANGE


# --------------------------------------------------------------------------
# Validation codes on hand-made malformed inputs
# --------------------------------------------------------------------------
def _mk(xadj, adj, ew, vw):
    class G:
        pass
    G.n = len(xadj) - 1
    G.xadj = np.array(xadj, dtype=np.int64)
    G.adj = np.array(adj, dtype=np.int32)
    G.ew = np.array(ew, dtype=np.uint32)
    G.vw = np.array(vw, dtype=np.uint32)
    return G


def test_validate_codes():
    ok = _mk([0, 1, 3, 4], [1, 0, 2, 1], [2, 2, 5, 5], [1, 1, 1])
    assert O.validate(ok) == O.OK
    assert O.validate(_mk([0, 1, 3, 4], [1, 0, 2, 0], [2, 2, 5, 5], [1, 1, 1])) == O.E_GRAPH   # asymmetric
    assert O.validate(_mk([0, 1, 3, 4], [1, 0, 2, 1], [2, 2, 5, 4], [1, 1, 1])) == O.E_GRAPH   # weight mismatch
    assert O.validate(_mk([0, 1, 3, 4], [1, 2, 0, 1], [2, 5, 2, 5], [1, 1, 1])) == O.E_GRAPH   # row not ascending
    assert O.validate(_mk([0, 2, 3, 3], [0, 1, 0], [1, 1, 1], [1, 1, 1])) == O.E_GRAPH         # self loop
    assert O.validate(_mk([0, 1, 2, 2], [5, 0], [1, 1], [1, 1, 1])) == O.E_GRAPH               # out of range
    assert O.validate(_mk([0, 2, 1, 2], [1, 1], [1, 1], [1, 1, 1])) == O.E_GRAPH               # offsets decrease
    assert O.validate(_mk([0, 1, 3, 4], [1, 0, 2, 1], [0, 0, 5, 5], [1, 1, 1])) == O.E_RANGE   # w = 0
    big = 0xFFFFFFFF
    assert O.validate(_mk([0, 1, 3, 4], [1, 0, 2, 1], [big, big, 1, 1], [1, 1, 1])) == O.E_RANGE  # sum w
    assert O.validate(_mk([0, 1, 2], [1, 0], [1, 1], [big, 1])) == O.E_RANGE                  # sum c
    assert O.validate(_mk([0, 1, 2], [1, 0], [big, big], [0, 0])) == O.OK                     # sum w = 2^32-1
    assert O.validate(_mk([0], [], [], [])) == O.OK                                           # empty graph


# --------------------------------------------------------------------------
# Multilevel loop: stop rules, C1 shape
# --------------------------------------------------------------------------
def test_stop_rules():
    g = grid2d(8, 8)
    H = O.coarsen(g, O.EXPANSION_STAR2, seed=42, stop_n=64)
    assert len(H.levels) == 1 and H.stop_reason == O.STOP_SIZE
    H = O.coarsen(g, O.EXPANSION_STAR2, seed=42, stop_n=1, max_levels=2)
    assert len(H.levels) == 3 and H.stop_reason == O.STOP_MAXLEVEL
    e = csr_from_edges(10, np.zeros(0), np.zeros(0))
    H = O.coarsen(e, O.EXPANSION_STAR2, seed=42, stop_n=1)
    assert len(H.levels) == 1 and H.stop_reason == O.STOP_EMPTY


def test_c1_grid_hierarchy_invariants():
    g = grid2d(64, 64)
    assert (g.n, g.m) == (4096, 8064)
    H = O.coarsen(g, O.EXPANSION_STAR2, seed=42, stop_n=256, cross_check=True)
    assert H.levels[-1].graph.n <= 256 < H.levels[-2].graph.n
    assert H.stop_reason == O.STOP_SIZE
    for l in range(len(H.levels) - 1):
        G, C, lv = H.levels[l].graph, H.levels[l + 1].graph, H.levels[l]
        assert int(C.vw.sum()) == 4096
        wM = sum(int(G.ew[j]) for v in range(G.n) for j in range(G.xadj[v], G.xadj[v + 1])
                 if lv.mate[v] == G.adj[j] and v < G.adj[j])
        assert int(C.ew.sum()) // 2 == int(G.ew.sum()) // 2 - wM
        assert O.greedy_certificate(G, O.EXPANSION_STAR2, O.level_seed(42, l), lv.mate) == 0


# --------------------------------------------------------------------------
# the two-phase matcher of Section 3.3
# --------------------------------------------------------------------------
def test_w7_two_phase_hand_worked():
    w = gold("w7_two_phase.json")
    for name in ("p5", "six"):
        c = w[name]
        g = graph_from(c["graph"])
        mate, m, loc, ge, gm = O.match_two_phase(g, O.EXPANSION_STAR2, O.level_seed(42, 0),
                                                 c["block_bits"])
        assert loc.tolist() == c["block_matching"], name
        assert ge == len(c["gap_edges"]), name
        assert mate.tolist() == c["mate"], name
        assert m == sum(1 for v, u in enumerate(c["mate"]) if u > v)
        if "gap_matched" in c:
            assert gm == c["gap_matched"]
    c = w["p5"]
    g = graph_from(c["graph"])
    gmate, _ = O.match_greedy(g, O.EXPANSION_STAR2, O.level_seed(42, 0))
    assert gmate.tolist() == c["greedy_mate"] != c["mate"]   # the two schemes differ here
    cmap, cg = O.contract(g, np.array(c["mate"], dtype=np.int32))
    assert cmap.tolist() == c["cmap"]
    k = c["coarse"]
    assert (cg.n, cg.xadj.tolist(), cg.adj.tolist(), cg.ew.tolist(), cg.vw.tolist()) == \
        (k["n"], k["xadj"], k["adj"], k["ew"], k["vw"])


@pytest.mark.parametrize("seed", range(20))
def test_two_phase_equal_ratings_follow_the_hash(seed):
    # P4 with unit weights, blocks {0,1} {2,3}: all three edges rate 1, so the
    # cross edge {1,2} enters the gap graph iff its hash beats both block edges
    g = path_graph([1, 1, 1])
    s = O.level_seed(seed, 0)
    mate, m, loc, ge, gm = O.match_two_phase(g, O.EXPANSION_STAR2, s, 1)
    assert loc.tolist() == [1, 0, 3, 2]
    h = lambda a, b: refpy.mix64(s ^ ((a << 32) | b))
    in_gap = h(1, 2) > h(0, 1) and h(1, 2) > h(2, 3)
    assert ge == int(in_gap)
    assert mate.tolist() == ([-1, 2, 1, -1] if in_gap else [1, 0, 3, 2])


@pytest.mark.parametrize("rating", RATING_NAMES)
def test_two_phase_one_block_and_singletons_are_greedy(rating):
    # one block: no gap edge, the block matcher is Greedy on G; blocks of one
    # node: no block edge, every edge is a gap edge, Greedy on G again
    for s, g in _small_graphs():
        seed = O.level_seed(s, 1)
        ref, mr = O.match_greedy(g, O.RATINGS[rating], seed)
        for bb in (0, 31, max(1, int(np.ceil(np.log2(max(g.n, 2)))))):
            mate, m, loc, ge, gm = O.match_two_phase(g, O.RATINGS[rating], seed, bb)
            assert np.array_equal(mate, ref) and m == mr, (s, bb)
            assert (ge == 0) if bb else (loc == -1).all()


def test_two_phase_light_cross_edges_give_greedy():
    # weight rating, every block edge heavier than every cross edge: Greedy
    # takes the block edges first (blocks do not interact) and then cross
    # edges between nodes the blocks left free -- exactly the gap graph
    rng = np.random.default_rng(5)
    for t in range(30):
        n, bb = int(rng.integers(8, 200)), int(rng.integers(1, 5))
        g0 = random_graph(n, int(rng.integers(n, 4 * n)), seed=300 + t, wmax=1)
        a = np.repeat(np.arange(n), np.diff(g0.xadj))
        keep = a < g0.adj
        a, b = a[keep], g0.adj[keep].astype(np.int64)
        inner = (a >> bb) == (b >> bb)
        w = np.where(inner, rng.integers(1001, 2000, len(a)), rng.integers(1, 1000, len(a)))
        g = csr_from_edges(n, a, b, w.astype(np.uint32))
        seed = O.level_seed(t, 0)
        mate = O.match_two_phase(g, O.WEIGHT, seed, bb)[0]
        assert np.array_equal(mate, O.match_greedy(g, O.WEIGHT, seed)[0]), t


@pytest.mark.parametrize("rating", RATING_NAMES)
def test_two_phase_equals_round_form(rating):
    # the oracle (sorted Greedy per phase) against the round form of both
    # phases written independently in Python, on many block sizes
    for s, g in _small_graphs():
        seed = O.level_seed(s, 2)
        for bb in (1, 2, 3, 5):
            mate = O.match_two_phase(g, O.RATINGS[rating], seed, bb)[0]
            assert mate.tolist() == refpy.two_phase_rounds(g, rating, seed, bb), (s, bb)


def test_two_phase_structure():
    # a matching of graph edges; matched cross edges were gap edges; matched
    # block edges come from the block matching; every node the block matching
    # paired is still paired unless its partner took a cross edge
    for s, g in _small_graphs():
        for bb in (1, 2, 4):
            seed = O.level_seed(s, 0)
            mate, m, loc, ge, gm = O.match_two_phase(g, O.EXPANSION_STAR2, seed, bb)
            es = {(a, b) for a, b, _ in refpy.edges_of(g)}
            cross = 0
            for v, u in enumerate(mate.tolist()):
                if u < 0:
                    assert loc[v] < 0 or mate[loc[v]] >= 0 and mate[loc[v]] != v
                    continue
                assert mate[u] == v and (min(u, v), max(u, v)) in es
                if (u >> bb) != (v >> bb):
                    cross += u > v
                else:
                    assert loc[v] == u
            assert cross == gm and gm <= ge


@pytest.mark.parametrize("rating", ["expansion*2", "innerOuter"])
def test_two_phase_hierarchy_invariants(rating):
    g = grid2d(40, 40)
    H = O.coarsen(g, O.RATINGS[rating], 42, 64, block_bits=5)
    assert H.stop_reason in (O.STOP_SIZE, O.STOP_STALL, O.STOP_EMPTY)
    total = int(g.vw.sum())
    for l, lv in enumerate(H.levels[:-1]):
        nxt = H.levels[l + 1].graph
        assert nxt.n == lv.graph.n - lv.matched
        assert int(nxt.vw.sum()) == total
        assert O.validate(nxt) == O.OK
        s = O.level_seed(42, l)
        assert np.array_equal(lv.mate, O.match_two_phase(lv.graph, O.RATINGS[rating], s, 5)[0])
