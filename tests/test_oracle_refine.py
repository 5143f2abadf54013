"""Pins of the oracle's pairwise refinement (Section 5): hand-worked local
searches, the quotient graph and its greedy edge colouring (Section 5.1),
the rollback against a replay of the moves with cuts computed from scratch,
a second writing of the local search on tiny graphs, and the invariants of
whole refinements."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from refpy import fm_pair_ref
from workloads import csr_from_edges, grid2d, random_graph, rgg


def two_triangles():
    # triangles {0,1,2} and {3,4,5} joined by the edge {2,3}, unit weights
    return csr_from_edges(6, np.array([0, 0, 1, 2, 3, 3, 4]), np.array([1, 2, 2, 3, 4, 5, 5]))


def test_two_triangles_hand_worked():
    # nodes 2 and 3 start on the wrong sides: cut 5.  Both have gain 3; either
    # order ends at the two triangles (cut 1) after two moves, the third move
    # (gain -2) breaks the patience of alpha = 1/20 and is rolled back.
    g = two_triangles()
    part = np.array([0, 0, 1, 0, 1, 1], np.int32)
    for seed in range(8):
        moves, r = O.fm_pair(g, part, 2, 0, 1, seed, alpha_num=1, alpha_den=20)
        assert sorted(moves[:2].tolist()) == [2, 3]
        assert r["start"] == (0, 5) and r["end"] == (0, 1) and r["kept"] == 2 and r["made"] == 3
    out, st = O.refine(g, part, 2)
    assert out.tolist() == [0, 0, 0, 1, 1, 1]
    # global iteration 0: one adoption, then a local iteration without change;
    # global iteration 1 changes nothing and ends it: 3 local iterations x 2 runs
    assert (st["global_iterations"], st["searches"], st["adoptions"], st["kept"]) == (2, 6, 1, 2)


def maxload_graph():
    # block A = {0,1,2,3}, B = {4}; w(4,0) = w(4,1) = 5, the path 0-1-2-3 weighs 1
    return csr_from_edges(5, np.array([4, 4, 0, 1, 2]), np.array([0, 1, 1, 2, 3]),
                          w=np.array([5, 5, 1, 1, 1]))


def test_maxload_exception_hand_worked():
    # eps = 0, k = 2: L_max = 5/2 + 1 = 3.5, so A (weight 4) is overloaded.
    # TopGain alone would move node 4 (gain 10); MaxLoad makes A give node 0
    # (gain 4): cut 6, balanced.  Then TopGain: node 1 (gain 5) -> cut 1;
    # node 2 (gain 0) overloads B and is rolled back.
    g = maxload_graph()
    part = np.array([0, 0, 0, 0, 1], np.int32)
    moves, r = O.fm_pair(g, part, 2, 0, 1, 7, alpha_num=1, alpha_den=20, eps_num=0, eps_den=1)
    assert moves.tolist() == [0, 1, 2]
    assert r["start"] == (1, 10) and r["end"] == (0, 1) and r["kept"] == 2
    # with eps = 1 nothing is overloaded (L_max = 6): TopGain moves node 4 first, cut 0
    moves, r = O.fm_pair(g, part, 2, 0, 1, 7, alpha_num=1, alpha_den=20, eps_num=1, eps_den=1)
    assert moves[0] == 4 and r["end"] == (0, 0) and r["kept"] == 1


def test_depth_bounds_the_search_area():
    # a path 0..9, A = 0..4, B = 5..9: only 4 and 5 are on the boundary; with
    # depth 0 nothing else ever enters a queue
    g = csr_from_edges(10, np.arange(9), np.arange(1, 10))
    part = np.array([0] * 5 + [1] * 5, np.int32)
    for depth, limit in ((0, {4, 5}), (2, {2, 3, 4, 5, 6, 7})):
        moves, r = O.fm_pair(g, part, 2, 0, 1, 3, alpha_num=100, alpha_den=1, depth=depth,
                             eps_num=100, eps_den=1)
        assert set(moves.tolist()) <= limit and set(moves.tolist()) == limit, depth


def partitions():
    out = []
    for s, g in enumerate([grid2d(12, 14), random_graph(300, 1200, seed=4, wmax=9, cmax=5, cmin=0),
                           rgg(2000, seed=5)]):
        for k in (2, 5, 16):
            rng = np.random.default_rng(10 * s + k)
            out.append((g, k, rng.integers(0, k, g.n).astype(np.int32)))
    return out


def test_quotient_colouring_properties():
    for g, k, part in partitions():
        pairs, col, nc = O.quotient_colouring(g, part, k)
        src = np.repeat(np.arange(g.n), np.diff(g.xadj))
        pa, pb = part[src], part[g.adj]
        want = sorted({(int(x), int(y)) for x, y in zip(pa, pb) if x < y})
        assert [tuple(p) for p in pairs.tolist()] == want
        deg = np.zeros(k, int)
        for a, b in want:
            deg[a] += 1
            deg[b] += 1
        assert nc == (col.max() + 1 if len(col) else 0) and nc <= max(1, 2 * deg.max() - 1)
        seen = {}
        for (a, b), c in zip(want, col.tolist()):
            # proper, and every smaller colour is taken at an end by an earlier pair
            assert c not in seen.get(a, set()) and c not in seen.get(b, set())
            assert all(x in seen.get(a, set()) | seen.get(b, set()) for x in range(c))
            seen.setdefault(a, set()).add(c)
            seen.setdefault(b, set()).add(c)


def pair_state(g, part, k, a, b, eps):
    """(scaled imbalance of the pair, cut between a and b) from scratch."""
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    sel = (part[src] == a) & (part[g.adj] == b)
    cut = int(g.ew[sel].sum())
    vw = g.vw.astype(np.int64)
    S = k * eps.denominator
    L = (eps.denominator + eps.numerator) * int(vw.sum()) + S * int(vw.max())
    wa, wb = int(vw[part == a].sum()), int(vw[part == b].sum())
    return max(0, S * max(wa, wb) - L), cut


def test_rollback_keeps_the_best_prefix():
    eps = Fraction(3, 100)
    for g, k, part in partitions():
        pairs, _, _ = O.quotient_colouring(g, part, k)
        for a, b in pairs[:: max(1, len(pairs) // 6)].tolist():
            for alpha in ((1, 100), (20, 100), (3, 1)):
                moves, r = O.fm_pair(g, part, k, a, b, 99, alpha[0], alpha[1], depth=3)
                assert len(set(moves.tolist())) == len(moves)
                assert all(part[v] in (a, b) for v in moves)
                p = part.copy()
                states = [pair_state(g, p, k, a, b, eps)]
                for v in moves:
                    p[v] = b if p[v] == a else a
                    states.append(pair_state(g, p, k, a, b, eps))
                assert states[0] == r["start"] and states[r["kept"]] == r["end"]
                assert r["kept"] == min(range(len(states)), key=lambda i: (states[i], i))
                size = min(int((part == a).sum()), int((part == b).sum()))
                assert r["made"] - r["kept"] <= alpha[0] * size // alpha[1] + 1


@pytest.mark.parametrize("case", range(24))
def test_local_search_equals_second_writing(case):
    rng = np.random.default_rng(case)
    n = 8 + case % 13
    g = random_graph(n, min(n * (n - 1) // 2, 2 * n + case), seed=300 + case, wmax=[1, 4, 20][case % 3],
                     cmax=[1, 3][case % 2], cmin=case % 3 == 0 and 0 or 1)
    k = 2 + case % 3
    part = rng.integers(0, k, n).astype(np.int32)
    eps = Fraction([3, 0, 50][case % 3], 100)
    for a, b in O.quotient_colouring(g, part, k)[0].tolist()[:3]:
        for depth in (0, 1, 4):
            for alpha in (Fraction(1, 20), Fraction(1, 2)):
                seed = O.run_seed(case, 0, a, b, depth, 0)
                moves, r = O.fm_pair(g, part, k, a, b, seed, alpha.numerator, alpha.denominator,
                                     depth, eps.numerator, eps.denominator)
                ref, kept = fm_pair_ref(g, part, k, a, b, seed, alpha, depth, eps)
                assert moves.tolist() == ref and r["kept"] == kept, (a, b, depth, alpha)


def test_refine_invariants():
    for g, k, part in partitions():
        for name in ("minimal", "fast", "strong"):
            prm = O.RefineParams.preset(name)
            out, st = O.refine(g, part, k, params=prm)
            before, after = O.cut_balance(g, part, k), O.cut_balance(g, out, k)
            assert (after.imb_num, after.cut) <= (before.imb_num, before.cut)
            assert after.total == before.total and ((out >= 0) & (out < k)).all()
            assert st["global_iterations"] <= prm.max_global
            assert st["kept"] <= st["moves"] and st["searches"] % 2 == 0
            if st["adoptions"] == 0:
                assert (out == part).all()
            # a second refinement from the result with the same seed keeps improving
            # or stays: never worse
            out2, _ = O.refine(g, out, k, params=prm)
            a2 = O.cut_balance(g, out2, k)
            assert (a2.imb_num, a2.cut) <= (after.imb_num, after.cut)


def test_refine_degenerate_cases():
    g = grid2d(6, 6)
    one = np.zeros(36, np.int32)
    out, st = O.refine(g, one, 1)
    assert (out == one).all() and st["searches"] == 0 and st["global_iterations"] == 1
    empty = csr_from_edges(0, np.zeros(0, np.int64), np.zeros(0, np.int64))
    out, st = O.refine(empty, np.zeros(0, np.int32), 4)
    assert len(out) == 0 and st["searches"] == 0
    # two grids' halves: the straight cut is optimal for a 2 x 2m grid split in halves
    g = grid2d(2, 10)
    part = (np.arange(20) % 10 >= 5).astype(np.int32)
    out, st = O.refine(g, part, 2)
    assert O.cut_balance(g, out, 2).cut == 2
    with pytest.raises(ValueError):
        O.refine(g, part, 300)
    with pytest.raises(ValueError):
        O.refine(g, part + 5, 2)


def test_refined_uncoarsening_improves_every_level():
    g = rgg(1 << 12, seed=3)
    H = O.coarsen(g, O.EXPANSION_STAR2, 42, 20 * 8)
    plain_parts, plain = O.uncoarsen(H, 8)
    parts, res, stats = O.uncoarsen_refined(H, 8)
    # the coarsest level starts from the same partition; refinement never worsens it
    assert (res[-1].imb_num, res[-1].cut) <= (plain[-1].imb_num, plain[-1].cut)
    assert res[0].cut < plain[0].cut // 3 and res[0].feasible
    assert all(s["global_iterations"] >= 1 for s in stats)
