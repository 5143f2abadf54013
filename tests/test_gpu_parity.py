"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact everywhere: the path is integer / exact-rational arithmetic only,
so every output (ratings, mate, rounds, coarse CSR, cmap, partitions, cut and
balance) must equal the oracle's.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import rgg_rcb, assert_graph_equal, check_hierarchy, dev, graph_np
from workloads import (complete_graph, csr_from_edges, cycle_graph, grid2d, path_graph,
                       random_graph, rgg, rmat, star_graph)

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
RATINGS = [0, 1, 2, 3, 4]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    K.lib()
    yield
    torch.cuda.synchronize()


def small_cases():
    cases = [("P2", path_graph([5])), ("W1", path_graph([3, 4, 2])), ("W2", path_graph([1, 2, 3, 4])),
             ("W6", path_graph([3, 4, 3])), ("tri", complete_graph(3)), ("C4", cycle_graph(4)),
             ("K1_3", star_graph(3)), ("K8", complete_graph(8)), ("grid5x7", grid2d(5, 7))]
    for s in range(16):
        n = 5 + (s * 13) % 60
        m = min(n * (n - 1) // 2, n + (s * 37) % (3 * n))
        cases.append((f"rnd{s}", random_graph(n, m, seed=500 + s, wmax=[1, 5, 1000][s % 3],
                                              cmax=[1, 3, 50][(s // 3) % 3], cmin=0 if s % 4 == 0 else 1)))
    return cases


# --------------------------------------------------------------------------
def test_validate_matches_oracle_codes():
    from test_oracle_pins import _mk
    big = 0xFFFFFFFF
    cases = [
        _mk([0, 1, 3, 4], [1, 0, 2, 1], [2, 2, 5, 5], [1, 1, 1]),
        _mk([0, 1, 3, 4], [1, 0, 2, 0], [2, 2, 5, 5], [1, 1, 1]),
        _mk([0, 1, 3, 4], [1, 0, 2, 1], [2, 2, 5, 4], [1, 1, 1]),
        _mk([0, 1, 3, 4], [1, 2, 0, 1], [2, 5, 2, 5], [1, 1, 1]),
        _mk([0, 2, 3, 3], [0, 1, 0], [1, 1, 1], [1, 1, 1]),
        _mk([0, 1, 2, 2], [5, 0], [1, 1], [1, 1, 1]),
        _mk([0, 2, 1, 2], [1, 1], [1, 1], [1, 1, 1]),
        _mk([0, 1, 3, 4], [1, 0, 2, 1], [0, 0, 5, 5], [1, 1, 1]),
        _mk([0, 1, 3, 4], [1, 0, 2, 1], [big, big, 1, 1], [1, 1, 1]),
        _mk([0, 1, 2], [1, 0], [1, 1], [big, 1]),
        _mk([0, 1, 2], [1, 0], [big, big], [0, 0]),
        _mk([0], [], [], []),
        _mk([0, 0, 0], [], [], [4, 5]),
    ]
    for i, g in enumerate(cases):
        want = O.validate(g)
        got = K.kappa_validate(dev(g))
        assert got == want, f"case {i}: {got} != {want}"
    # larger graphs
    for g in [grid2d(64, 64), rmat(12, 16, seed=1, wseed=2), random_graph(3000, 9000, 4, wmax=9)]:
        assert K.kappa_validate(dev(g)) == O.OK
    # break symmetry in a large graph: one weight changed
    g = random_graph(5000, 20000, 7, wmax=9)
    g.ew[12345] += 1
    assert K.kappa_validate(dev(g)) == O.E_GRAPH == O.validate(g)


@pytest.mark.parametrize("rating", RATINGS)
def test_rate_bit_exact(rating):
    for name, g in small_cases() + [("rmat12", rmat(12, 8, seed=5, wseed=6))]:
        num, den = K.kappa_rate(dev(g), rating)
        onum, oden = O.rate(g, rating)
        assert np.array_equal(num.cpu().numpy().view(np.uint64), onum), name
        assert np.array_equal(den.cpu().numpy().view(np.uint64), oden), name


@pytest.mark.parametrize("rating", RATINGS)
def test_match_bit_exact_small(rating):
    for name, g in small_cases():
        for s in (1, 99):
            seed = O.level_seed(s, 0)
            mate, rounds, matched = K.kappa_match(dev(g), rating, seed)
            omate, om_m, o_rounds, _, _ = O.match_rounds(g, rating, seed)
            gm, _ = O.match_greedy(g, rating, seed)
            assert np.array_equal(omate, gm)
            assert np.array_equal(mate.cpu().numpy(), omate), f"{name} seed {s}"
            assert rounds == o_rounds and matched == om_m, f"{name}: rounds {rounds} vs {o_rounds}"


def test_contract_bit_exact_small():
    for name, g in small_cases():
        omate, _ = O.match_greedy(g, 0, 17)
        ocmap, og = O.contract(g, omate)
        import torch
        cmap, cg = K.kappa_contract(dev(g), torch.from_numpy(omate).cuda())
        assert np.array_equal(cmap.cpu().numpy(), ocmap), name
        assert_graph_equal(graph_np(cg), og, name)


def test_contract_rejects_bad_matchings_and_small_capacity():
    import torch
    g = grid2d(6, 6)
    mate, _ = O.match_greedy(g, 0, 3)
    bad = mate.copy()
    v = int(np.flatnonzero(bad >= 0)[0])
    bad[v] = (bad[v] + 7) % g.n          # not symmetric / not an edge
    with pytest.raises(K.KappaError) as e:
        K.kappa_contract(dev(g), torch.from_numpy(bad).cuda())
    assert e.value.status == K.E_ARG
    with pytest.raises(K.KappaError) as e:
        K.kappa_contract(dev(g), torch.from_numpy(mate).cuda(), cap_n=3)
    assert e.value.status == K.E_CAPACITY


@pytest.mark.parametrize("rating", [0, 1])
def test_w1_hierarchy(rating):
    with open(os.path.join(GOLD, "w1_p4.json")) as f:
        w = json.load(f)
    g = path_graph([3, 4, 2])
    H, OH = check_hierarchy(g, rating, 42, stop_n=1, k=2)
    for l, want in enumerate(w["levels"]):
        lv = H.level(l)
        assert lv.graph.xadj.cpu().tolist() == want["xadj"]
        assert lv.graph.adj.cpu().tolist() == want["adj"]


@pytest.mark.parametrize("rating", RATINGS)
def test_hierarchy_small_graphs(rating):
    for name, g in small_cases():
        say("case", name, rating)
        check_hierarchy(g, rating, 7, stop_n=2, k=3)


def test_c1_grid_64x64():
    """64x64 grid, unit weights, expansion*2, seed 42, stop at 256, k=2."""
    g = grid2d(64, 64)
    H, OH = check_hierarchy(g, 0, 42, stop_n=256, k=2)
    assert H.level(len(H) - 1).graph.n <= 256
    assert H.info(len(H) - 1).stop_reason == K.STOP_SIZE


@pytest.mark.parametrize("rating", RATINGS)
def test_medium_rgg_and_rmat(rating):
    say("rgg 2^15", rating)
    check_hierarchy(rgg(1 << 15, seed=11), rating, 3, stop_n=20 * 16, k=16)
    say("rmat 13", rating)
    check_hierarchy(rmat(13, 16, seed=12, wseed=13), rating, 4, stop_n=20 * 64, k=64)


@pytest.mark.parametrize("rating", [0, 1])
def test_rgg_in_rcb_order(rating):
    # node ids in recursive coordinate bisection order (the locality a
    # geometric prepartition gives): the same kernels, the same oracle
    say("rgg 2^17 rcb order", rating)
    check_hierarchy(rgg_rcb(1 << 17, 21), rating, 42, stop_n=20 * 64, k=64)


def test_hub_rows_and_degree_classes():
    """Stars and cliques exercise the one-block pick (deg > 1024) and the mid
    and large coarse-row classes (bounds above 64 and above 4094)."""
    # star with 6000 leaves: hub degree 6000 (block pick, large coarse row)
    check_hierarchy(star_graph(6000), 0, 1, stop_n=2, k=2)
    # clique of 300 (mid rows), weighted
    rng = np.random.default_rng(5)
    k300 = complete_graph(300, w=rng.integers(1, 50, size=300 * 299 // 2))
    check_hierarchy(k300, 0, 2, stop_n=2, k=4)
    check_hierarchy(k300, 1, 2, stop_n=2, k=4)
    # two hubs joined to many common leaves: merged rows of two hubs
    a = np.concatenate([np.zeros(5000, np.int64), np.ones(5000, np.int64), [0]])
    b = np.concatenate([np.arange(2, 5002), np.arange(2, 5002), [1]])
    g = csr_from_edges(5002, a, b, np.arange(1, 10002, dtype=np.uint32) % 97 + 1)
    check_hierarchy(g, 0, 3, stop_n=2, k=2)
    check_hierarchy(g, 1, 3, stop_n=2, k=2)
    # rmat with big hubs (scale 16): bin-2 picks, large rows
    check_hierarchy(rmat(16, 16, seed=21, wseed=22), 0, 5, stop_n=20 * 256, k=256)


def test_edge_cases():
    # empty graph, isolated nodes only, one edge, zero node weights (infinite ratings)
    e = csr_from_edges(0, np.zeros(0), np.zeros(0))
    H = K.kappa_coarsen(dev(e), 0, 1, 0)
    assert len(H) == 1 and H.info(0).stop_reason == K.STOP_SIZE
    iso = csr_from_edges(50, np.zeros(0), np.zeros(0))
    check_hierarchy(iso, 0, 1, stop_n=1, k=2)
    check_hierarchy(path_graph([7]), 0, 1, stop_n=1, k=2)
    g = random_graph(400, 1500, seed=9, wmax=30, cmax=3, cmin=0)
    g.vw[:] = 0
    for r in RATINGS:
        check_hierarchy(g, r, 5, stop_n=4, k=5)
    # weights at the top of the range: sum w(E) = 2^32 - 1
    big = path_graph([2**31 - 1, 2**31])
    assert O.validate(big) == O.OK
    check_hierarchy(big, 0, 1, stop_n=1, k=2)
    check_hierarchy(big, 1, 1, stop_n=1, k=2)
    # max-level and no-stall settings
    check_hierarchy(grid2d(30, 30), 0, 1, stop_n=1, stall=(0, 1), max_levels=3, k=2)
    check_hierarchy(grid2d(30, 30), 0, 1, stop_n=1, stall=(0, 1), max_levels=0, k=2)


def test_project_and_cut_balance_standalone():
    import torch
    g = rgg(20000, seed=3)
    mate, _ = O.match_greedy(g, 0, 1)
    cmap, cg = O.contract(g, mate)
    for k in (1, 2, 7, 64, 4096):
        pc = O.initial_partition(cg.n, k, 9)
        got = K.kappa_initial_partition(cg.n, k, 9)
        assert np.array_equal(got.cpu().numpy(), pc)
        pf = K.kappa_project(torch.from_numpy(cmap).cuda(), cg.n, got)
        opf = O.project(cmap, pc)
        assert np.array_equal(pf.cpu().numpy(), opf)
        for eps in ((3, 100), (0, 1), (1, 1000000), (16000000, 1000000)):
            res, bw = K.kappa_cut_balance(dev(g), pf, k, *eps)
            ores = O.cut_balance(g, opf, k, *eps)
            assert res.as_tuple() == ores.as_tuple(), (k, eps)
            assert np.array_equal(bw.cpu().numpy().view(np.uint64), ores.block_w)
    # out-of-range map entry and block id
    bad = torch.from_numpy(cmap).cuda().clone()
    bad[5] = cg.n
    with pytest.raises(K.KappaError) as e:
        K.kappa_project(bad, cg.n, K.kappa_initial_partition(cg.n, 2, 1))
    assert e.value.status == K.E_RANGE
    p = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    p[17] = 2
    with pytest.raises(K.KappaError) as e:
        K.kappa_cut_balance(dev(g), p, 2)
    assert e.value.status == K.E_RANGE
    with pytest.raises(K.KappaError) as e:
        K.kappa_cut_balance(dev(g), p, 0)
    assert e.value.status == K.E_ARG


def test_deterministic_repeat():
    g = rmat(14, 16, seed=31, wseed=32)
    H1 = K.kappa_coarsen(dev(g), 1, 77, 500)
    H2 = K.kappa_coarsen(dev(g), 1, 77, 500)
    assert len(H1) == len(H2)
    for l in range(len(H1)):
        a, b = H1.level(l), H2.level(l)
        assert_graph_equal(graph_np(a.graph), graph_np(b.graph), f"level {l}")


def test_graph_replays_equal_oracle_and_direct_launches():
    """A launch sequence seen twice is captured as a HIP graph and replayed
    from then on.  Every call (direct, capture, replays with eager torch work
    and host synchronisation in between, and direct launches again with
    graphs switched off) must equal the oracle."""
    import torch
    g = rgg(1 << 14, seed=9)
    for rating in (O.EXPANSION_STAR2, O.INNER_OUTER):
        OH = O.coarsen(g, rating, 5, 64, 1, 20, 64, round_stats=True)
        dg = dev(g)
        part0 = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for rep in range(5):
            say(f"rating {rating} call {rep}")
            K.graphs_enable(rep < 4)
            try:
                H, _ = check_hierarchy(g, rating, 5, 64, k=8, oracle_h=OH, dg=dg, part0=part0)
                del H
            finally:
                K.graphs_enable(False)
            x = torch.arange(1 << 16, device="cuda", dtype=torch.int64)
            assert int((x * 2).sum().item()) == (1 << 16) * ((1 << 16) - 1)
            torch.cuda.synchronize()


def test_trusted_input_skips_entry_checks_only():
    """KAPPA_COARSEN_TRUSTED: the same hierarchy as the checked call; broken
    row offsets are still rejected; unknown flags are an argument error."""
    import ctypes
    g = rgg(5000, seed=21)
    OH = O.coarsen(g, 0, 42, 64, 1, 20, 64)
    dg = dev(g)
    assert K.kappa_validate(dg) == K.OK
    H = K.kappa_coarsen(dg, 0, 42, 64, trusted=True)
    from gpu_util import compare_hierarchy
    compare_hierarchy(H, OH, check_rounds=False, k=4)
    bad = dev(g)
    bad.xadj[7] = bad.xadj[8] + 1          # offsets no longer monotone
    with pytest.raises(K.KappaError) as e:
        K.kappa_coarsen(bad, 0, 42, 64, trusted=True)
    assert e.value.status == K.E_GRAPH
    p = K._lib.c_params(0, 42, 64, 1, 20, 64, 4)   # an unknown flag
    h = ctypes.c_void_p()
    st = K.lib().kappa_coarsen(ctypes.byref(dg.c()), ctypes.byref(p), ctypes.byref(h),
                               K._lib._stream())
    assert st == K.E_ARG


def test_many_rows_of_thousands_of_entries():
    """Hundreds of coarse rows of 4095..16382 entries (hubs of about 4500
    leaves each): more than a sixteen-thousandth of the entries, so the key
    buckets' row capacity must count such rows too."""
    rng = np.random.default_rng(31)
    hubs, leaves, deg = 300, 60000, 4500
    a = np.repeat(np.arange(hubs), deg)
    b = np.concatenate([rng.choice(leaves, size=deg, replace=False) for _ in range(hubs)]) + hubs
    g = csr_from_edges(hubs + leaves, a, b, rng.integers(1, 60, size=a.size).astype(np.uint32))
    assert int(np.diff(g.xadj)[:hubs].min()) > 4094
    check_hierarchy(g, 0, 7, stop_n=2000, k=16)
