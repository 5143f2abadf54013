"""The two-phase matcher of Section 3.3 on the GPU (kappa_match_two_phase and
kappa_coarsen with KAPPA_COARSEN_TWO_PHASE) against the oracle's
match_two_phase: the block matching, the merged matching, |M| and whole
hierarchies bit-exact, from hand-sized graphs to the random geometric graph
of 2^20 nodes in recursive coordinate bisection order."""
import ctypes
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import rgg_rcb, compare_hierarchy, dev
from workloads import (complete_graph, csr_from_edges, cycle_graph, grid2d, path_graph,
                       random_graph, rgg, rmat, star_graph)

pytestmark = pytest.mark.gpu
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


def check_match(g, rating, seed, bb, what=""):
    om, omm, oloc, _, _ = O.match_two_phase(g, rating, seed, bb)
    mate, loc, m = K.kappa_match_two_phase(dev(g), rating, seed, bb)
    assert np.array_equal(loc.cpu().numpy(), oloc), f"{what}: block matching differs"
    assert np.array_equal(mate.cpu().numpy(), om), f"{what}: matching differs"
    assert m == omm, f"{what}: |M| {m} != {omm}"
    return om


def small_graphs():
    cases = [("P2", path_graph([5])), ("W2", path_graph([1, 2, 3, 4])), ("tri", complete_graph(3)),
             ("C6", cycle_graph(6)), ("K1_5", star_graph(5)), ("K9", complete_graph(9)),
             ("grid7x9", grid2d(7, 9))]
    for s in range(12):
        n = 6 + (s * 17) % 90
        m = min(n * (n - 1) // 2, n + (s * 41) % (3 * n))
        cases.append((f"rnd{s}", random_graph(n, m, seed=700 + s, wmax=[1, 6, 1000][s % 3],
                                              cmax=[1, 3, 50][(s // 3) % 3],
                                              cmin=0 if s % 4 == 0 else 1)))
    return cases


@pytest.mark.parametrize("rating", RATINGS)
def test_small_graphs_every_block_size(rating):
    for name, g in small_graphs():
        for bb in (0, 1, 2, 3, 5, 11):
            check_match(g, rating, O.level_seed(9, bb), bb, f"{name} bb={bb}")


def test_hand_worked_path():
    g = path_graph([1, 2, 3, 4])
    mate, loc, m = K.kappa_match_two_phase(dev(g), O.EXPANSION_STAR2, 5, 1)
    assert loc.cpu().tolist() == [1, 0, 3, 2, -1]
    assert mate.cpu().tolist() == [1, 0, -1, 4, 3] and m == 2


def test_one_block_is_greedy():
    for s, g in enumerate([random_graph(2000, 9000, seed=31, wmax=50), grid2d(40, 50),
                           rmat(11, 8, seed=3, wseed=4)]):
        seed = O.level_seed(s, 0)
        for r in (0, 1):
            om = check_match(g, r, seed, 11, f"graph {s}")
            assert np.array_equal(om, O.match_greedy(g, r, seed)[0])


@pytest.mark.parametrize("rating", [0, 1, 4])
def test_medium_graphs(rating):
    cases = [("rgg2^15 rcb", rgg_rcb(1 << 15, 11), (6, 8, 10, 11)),
             ("rgg2^15", rgg(1 << 15, seed=11), (10,)),
             ("grid150", grid2d(150, 150), (4, 7, 11)),
             ("rmat13", rmat(13, 16, seed=12, wseed=13), (5, 9, 11))]
    for name, g, bbs in cases:
        for bb in bbs:
            say(name, "rating", rating, "bb", bb)
            check_match(g, rating, O.level_seed(3, 0), bb, f"{name} bb={bb}")


def test_hub_rows_inside_blocks():
    # rows above 16 entries take the wave path of the block phase; a star's
    # centre sees its whole block
    for name, g in [("star3000", star_graph(3000)), ("star100", star_graph(100)),
                    ("dense", random_graph(600, 40000, seed=5, wmax=9, cmax=3, cmin=1))]:
        for bb in (3, 8, 11):
            for r in (0, 1, 2):
                check_match(g, r, O.level_seed(1, r), bb, f"{name} bb={bb} r={r}")


def test_edge_cases():
    empty = csr_from_edges(0, np.zeros(0, np.int64), np.zeros(0, np.int64))
    mate, loc, m = K.kappa_match_two_phase(dev(empty), 0, 1, 4)
    assert m == 0 and mate.numel() == 0
    iso = csr_from_edges(50, np.zeros(0, np.int64), np.zeros(0, np.int64))
    mate, loc, m = K.kappa_match_two_phase(dev(iso), 0, 1, 2)
    assert m == 0 and (mate.cpu().numpy() == -1).all() and (loc.cpu().numpy() == -1).all()
    g = random_graph(300, 900, seed=2)
    # a ragged last block, sizes not a multiple of the block
    check_match(g, 0, 7, 7, "ragged")
    d = dev(g)
    for bb in (-1, 12, 40):
        with pytest.raises(K.KappaError) as e:
            K.kappa_match_two_phase(d, 0, 7, bb)
        assert e.value.status == K.E_ARG


def test_flag_rules():
    g = grid2d(20, 20)
    d = dev(g)
    L = K.lib()
    h = ctypes.c_void_p()
    for bb in (-1, 12):
        p = K._lib.c_params(0, 42, 64, 1, 20, 64, K._lib.COARSEN_TWO_PHASE, bb)
        assert L.kappa_coarsen(ctypes.byref(d.c()), ctypes.byref(p), ctypes.byref(h),
                               K._lib._stream()) == K.E_ARG
    # the batched forms take no two-phase flag
    du, noff = K.DeviceGraph.union([g, g])
    p = K._lib.c_params(0, 42, 64, 1, 20, 64, K._lib.COARSEN_TWO_PHASE, 4)
    nof = np.ascontiguousarray(noff, dtype=np.int32)
    assert L.kappa_coarsen_batch(ctypes.byref(du.c()), 2, nof.ctypes.data, None, ctypes.byref(p),
                                 ctypes.byref(h), K._lib._stream()) == K.E_ARG


HIER = [("grid128", lambda: grid2d(128, 128), 64, (6, 10)),
        ("rgg2^16 rcb", lambda: rgg_rcb(1 << 16, 21), 1280, (8, 11)),
        ("rmat13", lambda: rmat(13, 16, seed=5, wseed=6), 256, (9,)),
        ("random", lambda: random_graph(20000, 70000, seed=8, wmax=9, cmax=4, cmin=0), 64, (5,))]


@pytest.mark.parametrize("rating", [0, 1, 4])
@pytest.mark.parametrize("name,make,stop_n,bbs", HIER, ids=[h[0] for h in HIER])
def test_hierarchy_equals_oracle(name, make, stop_n, bbs, rating):
    g = make()
    d = dev(g)
    for bb in bbs:
        OH = O.coarsen(g, rating, 42, stop_n, 1, 20, 64, block_bits=bb)
        H = K.kappa_coarsen(d, rating, 42, stop_n, block_bits=bb)
        say(f"{name} rating {rating} bb {bb}: levels {[H.info(l).n for l in range(len(H))]}")
        compare_hierarchy(H, OH, check_rounds=False, k=8)


@pytest.mark.parametrize("rating", [0, 1])
def test_full_size_rgg_rcb(rating):
    # the benchmark graph in recursive coordinate bisection order, blocks of 1024
    g = rgg_rcb(1 << 20, 2)
    OH = O.coarsen(g, rating, 42, 1280, 1, 20, 64, block_bits=10)
    H = K.kappa_coarsen(dev(g), rating, 42, 1280, block_bits=10)
    say(f"rgg 2^20 rcb rating {rating}: levels {[H.info(l).n for l in range(len(H))]}")
    compare_hierarchy(H, OH, check_rounds=False, k=64)
