"""The tuning table (kappa_tuning) moves work between kernels and never
changes a result: under tables at both ends of every range, the hierarchy,
the batched form and the way back up equal the oracle's, bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import assert_graph_equal, check_hierarchy, dev, graph_np
from workloads import batch_graphs, grid2d, rgg, rmat, star_graph

pytestmark = pytest.mark.gpu

LOW = {"bin_small_max": 1, "tail_max": 0, "finish_max": 0, "finish_max_big": 0,
       "row_small_max": 2, "scan_one_block_max": 0, "rounds_base": 1, "rounds_n0": 1,
       "rounds_growth": 2, "rounds_cap": 1}
HIGH = {"bin_small_max": 16, "tail_max": 4096, "finish_max": 1 << 20, "finish_max_big": 1 << 16,
        "row_small_max": 64, "scan_one_block_max": 1 << 22, "rounds_base": 16,
        "rounds_n0": 1 << 24, "rounds_growth": 1024, "rounds_cap": 32}
MID = {"bin_small_max": 4, "tail_max": 512, "finish_max": 1024, "finish_max_big": 8,
       "row_small_max": 16, "scan_one_block_max": 4096, "rounds_base": 2, "rounds_n0": 512,
       "rounds_growth": 4, "rounds_cap": 12}


@pytest.fixture
def table():
    saved = K.tuning_get()
    yield
    K.tuning_set(saved)


@pytest.mark.parametrize("name", ["LOW", "MID", "HIGH"])
def test_hierarchy_does_not_depend_on_the_table(table, name):
    K.tuning_set({"LOW": LOW, "MID": MID, "HIGH": HIGH}[name])
    print(f"table {name}: {K.tuning_get()}", flush=True)
    sys.stdout.flush()
    cases = [("rgg2^14", rgg(1 << 14, seed=3), O.EXPANSION_STAR2, 64),
             ("rgg2^14 io", rgg(1 << 14, seed=4), O.INNER_OUTER, 64),
             ("rmat13", rmat(13, 16, seed=5, wseed=6), O.EXPANSION_STAR2, 256),
             ("grid90", grid2d(90, 90), O.INNER_OUTER, 40),
             ("star3000", star_graph(3000), O.EXPANSION_STAR2, 8)]
    for what, g, rating, stop in cases:
        print(f"  {what}", flush=True)
        check_hierarchy(g, rating, 17, stop_n=stop, k=8)


def test_batched_form_does_not_depend_on_the_table(table):
    graphs = batch_graphs(count=24, seed=12, nmin=50, nmax=6000)
    du, off = K.DeviceGraph.union(graphs)
    want = K.kappa_coarsen_batch(du, off, O.EXPANSION_STAR2, 5, 64)
    for t in (LOW, MID, HIGH):
        K.tuning_set(t)
        got = K.kappa_coarsen_batch(du, off, O.EXPANSION_STAR2, 5, 64)
        for gi in range(len(graphs)):
            a, b = want.hierarchy(gi), got.hierarchy(gi)
            assert len(a) == len(b)
            for l in range(len(a)):
                assert_graph_equal(graph_np(b.level(l).graph), graph_np(a.level(l).graph),
                                   f"graph {gi} level {l}")
                if a.level(l).cmap is not None:
                    assert np.array_equal(a.level(l).cmap.cpu().numpy(), b.level(l).cmap.cpu().numpy())


def test_full_size_rmat_under_a_low_table(table):
    """R-MAT scale 18 (hubs, handed-back levels, the large-row merge) under
    the low table against the default table's hierarchy."""
    g = rmat(18, 16, seed=7, wseed=8)
    d = dev(g)
    A = K.kappa_coarsen(d, O.EXPANSION_STAR2, 3, 1024)
    K.tuning_set(MID)
    B = K.kappa_coarsen(d, O.EXPANSION_STAR2, 3, 1024)
    assert len(A) == len(B)
    for l in range(len(A)):
        assert_graph_equal(graph_np(B.level(l).graph), graph_np(A.level(l).graph), f"level {l}")
