"""Persistent matching rounds (kappa_persistent_enable): a level's rounds
after the first in one cooperative launch with grid barriers.  The
hierarchy, the batched form and the served steps must equal the oracle's (and
the round kernels'), bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import assert_graph_equal, check_hierarchy, dev, graph_np
from workloads import batch_graphs, grid2d, random_graph, rgg, rmat

pytestmark = pytest.mark.gpu


@pytest.fixture
def persistent():
    K.persistent_enable(True)
    yield
    K.persistent_enable(False)


@pytest.mark.parametrize("rating", [O.EXPANSION_STAR2, O.INNER_OUTER])
def test_hierarchy_equals_oracle(persistent, rating):
    cases = [("rgg2^16", rgg(1 << 16, seed=31), 256), ("grid200", grid2d(200, 210), 100),
             ("rmat12", rmat(12, 8, seed=32, wseed=33), 64),
             ("random", random_graph(5000, 30000, seed=34, wmax=9, cmax=4, cmin=0), 40)]
    for what, g, stop in cases:
        print(f"{what} rating {rating}", flush=True)
        sys.stdout.flush()
        check_hierarchy(g, rating, 8, stop_n=stop, k=8)


def test_full_size_rgg_equals_round_kernels(persistent):
    g = rgg(1 << 20, seed=2)
    d = dev(g)
    for rating in (O.EXPANSION_STAR2, O.INNER_OUTER):
        B = K.kappa_coarsen(d, rating, 42, 1280)
        K.persistent_enable(False)
        A = K.kappa_coarsen(d, rating, 42, 1280)
        K.persistent_enable(True)
        assert len(A) == len(B)
        for l in range(len(A)):
            assert_graph_equal(graph_np(B.level(l).graph), graph_np(A.level(l).graph), f"level {l}")
            if A.level(l).cmap is not None:
                assert np.array_equal(A.level(l).cmap.cpu().numpy(), B.level(l).cmap.cpu().numpy())


def test_batched_form_equals_oracle(persistent):
    graphs = batch_graphs(count=32, seed=35, nmin=200, nmax=20000)
    du, off = K.DeviceGraph.union(graphs)
    B = K.kappa_coarsen_batch(du, off, O.EXPANSION_STAR2, 6, 128)
    for gi in range(0, len(graphs), 5):
        OH = O.coarsen(graphs[gi], O.EXPANSION_STAR2, 6, 128, 1, 20, 64)
        H = B.hierarchy(gi)
        assert len(H) == len(OH.levels)
        for l, ol in enumerate(OH.levels):
            assert_graph_equal(graph_np(H.level(l).graph), ol.graph, f"graph {gi} level {l}")
