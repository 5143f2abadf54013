"""Batched form (kappa_coarsen_batch): many graphs coarsened together as one
block-diagonal union.  Every graph's hierarchy must equal, bit for bit, the
oracle's hierarchy of that graph alone (levels, maps, matched counts, stop
reasons, and the way back up), and kappa_coarsen's on that graph alone."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import assert_graph_equal, compare_hierarchy, dev, graph_np
from workloads import (CSR, batch_graphs, complete_graph, cycle_graph, grid2d, path_graph,
                       random_graph, rgg, rmat, star_graph)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _empty():
    return CSR(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint32),
               np.zeros(0, np.uint32))


def _isolated(n):
    return CSR(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint32),
               np.ones(n, np.uint32))


def _mix():
    gs = [grid2d(5, 7), path_graph([3, 4, 2]), complete_graph(8), star_graph(40), cycle_graph(9),
          _empty(), grid2d(1, 1), _isolated(30), path_graph([1, 2, 3, 4, 5, 6, 7]),
          random_graph(60, 150, seed=71, wmax=5, cmax=3, cmin=0), rgg(3000, seed=5),
          rmat(10, 8, seed=13, wseed=14), star_graph(5000), grid2d(40, 41)]
    gs += batch_graphs(count=16, seed=9, nmin=50, nmax=4000)
    return gs


@pytest.mark.parametrize("rating", [0, 1, 4])
def test_batch_matches_oracle_per_graph(rating):
    graphs = _mix()
    du, off = K.DeviceGraph.union(graphs)
    stop = [4 + (7 * g) % 40 for g in range(len(graphs))]
    say(f"batch of {len(graphs)} graphs, n={du.n} nnz={du.nnz}, rating {rating}")
    B = K.kappa_coarsen_batch(du, off, rating, seed=42, stop_n=stop)
    assert len(B) == len(graphs)
    for g, G in enumerate(graphs):
        OH = O.coarsen(G, rating, 42, stop[g], 1, 20, 64)
        levels, reason = B.info(g)
        assert levels == len(OH.levels), f"graph {g}: levels {levels} != {len(OH.levels)}"
        assert reason == OH.levels[-1].stop_reason, f"graph {g}: stop {reason}"
        H = B.hierarchy(g)
        compare_hierarchy(H, OH, check_rounds=False, check_uncoarsen=G.n > 0, k=1 + g % 5)
        del H


def test_batch_equals_single_calls():
    graphs = _mix()[10:]
    du, off = K.DeviceGraph.union(graphs)
    B = K.kappa_coarsen_batch(du, off, 1, seed=7, stop_n=30)
    for g, G in enumerate(graphs):
        H1 = K.kappa_coarsen(dev(G), 1, 7, 30)
        H2 = B.hierarchy(g)
        assert len(H1) == len(H2)
        for l in range(len(H1)):
            a, b = H1.level(l), H2.level(l)
            assert_graph_equal(graph_np(b.graph), graph_np(a.graph), f"graph {g} level {l}")
            if a.cmap is not None:
                assert np.array_equal(a.cmap.cpu().numpy(), b.cmap.cpu().numpy())
            assert a.matched == b.matched and a.stop_reason == b.stop_reason


def test_batch_max_levels_and_stall():
    graphs = [rgg(2000, seed=s) for s in range(5)] + [star_graph(300)]
    du, off = K.DeviceGraph.union(graphs)
    for max_levels in (0, 1, 3):
        B = K.kappa_coarsen_batch(du, off, 0, seed=3, stop_n=10, max_levels=max_levels)
        for g, G in enumerate(graphs):
            OH = O.coarsen(G, 0, 3, 10, 1, 20, max_levels)
            compare_hierarchy(B.hierarchy(g), OH, check_rounds=False, check_uncoarsen=False)


def test_batch_rejects_edges_between_graphs():
    g = grid2d(4, 4)
    with pytest.raises(K.KappaError) as e:
        K.kappa_coarsen_batch(dev(g), np.array([0, 8, 16], np.int32), 0)
    assert e.value.status == K.E_GRAPH
    with pytest.raises(K.KappaError) as e:
        K.kappa_coarsen_batch(dev(g), np.array([0, 9, 8], np.int32), 0)
    assert e.value.status == K.E_ARG


@pytest.mark.parametrize("rating", [0, 1])
def test_graphs_form_equals_union_form_and_oracle(rating):
    """kappa_coarsen_graphs (separate device graphs, union built by the
    library) gives every graph the oracle's hierarchy, and the same levels as
    kappa_coarsen_batch on a union built on the host."""
    graphs = _mix()
    stop = [4 + (5 * g) % 33 for g in range(len(graphs))]
    dgs = [dev(G) for G in graphs]
    B = K.kappa_coarsen_graphs(dgs, rating, seed=42, stop_n=stop)
    del dgs   # the batch owns its union
    du, off = K.DeviceGraph.union(graphs)
    B2 = K.kappa_coarsen_batch(du, off, rating, seed=42, stop_n=stop)
    assert len(B) == len(graphs)
    for g, G in enumerate(graphs):
        OH = O.coarsen(G, rating, 42, stop[g], 1, 20, 64)
        assert B.info(g) == B2.info(g) == (len(OH.levels), OH.levels[-1].stop_reason), f"graph {g}"
        compare_hierarchy(B.hierarchy(g), OH, check_rounds=False, check_uncoarsen=G.n > 0, k=1 + g % 7)
    say(f"{len(graphs)} graphs equal, rating {rating}")
