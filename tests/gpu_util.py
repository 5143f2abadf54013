"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle element by element."""
import numpy as np

import oracle as O
import paper_0910_2004_amd as K


def dev(g):
    return K.DeviceGraph.from_csr(g, "cuda")


def graph_np(dg):
    x, a, e, v = dg.numpy()
    return O.Graph(int(dg.n), x.astype(np.int64), a.astype(np.int32), e, v)


def assert_graph_equal(got: O.Graph, want: O.Graph, what=""):
    assert got.n == want.n, f"{what}: n {got.n} != {want.n}"
    assert np.array_equal(got.xadj, want.xadj), f"{what}: xadj differs"
    assert np.array_equal(got.adj, want.adj), f"{what}: adj differs"
    assert np.array_equal(got.ew, want.ew), f"{what}: ew differs"
    assert np.array_equal(got.vw, want.vw), f"{what}: vw differs"


def check_hierarchy(g, rating, seed, stop_n, stall=(1, 20), max_levels=64, k=2,
                    part_seed=1, eps=(3, 100), check_rounds=True, check_uncoarsen=True,
                    oracle_h=None, dg=None, part0=None):
    """Coarsen on the GPU and with the oracle; compare every level, map,
    round count, round statistics and the way back up.  Returns the
    hierarchy (GPU) and the oracle hierarchy.  dg / part0: device input
    graph and level-0 partition buffer to use (fresh ones by default)."""
    H = K.kappa_coarsen(dg if dg is not None else dev(g), rating, seed, stop_n, stall[0], stall[1],
                        max_levels)
    OH = oracle_h or O.coarsen(g, rating, seed, stop_n, stall[0], stall[1], max_levels,
                               round_stats=check_rounds)
    compare_hierarchy(H, OH, check_rounds=check_rounds, check_uncoarsen=check_uncoarsen, k=k,
                      part_seed=part_seed, eps=eps, part0=part0)
    return H, OH


def compare_hierarchy(H, OH, check_rounds=True, check_uncoarsen=True, k=2, part_seed=1,
                      eps=(3, 100), part0=None):
    """Every level, map, matched count, stop reason (and, optionally, round
    count, round statistics and the way back up) of the GPU hierarchy H
    against the oracle hierarchy OH."""
    assert len(H) == len(OH.levels), f"levels {len(H)} != {len(OH.levels)}"
    for l, ol in enumerate(OH.levels):
        lv = H.level(l)
        assert_graph_equal(graph_np(lv.graph), ol.graph, f"level {l}")
        assert lv.stop_reason == ol.stop_reason, f"level {l} stop {lv.stop_reason} != {ol.stop_reason}"
        if ol.cmap is not None:
            assert np.array_equal(lv.cmap.cpu().numpy(), ol.cmap), f"level {l}: cmap differs"
            assert lv.matched == ol.matched
        if check_rounds and ol.mate is not None:
            assert lv.rounds == ol.rounds, f"level {l}: rounds {lv.rounds} != {ol.rounds}"
            gr = int(H.info(l).grid_rounds)   # 0 on levels the one-workgroup tail ran
            assert 0 <= gr <= lv.rounds, f"level {l}: grid rounds {gr}"
            r, p, d = H.round_stats(l)
            kk = min(r, 64)
            assert np.array_equal(p, ol.round_active[:kk]), f"level {l}: round activity differs"
            assert np.array_equal(d, ol.round_degree[:kk]), f"level {l}: round degrees differ"
    if check_uncoarsen:
        part0, res = K.kappa_uncoarsen(H, k, part_seed, eps[0], eps[1], part0=part0)
        oparts, ores = O.uncoarsen(OH, k, part_seed, eps[0], eps[1])
        assert np.array_equal(part0.cpu().numpy(), oparts[0])
        for l in range(len(OH.levels)):
            assert res[l].as_tuple() == ores[l].as_tuple(), f"level {l}: cut/balance differs"


def rgg_rcb(n, seed):
    """The random geometric graph of n points (seed) with its nodes renamed in
    recursive coordinate bisection order (the oracle's reference order)."""
    from oracle.rcb import rcb_order, relabel
    from workloads import rgg, rgg_points
    return relabel(O.Graph.of(rgg(n, seed=seed)), rcb_order(rgg_points(n, seed)))



def gpu_hierarchy_digest(H, k, part_seed=1, eps=(3, 100)):
    """The digests of oracle_digest.hierarchy_digest for a GPU hierarchy and
    its way back up (stand-in partition with k, part_seed, eps)."""
    from oracle_digest import digest
    lvls = []
    for l in range(len(H)):
        lv = H.level(l)
        x, a, e, v = lv.graph.numpy()
        lvls.append((int(lv.graph.n), int(x[-1]) if len(x) else 0, digest(x, np.int64),
                     digest(a, np.int32), digest(e, np.uint32), digest(v, np.uint32),
                     None if lv.cmap is None else digest(lv.cmap.cpu().numpy(), np.int32),
                     int(lv.matched), int(lv.stop_reason)))
    part0, res = K.kappa_uncoarsen(H, k, part_seed, eps[0], eps[1])
    return (lvls, digest(part0.cpu().numpy(), np.int32),
            [tuple(int(t) for t in r.as_tuple()) for r in res])
