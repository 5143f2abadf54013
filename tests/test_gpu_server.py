"""Level-granular continuous batching (kappa_server_*, serve.LevelServer).

A request's hierarchy must not depend on what it was batched with or when it
joined: every level (CSR, map, |M|), its stop reason and its way back up equal
kappa_coarsen's on the request alone and the oracle's on that graph, bit for
bit.  Requests join between steps at their level 0 while others are several
levels deep, so every step mixes tie-break seeds of different levels."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import assert_graph_equal, compare_hierarchy, dev, graph_np
from workloads import (CSR, complete_graph, cycle_graph, grid2d, path_graph, random_graph, rgg,
                       rmat, serve_requests, star_graph)

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


def _same_as(H, A, what):
    """Served hierarchy H against kappa_coarsen's A (both on the device)."""
    assert len(H) == len(A), f"{what}: levels {len(H)} != {len(A)}"
    for l in range(len(A)):
        x, y = H.level(l), A.level(l)
        assert_graph_equal(graph_np(x.graph), graph_np(y.graph), f"{what} level {l}")
        assert x.stop_reason == y.stop_reason, f"{what} level {l}: stop {x.stop_reason} != {y.stop_reason}"
        if y.cmap is not None:
            assert np.array_equal(x.cmap.cpu().numpy(), y.cmap.cpu().numpy()), f"{what} level {l}"
            assert x.matched == y.matched, f"{what} level {l}"


def _drain(srv, admit_plan):
    """Steps srv until no request is active; admit_plan[s] (graph, stop) pairs
    are admitted before step s.  Returns {id: (graph, stop)} and the order of
    finishing ids."""
    reqs, order, s = {}, [], 0
    while True:
        for g, stop in admit_plan.get(s, []):
            reqs[srv.admit(dev(g), stop)] = (g, stop)
        if srv.active() == 0 and s >= max(admit_plan, default=0):
            break
        order += srv.step()
        s += 1
    return reqs, order


@pytest.mark.parametrize("rating", [O.EXPANSION_STAR2, O.INNER_OUTER])
def test_server_staggered_equals_alone_and_oracle(rating):
    mix = [g for g, _, _ in serve_requests(18, seed=11, emax=1.5e5)]
    mix += [star_graph(2000), rmat(11, 16, seed=3, wseed=4), grid2d(30, 31)]
    stops = [40 + 13 * i for i in range(len(mix))]
    plan = {}
    for i, g in enumerate(mix):   # joins at steps 0, 0, 1, 2, 2, 3, ...
        plan.setdefault((2 * i) // 3, []).append((g, stops[i]))
    srv = K.Server(rating, seed=9)
    reqs, order = _drain(srv, plan)
    assert sorted(order) == sorted(reqs) and len(order) == len(mix)
    for rid in order:
        g, stop = reqs[rid]
        H = srv.take(rid)
        _same_as(H, K.kappa_coarsen(dev(g), rating, 9, stop), f"request {rid}")
        if g.n <= 60000:
            compare_hierarchy(H, O.coarsen(g, rating, 9, stop, 1, 20, 64), check_rounds=False,
                              k=1 + rid % 7)
    say(f"{len(mix)} staggered requests equal kappa_coarsen alone and the oracle")


@pytest.mark.parametrize("max_levels", [0, 1, 2, 64])
def test_server_edge_cases(max_levels):
    graphs = [_empty(), grid2d(1, 1), _isolated(30), path_graph([3, 4, 2]), complete_graph(8),
              star_graph(300), cycle_graph(9), random_graph(60, 150, seed=71, wmax=5, cmax=3, cmin=0),
              grid2d(40, 41), rgg(3000, seed=5), rmat(10, 8, seed=13, wseed=14)]
    # stop sizes: 0, below n, at n, above n (the size rule at level 0)
    stops = [0, 1, 30, 1, 8, 10, 100, 5, 1640, 30, 64]
    plan = {0: list(zip(graphs[:6], stops[:6])), 1: list(zip(graphs[6:], stops[6:]))}
    srv = K.Server(O.EXPANSION_STAR2, seed=4, max_levels=max_levels)
    reqs, order = _drain(srv, plan)
    assert len(order) == len(graphs)
    for rid in order:
        g, stop = reqs[rid]
        H = srv.take(rid)
        _same_as(H, K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 4, stop, 1, 20, max_levels),
                 f"request {rid} (max_levels {max_levels})")
        compare_hierarchy(H, O.coarsen(g, O.EXPANSION_STAR2, 4, stop, 1, 20, max_levels),
                          check_rounds=False, check_uncoarsen=g.n > 0, k=2)


def test_server_stall_rule_and_no_stall():
    graphs = [star_graph(500), rgg(4000, seed=8), path_graph([1] * 200)]
    for stall in ((1, 20), (0, 1), (1, 2)):
        srv = K.Server(O.INNER_OUTER, seed=2, stall_num=stall[0], stall_den=stall[1])
        reqs, order = _drain(srv, {0: [(g, 3) for g in graphs]})
        for rid in order:
            g, stop = reqs[rid]
            H = srv.take(rid)
            _same_as(H, K.kappa_coarsen(dev(g), O.INNER_OUTER, 2, stop, stall[0], stall[1]),
                     f"request {rid} stall {stall}")


def test_server_step_boundaries_and_interrupt():
    """A step runs until a request's hierarchy ends; with the interrupt raised
    it ends after every level; an interrupt from another thread in the middle
    of a step ends it at a level boundary.  The hierarchy is the same in
    every case."""
    import threading
    g, stop = grid2d(64, 64), 20
    A = K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 3, stop)
    L = len(A)
    assert L > 3 and A.level(L - 1).stop_reason == K.STOP_SIZE
    srv = K.Server(O.EXPANSION_STAR2, seed=3)
    i = srv.admit(dev(g), stop)
    assert srv.step() == [i]                      # alone: one step, every level
    _same_as(srv.take(i), A, "one step")
    srv.interrupt(True)
    i = srv.admit(dev(g), stop)
    steps = 0
    while srv.active():
        fin = srv.step()
        steps += 1
    assert fin == [i] and steps == L - 1          # one level per step
    _same_as(srv.take(i), A, "a level per step")
    srv.interrupt(False)
    small, big = grid2d(16, 16), grid2d(128, 128)
    a = srv.admit(dev(small), stop)
    b = srv.admit(dev(big), stop)
    assert srv.step() == [a] and srv.active() == 1   # the step ends where the small one does
    assert srv.step() == [b]
    _same_as(srv.take(a), K.kappa_coarsen(dev(small), O.EXPANSION_STAR2, 3, stop), "small")
    _same_as(srv.take(b), K.kappa_coarsen(dev(big), O.EXPANSION_STAR2, 3, stop), "big")
    # interrupts from another thread while steps run
    h = rgg(1 << 20, seed=12)
    c = srv.admit(dev(h), 64)
    done, steps = [], 0
    while srv.active():
        t = threading.Timer(0.002, srv.interrupt)
        t.start()
        done += srv.step()
        t.join()
        srv.interrupt(False)
        steps += 1
    assert done == [c]
    say(f"rgg 2^20 in {steps} steps under interrupts")
    _same_as(srv.take(c), K.kappa_coarsen(dev(h), O.EXPANSION_STAR2, 3, 64), "interrupted")


def test_server_api_errors_and_reuse():
    import ctypes
    srv = K.Server(O.EXPANSION_STAR2, seed=1)
    assert srv.step() == [] and srv.active() == 0
    with pytest.raises(K.KappaError) as e:
        srv.take(0)
    assert e.value.status == K.E_ARG
    # an asymmetric graph is rejected at admission and leaves nothing behind
    bad = CSR(3, np.array([0, 1, 1, 1], np.int64), np.array([1], np.int32),
              np.array([1], np.uint32), np.ones(3, np.uint32))
    with pytest.raises(K.KappaError) as e:
        srv.admit(dev(bad), 1)
    assert e.value.status == K.E_GRAPH and srv.active() == 0
    a = srv.admit(dev(grid2d(20, 20)), 10)
    b = srv.admit(dev(grid2d(30, 30)), 10)
    with pytest.raises(K.KappaError):
        srv.take(a)   # not finished yet
    # cap 0: finished ids are counted, not listed
    done = 0
    while srv.active():
        nf = ctypes.c_int32()
        st = K.lib().kappa_server_step(srv.handle, None, 0, ctypes.byref(nf))
        assert st == 0
        done += nf.value
    assert done == 2
    for rid, side in ((b, 30), (a, 20)):
        H = srv.take(rid)
        _same_as(H, K.kappa_coarsen(dev(grid2d(side, side)), O.EXPANSION_STAR2, 1, 10), f"{rid}")
        with pytest.raises(K.KappaError):
            srv.take(rid)   # taken already
    # the server takes new requests after draining
    c = srv.admit(dev(grid2d(8, 9)), 5)
    _, order = _drain(srv, {})
    assert order == [c]
    _same_as(srv.take(c), K.kappa_coarsen(dev(grid2d(8, 9)), O.EXPANSION_STAR2, 1, 5), "reuse")


def test_taken_hierarchy_outlives_server_and_step_arenas():
    """Levels live in step arenas shared by the requests of a step: a
    hierarchy taken, with its server freed and the other requests of its
    steps freed, still reads back whole."""
    g1, g2 = rgg(20000, seed=3), grid2d(60, 70)
    srv = K.Server(O.EXPANSION_STAR2, seed=5)
    i1 = srv.admit(dev(g1), 50)
    i2 = srv.admit(dev(g2), 50)
    _drain(srv, {})
    H2 = srv.take(i2)
    H1 = srv.take(i1)
    del srv, H1
    import gc
    gc.collect()
    junk = [K.kappa_coarsen(dev(rgg(30000, seed=s)), 0, 1, 100) for s in range(3)]   # reuse memory
    del junk
    _same_as(H2, K.kappa_coarsen(dev(g2), O.EXPANSION_STAR2, 5, 50), "kept")


def _level_requests(count, spread, seed):
    from paper_0910_2004_amd.serve import Request
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(spread, size=count)) if spread > 0 else np.zeros(count)
    return [Request(i, g, rating, k, arrival=float(t[i]))
            for i, (g, rating, k) in enumerate(serve_requests(count, seed=seed, emax=2e5))]


@pytest.mark.parametrize("spread", [0.0, 0.002])
def test_level_server_equals_alone(spread):
    from paper_0910_2004_amd.serve import LevelServer, latency_stats, serve_plain
    reqs = _level_requests(40, spread, seed=5)
    say(f"{len(reqs)} requests, mean gap {spread * 1e3} ms")
    served = LevelServer().run(reqs, keep=True)
    alone = serve_plain(reqs, keep=True)
    assert [r.rid for r in served] == [r.rid for r in alone] == list(range(len(reqs)))
    for a, b in zip(served, alone):
        assert (a.levels, a.stop_reason, a.cut) == (b.levels, b.stop_reason, b.cut), f"request {a.rid}"
        _same_as(a.hierarchy, b.hierarchy, f"request {a.rid}")
    say(latency_stats(reqs, served))
    if spread == 0.0:
        assert max(r.batch for r in served) > 1   # requests were mixed


def test_level_server_budget_admits_one_at_a_time():
    from paper_0910_2004_amd.serve import LevelServer
    reqs = _level_requests(8, 0.0, seed=6)
    served = LevelServer(hbm_budget=1).run(reqs)
    assert all(r.batch == 1 for r in served)


def test_level_server_mix_at_full_size_equals_oracle():
    """The served mix at its largest sizes (|E| from 10^3 to 4 * 10^6,
    R-MAT up to scale 18, with the three largest members of each kind added:
    a 1414 x 1414 grid, an RGG of 10^6 nodes, R-MAT scale 18), arriving over
    time into the level-granular server: every request's hierarchy and way
    back up against the oracle's run on that graph alone (digests computed in
    worker processes beside the GPU)."""
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor

    from gpu_util import gpu_hierarchy_digest
    from oracle_digest import served_digest, served_graph
    from paper_0910_2004_amd.serve import LevelServer, Request
    from workloads.graphs import _serve_member

    count, seed = 40, 23
    specs, ratings, ks = [], [], []
    for i in range(count):
        _, rating, k = _serve_member(seed, i, 1e3, 4e6)
        specs.append(("mix", seed, i, 1e3, 4e6))
        ratings.append(rating)
        ks.append(k)
    for spec, rating, k in ((("grid", 1414), 0, 64), (("rgg", 1000000, 77), 1, 32),
                            (("rmat", 18, 78, 79), 0, 8)):
        specs.append(spec)
        ratings.append(rating)
        ks.append(k)
    jobs = [(specs[i], ratings[i], 42, 20 * ks[i], 64, ks[i]) for i in range(len(specs))]
    workers = min(16, os.cpu_count() or 1)
    pool = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))
    futs = [pool.submit(served_digest, j) for j in jobs]
    graphs = [served_graph(s) for s in specs]
    say(f"{len(graphs)} requests, |E| up to {max(int(g.xadj[-1]) // 2 for g in graphs)}")
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(0.01, size=len(graphs)))
    reqs = [Request(i, graphs[i], ratings[i], ks[i], arrival=float(t[i])) for i in range(len(graphs))]
    served = LevelServer().run(reqs, keep=True)
    say(f"served; mean batch {np.mean([r.batch for r in served]):.2f}")
    got = [gpu_hierarchy_digest(r.hierarchy, ks[r.rid]) for r in served]
    bad = []
    for i, f in enumerate(futs):
        if got[i] != f.result():
            bad.append(i)
        if i % 8 == 7:
            say(f"{i + 1} of {len(futs)} compared")
    pool.shutdown()
    assert not bad, f"requests {bad} differ from the oracle"
