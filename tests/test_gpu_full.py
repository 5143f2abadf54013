"""Full-size parity: the benchmark's workload (random geometric graph,
n = 2^20, mean degree 8, unit weights, k = 64, stop at 20k nodes) through the
same entry points and launch configuration bench.py times (each rating alone,
and both at once on two streams as in the timed step), compared with the
oracle level by level (every array, map, round count, cut and balance); the
R-MAT of scale 22; and every graph of the 4096-graph batch."""
import sys

import pytest

import oracle as O
from gpu_util import check_hierarchy
from workloads import rgg

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

_G = {}


def _graph():
    if "g" not in _G:
        _G["g"] = rgg(1 << 20, seed=2)
    return _G["g"]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("rating", [O.EXPANSION_STAR2, O.INNER_OUTER])
def test_rgg_2_20_full_hierarchy(rating):
    g = _graph()
    print(f"rgg n={g.n} m={g.m} rating={rating}", flush=True)
    H, OH = check_hierarchy(g, rating, 42, stop_n=20 * 64, k=64)
    print("levels", [lv.graph.n for lv in OH.levels], flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(600)
def test_rgg_2_20_both_ratings_on_two_streams():
    # the timed step itself: one validation, then both ratings' hierarchies
    # and uncoarsenings at once, one host thread and stream each
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import paper_0910_2004_amd as K
    from gpu_util import compare_hierarchy, dev
    g = _graph()
    ratings = [O.EXPANSION_STAR2, O.INNER_OUTER]
    OH = {r: O.coarsen(g, r, 42, 1280, 1, 20, 64, round_stats=True) for r in ratings}
    OP = {r: O.uncoarsen(OH[r], 64, 1, 3, 100) for r in ratings}
    dg = dev(g)
    assert K.kappa_validate(dg) == K.OK
    streams = [torch.cuda.Stream() for _ in ratings]
    part0s = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in ratings]
    torch.cuda.synchronize()

    def one(i):
        with torch.cuda.stream(streams[i]):
            H = K.kappa_coarsen(dg, ratings[i], 42, 1280, 1, 20, 64, trusted=True)
            part, res = K.kappa_uncoarsen(H, 64, 1, 3, 100, part0=part0s[i])
            torch.cuda.current_stream().synchronize()
            return H, part.cpu().numpy(), [x.as_tuple() for x in res]

    with ThreadPoolExecutor(max_workers=2) as pool:
        got = [f.result() for f in [pool.submit(one, i) for i in range(2)]]
    for i, r in enumerate(ratings):
        H, part, res = got[i]
        print(f"rating {r}: levels {len(H)}", flush=True)
        compare_hierarchy(H, OH[r], check_rounds=True, check_uncoarsen=False)
        oparts, ores = OP[r]
        assert np.array_equal(part, oparts[0])
        assert [x for x in res] == [x.as_tuple() for x in ores]


def _sha(a, dtype):
    import hashlib

    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


@pytest.mark.timeout(900)
def test_rmat_scale22_full_hierarchy():
    """R-MAT scale 22 (n = 2^22, 16 * 2^22 samples, (a, b, c) = (0.57, 0.19,
    0.19), w uniform in [1, 100]), expansion*2, k = 256, stop at 20k nodes,
    stall 1/20, in the launch configuration bench.py times (one validation,
    then a trusted kappa_coarsen and kappa_uncoarsen): every level's graph,
    map (which fixes the matching), |M|, round count and round statistics, the level-0
    partition and every level's cut/balance against the oracle's, stored as
    SHA-256 digests by tests/golden/make_rmat22.py (oracle only; the oracle
    takes minutes at this size)."""
    import json
    import os

    import numpy as np

    import paper_0910_2004_amd as K
    from gpu_util import dev
    from workloads import rmat
    with open(os.path.join(os.path.dirname(__file__), "golden", "rmat22_levels.json")) as f:
        want = json.load(f)
    g = rmat(22, 16, seed=3, wseed=33)
    wi = want["input"]
    assert (g.n, g.nnz) == (wi["n"], wi["nnz"])
    assert _sha(g.xadj, np.int64) == wi["xadj"] and _sha(g.adj, np.int32) == wi["adj"]
    assert _sha(g.ew, np.uint32) == wi["ew"] and _sha(g.vw, np.uint32) == wi["vw"]
    print(f"rmat scale 22: n={g.n} m={g.m} (input digests equal)", flush=True)
    dg = dev(g)
    assert K.kappa_validate(dg) == K.OK
    H = K.kappa_coarsen(dg, O.EXPANSION_STAR2, 42, 5120, 1, 20, 64, trusted=True)
    print(f"GPU levels: {[H.info(l).n for l in range(len(H))]}", flush=True)
    assert len(H) == len(want["levels"])
    for l, wl in enumerate(want["levels"]):
        lv = H.level(l)
        x, a, e, v = lv.graph.numpy()
        wg = wl["graph"]
        assert (int(lv.graph.n), int(x[-1]) if len(x) else 0) == (wg["n"], wg["nnz"]), f"level {l}"
        assert _sha(x, np.int64) == wg["xadj"], f"level {l}: xadj"
        assert _sha(a, np.int32) == wg["adj"], f"level {l}: adj"
        assert _sha(e, np.uint32) == wg["ew"], f"level {l}: ew"
        assert _sha(v, np.uint32) == wg["vw"], f"level {l}: vw"
        assert lv.stop_reason == wl["stop_reason"], f"level {l}: stop"
        if "cmap" in wl:
            assert _sha(lv.cmap.cpu().numpy(), np.int32) == wl["cmap"], f"level {l}: cmap"
            assert lv.matched == wl["matched"] and lv.rounds == wl["rounds"], f"level {l}"
            r, p, d = H.round_stats(l)
            kk = min(r, 64)
            assert p.tolist() == wl["round_active"][:kk], f"level {l}: round activity"
            assert d.tolist() == wl["round_degree"][:kk], f"level {l}: round degrees"
        print(f"level {l}: n={wg['n']} equal", flush=True)
    part0, res = K.kappa_uncoarsen(H, 256, 1, 3, 100)
    assert _sha(part0.cpu().numpy(), np.int32) == want["levels"][0]["part"]
    for l, wl in enumerate(want["levels"]):
        assert list(res[l].as_tuple()) == wl["cut_balance"], f"level {l}: cut/balance"
    print("uncoarsen: level-0 partition and every cut/balance equal", flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(900)
def test_batch_4096_every_graph():
    """The batched workload at full size (4096 uneven graphs, one union, one
    kappa_coarsen_batch call): every graph's hierarchy (every level's CSR,
    map, |M| and stop reason) and its way back up (k = 8) against the
    oracle's run on that graph alone.  The oracle runs in worker processes
    over the host's cores while the GPU side is extracted."""
    import math
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    import paper_0910_2004_amd as K
    from oracle_digest import batch_member_digest, digest
    from workloads import batch_graphs

    count, seed, wmax, stop_n, k = 4096, 4, 16, 256, 8
    workers = min(16, os.cpu_count() or 1)
    top = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(top.uniform(math.log(1e3), math.log(6.4e4), size=count))).astype(np.int64)
    jobs = [(seed, g, int(sizes[g]), wmax, O.EXPANSION_STAR2, 4, stop_n, k) for g in range(count)]
    pool = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))
    futs = pool.map(batch_member_digest, jobs, chunksize=32)
    graphs = batch_graphs(count, seed=seed, workers=workers)   # the same members as the jobs
    du, off = K.DeviceGraph.union(graphs)
    print(f"batch n={du.n} nnz={du.nnz}", flush=True)
    B = K.kappa_coarsen_batch(du, off, O.EXPANSION_STAR2, 4, stop_n)
    got = []
    for g in range(count):
        H = B.hierarchy(g)
        lvls = []
        for l in range(len(H)):
            lv = H.level(l)
            x, a, e, v = lv.graph.numpy()
            lvls.append((int(lv.graph.n), int(x[-1]) if len(x) else 0, digest(x, np.int64),
                         digest(a, np.int32), digest(e, np.uint32), digest(v, np.uint32),
                         None if lv.cmap is None else digest(lv.cmap.cpu().numpy(), np.int32),
                         int(lv.matched), int(lv.stop_reason)))
        part0, res = K.kappa_uncoarsen(H, k, 1, 3, 100)
        got.append((lvls, digest(part0.cpu().numpy(), np.int32),
                    [tuple(int(t) for t in r.as_tuple()) for r in res]))
        del H
    print("GPU side extracted", flush=True)
    bad = []
    for g, want in enumerate(futs):
        if got[g] != want:
            bad.append(g)
    pool.shutdown()
    assert not bad, f"{len(bad)} graphs differ from the oracle, first {bad[:10]}"
    print(f"all {count} graphs equal the oracle", flush=True)
