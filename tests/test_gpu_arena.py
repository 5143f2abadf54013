"""Arena overflow and retry.  All levels of a call live in one device arena
that the level kernels bump-allocate from; a level whose arrays do not fit
ends the level loop and the call starts again with four times the arena.
With the first attempt's arena set to end inside each allocation group in
turn (a level's node arrays, then its edge arrays), at levels whose scans run
in one workgroup and at levels that use the two-kernel scan, every result
must still equal the oracle's."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import check_hierarchy, compare_hierarchy
from workloads import grid2d, rgg, rmat, star_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _al(x):
    return (x + 255) // 256 * 256


def _group_ends(level_sizes, count=0):
    """Arena offsets at which each allocation group ends, in the arena's
    layout: level 0's mate and cmap (and, batched, graph ids and offsets)
    first; then for every built level its node arrays (c, xadj, mate, cmap,
    and batched graph ids and offsets) and its edge arrays (adj, ew)."""
    n0 = level_sizes[0][0]
    cur = 3 * _al(4 * n0) + _al(4 * (count + 1)) if count else 2 * _al(4 * n0)
    ends = []
    for nc, ec in level_sizes[1:]:
        node = [4 * nc, 8 * (nc + 1), 4 * nc, 4 * nc] + ([4 * nc, 4 * (count + 1)] if count else [])
        for group in (node, [4 * ec, 4 * ec]):
            for b in group:
                cur = _al(cur) + max(b, 1)
            ends.append(cur)
    return ends


@pytest.fixture
def tight_arena():
    yield K.arena_first
    K.arena_first(0)


CASES = [
    # (name, graph, rating, stop_n): every level of the first one scans in one
    # workgroup; the second's level 0 uses the two-kernel scan; the third has
    # rows above the mid-row size (hub accumulators)
    ("rgg3000", lambda: rgg(3000, seed=5), O.EXPANSION_STAR2, 20),
    ("grid160", lambda: grid2d(160, 160), O.INNER_OUTER, 40),
    ("rmat12", lambda: rmat(12, 16, seed=3, wseed=4), O.INNER_OUTER, 40),
]


@pytest.mark.parametrize("name,make,rating,stop_n", CASES, ids=[c[0] for c in CASES])
def test_retry_after_overflow_at_every_group(name, make, rating, stop_n, tight_arena):
    g = make()
    OH = O.coarsen(g, rating, 42, stop_n, 1, 20, 64, round_stats=True)
    sizes = [(lv.graph.n, int(lv.graph.xadj[-1])) for lv in OH.levels]
    ends = _group_ends(sizes)
    say(f"{name}: n={g.n} levels={len(sizes)} group ends={ends}")
    for cut in ends:
        say(f"first-attempt arena {cut - 1}")
        tight_arena(cut - 1)
        check_hierarchy(g, rating, 42, stop_n, k=4, oracle_h=OH)
    tight_arena(0)
    check_hierarchy(g, rating, 42, stop_n, k=4, oracle_h=OH)


def test_batch_retry_after_overflow(tight_arena):
    graphs = [rgg(3000, seed=5), grid2d(40, 41), rmat(10, 8, seed=13, wseed=14), star_graph(500),
              grid2d(90, 90)]
    stop = [20, 16, 30, 8, 50]
    OHs = [O.coarsen(G, O.EXPANSION_STAR, 42, stop[i], 1, 20, 64) for i, G in enumerate(graphs)]
    du, off = K.DeviceGraph.union(graphs)
    n0, e0 = du.n, du.nnz
    full = 3 * (28 * n0 + 8 * e0)
    cuts = sorted(set(int(x) for x in np.geomspace(3 * _al(4 * n0) + 256, full, 14)))
    say(f"batch n={n0} nnz={e0}, first-attempt arenas {cuts}")
    for cut in cuts + [0]:
        tight_arena(cut)
        B = K.kappa_coarsen_batch(du, off, O.EXPANSION_STAR, seed=42, stop_n=stop)
        for i, OH in enumerate(OHs):
            assert B.info(i) == (len(OH.levels), OH.levels[-1].stop_reason), f"arena {cut} graph {i}"
            compare_hierarchy(B.hierarchy(i), OH, check_rounds=False, check_uncoarsen=(i == 0), k=4)
        del B
