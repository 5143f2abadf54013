"""The one-workgroup tail: once a level has at most 16384 nodes and 131072
entries, kappa_coarsen can run it and every later level in a single
workgroup (kappa_tail_enable).  With the tail on and off (the default), every
hierarchy must equal the
oracle's, round statistics included; the levels the tail ran report no
grid-launched rounds, and with the tail off every matched level reports at
least one."""
import sys

import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import check_hierarchy
from workloads import grid2d, random_graph, rgg, rmat, star_graph

pytestmark = pytest.mark.gpu

TAIL_N, TAIL_NNZ = 16384, 131072


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture
def tail_switch():
    yield K.tail_enable
    K.tail_enable(False)


CASES = [
    ("rgg2^15", lambda: rgg(1 << 15, seed=11), 40),
    ("rgg2^17", lambda: rgg(1 << 17, seed=12), 128),
    ("grid200", lambda: grid2d(200, 200), 64),
    ("rmat13", lambda: rmat(13, 16, seed=5, wseed=6), 64),
    ("star6000", lambda: star_graph(6000), 8),
    ("random", lambda: random_graph(20000, 60000, seed=7, wmax=9, cmax=4, cmin=0), 32),
]


@pytest.mark.parametrize("rating", [O.EXPANSION_STAR2, O.INNER_OUTER, O.EXPANSION_STAR])
@pytest.mark.parametrize("name,make,stop_n", CASES, ids=[c[0] for c in CASES])
def test_tail_on_and_off_equal_oracle(name, make, stop_n, rating, tail_switch):
    g = make()
    OH = O.coarsen(g, rating, 42, stop_n, 1, 20, 64, round_stats=True)
    for on in (True, False):
        tail_switch(on)
        H, _ = check_hierarchy(g, rating, 42, stop_n, k=8, oracle_h=OH)
        grid = [int(H.info(l).grid_rounds) for l in range(len(H))]
        rounds = [int(H.info(l).rounds) for l in range(len(H))]
        say(f"{name} rating {rating} tail {on}: n {[H.info(l).n for l in range(len(H))]} "
            f"rounds {rounds} grid rounds {grid}")
        first = None   # first level past 0 that fits the tail
        for l in range(1, len(H)):
            inf = H.info(l)
            if inf.n <= TAIL_N and inf.nnz <= TAIL_NNZ:
                first = l
                break
        for l in range(len(H) - 1):
            if rounds[l] == 0:
                continue
            if on and first is not None and l >= first:
                assert grid[l] == 0, f"level {l} should have run in the tail"
            else:
                assert grid[l] >= 1, f"level {l} ran no grid round"
