"""Full-size parity: the benchmark's workload (random geometric graph,
n = 2^20, mean degree 8, unit weights, k = 64, stop at 20k nodes) through the
same entry points and launch configuration bench.py times, compared with the
oracle level by level (every array, map, round count, cut and balance)."""
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
