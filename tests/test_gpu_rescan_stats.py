"""Rescan statistics (kappa_hierarchy_rescan_stats).  A later round's
pending nodes pointed in the round before, so every count is bounded by the
previous round's pointing nodes.  Without chunked rows the pick scans every
pending row, so the count also covers the round's own pointing nodes; on a
power-law graph (long rows in chunks) only the nodes whose choice was
matched away scan again."""
import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import dev
from workloads import rgg, rmat

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def profiling():
    """The rescan statistics are recorded while the profiler is on."""
    K.profile_enable(True)
    yield
    K.profile_enable(False)
    K.profile_reset()


def test_every_pending_row_without_chunks():
    g = rgg(1 << 15, seed=5)
    assert int(np.diff(g.xadj).max()) <= 1024   # no chunked rows
    H = K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 7, 64)
    for l in range(len(H) - 1):
        r, p, d = H.round_stats(l)
        r2, rr, rd = H.rescan_stats(l)
        assert r == r2 and r > 0
        assert rr[0] == 0 and rd[0] == 0   # the first round scans every row
        for i in range(1, min(r, len(p))):
            assert p[i] <= rr[i] <= p[i - 1] and d[i] <= rd[i] <= d[i - 1], f"level {l} round {i + 1}"


def test_bounded_by_round_stats_with_chunks():
    g = rmat(16, 16, seed=9, wseed=10)
    assert int(np.diff(g.xadj).max()) > 1024   # chunked rows
    H = K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 7, 512)
    total = 0
    for l in range(len(H) - 1):
        inf = H.info(l)
        r, p, d = H.round_stats(l)
        _, rr, rd = H.rescan_stats(l)
        assert len(rr) == len(p)
        assert rr[0] == 0 and rd[0] == 0   # the first round scans every row
        for i in range(1, min(int(inf.grid_rounds), len(p))):
            assert 0 <= rr[i] <= p[i - 1] and 0 <= rd[i] <= d[i - 1], f"level {l} round {i + 1}"
            assert rd[i] >= rr[i]   # a pointing node has a neighbour
        total += int(rr.sum())
    assert total > 0


def test_zero_without_the_profiler():
    K.profile_enable(False)
    g = rmat(14, 16, seed=9, wseed=10)
    H = K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 7, 256)
    for l in range(len(H) - 1):
        _, rr, rd = H.rescan_stats(l)
        assert not rr.any() and not rd.any()
