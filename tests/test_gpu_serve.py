"""Served form: every request's result (hierarchy, stop reason, level-0
cut and balance) is the same when served inside concurrent batches as when
served alone, one kappa_coarsen call at a time."""
import sys

import numpy as np
import pytest

import paper_0910_2004_amd as K
from gpu_util import assert_graph_equal, graph_np
from paper_0910_2004_amd.serve import BatchServer, Request, latency_stats, serve_plain
from workloads import serve_requests

pytestmark = pytest.mark.gpu


def _requests(count, spread, seed=5):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(spread, size=count)) if spread > 0 else np.zeros(count)
    return [Request(i, g, rating, k, arrival=float(t[i]))
            for i, (g, rating, k) in enumerate(serve_requests(count, seed=seed, emax=2e5))]


def _same(a, b):
    assert (a.levels, a.stop_reason, a.cut) == (b.levels, b.stop_reason, b.cut), f"request {a.rid}"
    Ha, Hb = a.hierarchy, b.hierarchy
    for l in range(len(Ha)):
        x, y = Ha.level(l), Hb.level(l)
        assert_graph_equal(graph_np(x.graph), graph_np(y.graph), f"request {a.rid} level {l}")
        if y.cmap is not None:
            assert np.array_equal(x.cmap.cpu().numpy(), y.cmap.cpu().numpy())


@pytest.mark.parametrize("spread", [0.0, 0.002])
def test_served_equals_alone(spread):
    reqs = _requests(40, spread)
    print(f"{len(reqs)} requests, mean gap {spread * 1e3} ms", flush=True)
    served = BatchServer(workers=2).run(reqs, keep=True)
    alone = serve_plain(reqs, keep=True)
    assert [r.rid for r in served] == [r.rid for r in alone] == list(range(len(reqs)))
    for a, b in zip(served, alone):
        _same(a, b)
    st = latency_stats(reqs, served)
    print(st, flush=True)
    sys.stdout.flush()
    if spread == 0.0:
        assert max(r.batch for r in served) > 1   # requests were mixed


def test_budget_splits_batches():
    reqs = _requests(12, 0.0, seed=6)
    served = BatchServer(workers=1, budget_bytes=1).run(reqs)
    assert all(r.batch == 1 for r in served)   # one request per batch under a tiny budget


def test_kept_hierarchies_count_against_the_device_budget():
    """Hierarchies kept on the device hold their share of the device budget
    until released: a second run that does not fit next to them fails with
    MemoryError instead of waiting forever, and runs once they are released."""
    from paper_0910_2004_amd.serve import footprint, kept_bytes
    reqs = _requests(6, 0.0, seed=7)
    big = max(reqs, key=lambda r: footprint(r.graph))
    budget = footprint(big.graph) + sum(kept_bytes(r.graph) for r in reqs) - 1
    srv = BatchServer(workers=1, hbm_budget=budget)
    first = srv.run(reqs, keep=True)
    assert all(r.hierarchy is not None for r in first)
    again = [Request(100, big.graph, big.rating, big.k)]
    with pytest.raises(MemoryError):
        srv.run(again, keep=True)
    for r in first:
        srv.release(r)
    out = srv.run(again)
    assert out[0].rid == 100
