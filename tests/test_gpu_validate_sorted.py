"""Validation of large graphs (at least 2^22 entries) with rows above 1024
entries: the symmetry test by sorting the entries above the diagonal and
matching them one for one with those below it (large graphs with short rows
keep the binary searches).  Valid graphs pass; every way of breaking
symmetry, order or weights is rejected, as by the binary searches."""
import numpy as np
import pytest

import paper_0910_2004_amd as K
from workloads import CSR, rgg, rmat

pytestmark = pytest.mark.gpu


def _status(g):
    return K.kappa_validate(K.DeviceGraph.from_csr(g, "cuda"))


def _copy(g):
    return CSR(g.n, g.xadj.copy(), g.adj.copy(), g.ew.copy(), g.vw.copy())


def _entry(g, rng, upper):
    """An entry above (or below) the diagonal, with its row."""
    for _ in range(100000):
        v = int(rng.integers(0, g.n))
        a, b = int(g.xadj[v]), int(g.xadj[v + 1])
        if b - a < 3:
            continue
        j = int(rng.integers(a, b))
        if (g.adj[j] > v) == upper:
            return v, j
    raise AssertionError("no such entry")


@pytest.fixture(scope="module")
def big():
    g = rgg(1 << 20, seed=2)
    assert g.xadj[-1] >= (1 << 22)
    return g


@pytest.fixture(scope="module")
def big_weighted():
    g = rmat(18, 16, seed=3, wseed=4)   # weights in [1, 100]; rows above 1024 entries
    assert g.xadj[-1] >= (1 << 22) and int(np.diff(g.xadj).max()) > 1024
    return g


def test_valid_graphs_pass(big, big_weighted):
    assert _status(big) == K.OK
    assert _status(big_weighted) == K.OK


@pytest.mark.parametrize("upper", [True, False])
def test_one_weight_changed(big_weighted, upper):
    rng = np.random.default_rng(5 + upper)
    g = _copy(big_weighted)
    _, j = _entry(g, rng, upper)
    g.ew[j] = g.ew[j] + 1
    assert _status(g) == K.E_GRAPH


@pytest.mark.parametrize("upper", [True, False])
def test_one_neighbour_changed(big_weighted, upper):
    rng = np.random.default_rng(7 + upper)
    g = _copy(big_weighted)
    for _ in range(10000):
        v, j = _entry(g, rng, upper)
        a, b = int(g.xadj[v]), int(g.xadj[v + 1])
        lo = int(g.adj[j - 1]) if j > a else -1
        hi = int(g.adj[j + 1]) if j + 1 < b else g.n
        cands = [x for x in range(lo + 1, hi) if x != v and x != int(g.adj[j])]
        if cands and ((cands[0] > v) == upper):
            g.adj[j] = cands[0]   # still ascending, no self loop: only the symmetry breaks
            break
    else:
        raise AssertionError("no entry to move")
    assert _status(g) == K.E_GRAPH


def test_unsorted_row_and_self_loop(big_weighted):
    rng = np.random.default_rng(9)
    g = _copy(big_weighted)
    v, j = _entry(g, rng, True)
    a = int(g.xadj[v])
    g.adj[a], g.adj[a + 1] = g.adj[a + 1], g.adj[a]
    g.ew[a], g.ew[a + 1] = g.ew[a + 1], g.ew[a]
    assert _status(g) == K.E_GRAPH
    g = _copy(big_weighted)
    v, j = _entry(g, rng, True)
    g.adj[j] = v
    assert _status(g) == K.E_GRAPH


def test_two_rows_swap_weights(big_weighted):
    """Two entries above the diagonal exchange weights: counts and sums stay
    equal, only the pairing breaks."""
    rng = np.random.default_rng(11)
    g = _copy(big_weighted)
    for _ in range(1000):
        _, j1 = _entry(g, rng, True)
        _, j2 = _entry(g, rng, True)
        if g.ew[j1] != g.ew[j2]:
            break
    else:
        raise AssertionError("no two different weights")
    g.ew[j1], g.ew[j2] = g.ew[j2], g.ew[j1]
    assert _status(g) == K.E_GRAPH


def test_large_graph_with_short_rows_keeps_the_searches(big):
    """rgg 2^20 (rows of about 8 entries): the binary searches, rejecting a
    changed weight as well."""
    rng = np.random.default_rng(13)
    g = _copy(big)
    _, j = _entry(g, rng, True)
    g.ew[j] = g.ew[j] + 1
    assert _status(g) == K.E_GRAPH
