"""Host logic of the served forms (no GPU): how BatchServer's dispatcher
forms a batch out of the requests that have arrived, and how LevelServer's
threads hand requests through upload, admission, steps and the way back up."""
import numpy as np

from paper_0910_2004_amd.serve import WEIGHT_CAP, Request, footprint, take_batch, weight_sums
from workloads import CSR, grid2d, path_graph


def _heavy(n, w):
    """A path on n nodes with every edge weight w and every node weight 1."""
    g = path_graph([1] * (n - 1))
    return CSR(g.n, g.xadj, g.adj, np.full(len(g.adj), w, np.uint32), g.vw)


def test_weight_sums():
    g = grid2d(3, 4)   # 17 edges of weight 1, 12 nodes of weight 1
    assert weight_sums(g) == (17, 12)
    h = _heavy(5, 7)
    assert weight_sums(h) == (4 * 7, 5)


def test_batch_keeps_rating_seed_and_order():
    g = grid2d(4, 4)
    reqs = [Request(0, g, 0, 2), Request(1, g, 1, 2), Request(2, g, 0, 2), Request(3, g, 0, 2, seed=7),
            Request(4, g, 0, 8)]
    batch, rest = take_batch(reqs, 1 << 40, 512, {})
    assert [r.rid for r in batch] == [0, 2, 4]
    assert [r.rid for r in rest] == [1, 3]


def test_batch_limits():
    g = grid2d(10, 10)
    reqs = [Request(i, g, 0, 2) for i in range(6)]
    fp = footprint(g)
    batch, rest = take_batch(reqs, 3 * fp, 512, {})
    assert len(batch) == 3 and len(rest) == 3
    batch, rest = take_batch(reqs, 1, 512, {})          # a tiny budget: one at a time
    assert [r.rid for r in batch] == [0]
    batch, rest = take_batch(reqs, 1 << 40, 4, {})
    assert len(batch) == 4


def test_batch_union_weight_sums_fit_32_bits():
    w = (WEIGHT_CAP // 3) // 9 + 1        # 9 edges: each graph holds a bit over a third of the cap
    g = _heavy(10, w)
    assert 3 * weight_sums(g)[0] > WEIGHT_CAP >= 2 * weight_sums(g)[0]
    reqs = [Request(i, g, 0, 2) for i in range(5)]
    batch, rest = take_batch(reqs, 1 << 40, 512, {})
    assert [r.rid for r in batch] == [0, 1]
    assert sum(weight_sums(r.graph)[0] for r in batch) <= WEIGHT_CAP


# ---------------------------------------------------------------------------
# LevelServer's threads (uploaders, engines, finishers) against a stand-in
# library: every request of every class completes exactly once, in the right
# engine, under any device budget, and a failing step is raised, not hung.
# ---------------------------------------------------------------------------
class _FakeServer:
    """Stand-in for K.Server: a request lives a fixed number of steps."""
    log = []
    fail_at = 0

    def __init__(self, rating, seed, trusted=False, device=None):
        self.rating, self.seed = rating, seed
        self.act, self.done, self.nid, self.steps = {}, set(), 0, 0

    def admit(self, dg, stop):
        i = self.nid
        self.nid += 1
        self.act[i] = 1 + dg.n % 5
        _FakeServer.log.append((self.rating, self.seed, dg.n))
        return i

    def active(self):
        return len(self.act)

    def interrupt(self, on=True):
        pass

    def step(self):
        self.steps += 1
        if _FakeServer.fail_at and self.steps == _FakeServer.fail_at:
            raise RuntimeError("step failed")
        fin = []
        for i in list(self.act):
            self.act[i] -= 1
            if self.act[i] == 0:
                del self.act[i]
                self.done.add(i)
                fin.append(i)
        return fin

    def take(self, i):
        self.done.remove(i)
        return ("hierarchy", i)


def _fake_level_server(monkeypatch):
    import types

    import torch

    import paper_0910_2004_amd.serve as S

    class _T:
        def record_stream(self, s):
            pass

    class _DG:
        def __init__(self, g):
            self.n = g.n
            self.xadj = self.adj = self.ew = self.vw = _T()

    class _Stream:
        def synchronize(self):
            pass

    class _Ctx:
        def __init__(self, s):
            pass

        def __enter__(self):
            return self

        def __exit__(self, *a):
            return False

    monkeypatch.setattr(torch.cuda, "set_device", lambda i: None)
    monkeypatch.setattr(torch.cuda, "Stream", _Stream)
    monkeypatch.setattr(torch.cuda, "stream", _Ctx)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)
    fake = types.SimpleNamespace(
        DeviceGraph=types.SimpleNamespace(from_csr=lambda g, device: _DG(g)), Server=_FakeServer,
        OK=0, KappaError=RuntimeError, kappa_validate=lambda dg: 0)
    monkeypatch.setattr(S, "K", fake)
    monkeypatch.setattr(S, "_finish", lambda r, H, t0, start, batch, keep: S.Result(
        r.rid, H[1], 0, (0,), start, 0.0, batch, None))
    return S


def test_level_server_threads_complete_every_request(monkeypatch):
    S = _fake_level_server(monkeypatch)
    _FakeServer.fail_at = 0
    gs = [grid2d(4 + i % 9, 3 + i % 4) for i in range(150)] + [grid2d(300, 300)] * 6
    reqs = [Request(i, g, i % 2, 2, arrival=0.0002 * i, seed=42 + i % 3) for i, g in enumerate(gs)]
    for budget in (1 << 40, 1, 3 * footprint(gs[-1])):
        _FakeServer.log = []
        ls = S.LevelServer(hbm_budget=budget, split_entries=1000, max_entries=200000)
        out = ls.run(reqs)
        assert [r.rid for r in out] == list(range(len(reqs)))
        assert len(_FakeServer.log) == len(reqs)   # each admitted once
        # every request went to the engine of its (rating, seed, size class)
        assert set(ls.profile) == {(r.rating, r.seed, r.graph.nnz > 1000) for r in reqs}
        if budget == 1:
            assert all(r.batch == 1 for r in out)   # one request on the device at a time


def test_level_server_raises_a_failed_step(monkeypatch):
    S = _fake_level_server(monkeypatch)
    _FakeServer.fail_at = 2
    g = grid2d(6, 6)
    reqs = [Request(i, g, 0, 2, arrival=0.0) for i in range(20)]
    try:
        S.LevelServer().run(reqs)
    except RuntimeError as e:
        assert "step failed" in str(e)
    else:
        raise AssertionError("the failed step was not raised")
    finally:
        _FakeServer.fail_at = 0
