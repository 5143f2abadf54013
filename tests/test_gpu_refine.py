"""Pairwise refinement of Section 5 on the GPU (kappa_refine,
kappa_uncoarsen_refined) against the oracle's refine / uncoarsen_refined:
the refined partition, the statistics and every level's cut and balance,
bit-exact."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import dev
from workloads import csr_from_edges, grid2d, random_graph, rgg, rmat, star_graph

pytestmark = pytest.mark.gpu

STAT_KEYS = ("global_iterations", "searches", "moves", "kept", "adoptions", "colours")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    K.lib()
    yield
    torch.cuda.synchronize()


def oracle_params(preset, seed):
    d = K.REFINE_PRESETS[preset]
    return O.RefineParams(seed=seed, **d)


def check_refine(g, part, k, preset="fast", seed=1, eps=(3, 100), what="", **over):
    import torch
    prm = oracle_params(preset, seed)
    for key, v in over.items():
        setattr(prm, key, v)
    want, wst = O.refine(g, part, k, eps[0], eps[1], prm)
    p = torch.from_numpy(np.ascontiguousarray(part, dtype=np.int32)).cuda()
    st = K.kappa_refine(dev(g), p, k, eps[0], eps[1], preset, seed, **over)
    got = p.cpu().numpy()[:g.n]
    assert np.array_equal(got, want), f"{what}: partition differs ({(got != want).sum()} nodes)"
    assert st.pop("bytes") >= 0 and st.pop("init_ticks") >= 0 and st.pop("move_ticks") >= 0
    assert st == wst, f"{what}: stats {st} != {wst}"
    return want, wst


def test_hand_worked_two_triangles():
    g = csr_from_edges(6, np.array([0, 0, 1, 2, 3, 3, 4]), np.array([1, 2, 2, 3, 4, 5, 5]))
    part = np.array([0, 0, 1, 0, 1, 1], np.int32)
    out, st = check_refine(g, part, 2, what="two triangles")
    assert out.tolist() == [0, 0, 0, 1, 1, 1] and st["adoptions"] == 1


def test_hand_worked_maxload():
    g = csr_from_edges(5, np.array([4, 4, 0, 1, 2]), np.array([0, 1, 1, 2, 3]),
                       w=np.array([5, 5, 1, 1, 1]))
    part = np.array([0, 0, 0, 0, 1], np.int32)
    out, _ = check_refine(g, part, 2, eps=(0, 1), what="maxload", alpha_num=1, alpha_den=20)
    assert out.tolist() == [1, 1, 0, 0, 1]


def cases():
    return [("grid40x50", grid2d(40, 50)),
            ("rnd-weighted", random_graph(3000, 12000, seed=7, wmax=30, cmax=6, cmin=0)),
            ("rgg2^13", rgg(1 << 13, seed=9)),
            ("rmat11", rmat(11, 8, seed=4, wseed=5, wmax=20)),
            ("star300", star_graph(300))]


@pytest.mark.parametrize("preset", ["minimal", "fast", "strong"])
@pytest.mark.parametrize("k", [2, 5, 16, 64])
def test_random_partitions_equal_oracle(preset, k):
    for name, g in cases():
        rng = np.random.default_rng(k * 7 + len(name))
        part = rng.integers(0, k, g.n).astype(np.int32)
        say(name, "k", k, preset)
        check_refine(g, part, k, preset, seed=k + 3, what=f"{name} k={k} {preset}")


def test_blocky_partitions_and_eps():
    # contiguous id ranges on an rgg (few boundary nodes, a sparse Q) and an
    # unbalanced start with several eps
    g = rgg(1 << 14, seed=12)
    for k in (4, 32, 256):
        part = (np.arange(g.n) * k // g.n).astype(np.int32)
        for eps in ((3, 100), (0, 1), (1, 1)):
            check_refine(g, part, k, "strong", seed=5, eps=eps, what=f"blocks k={k} eps={eps}")
    part = np.zeros(g.n, np.int32)
    part[: g.n // 10] = 1
    check_refine(g, part, 2, "fast", what="unbalanced")


def test_degenerate_and_errors():
    import torch
    g = grid2d(8, 8)
    d = dev(g)
    one = torch.zeros(64, dtype=torch.int32, device="cuda")
    st = K.kappa_refine(d, one, 1)
    assert st["searches"] == 0 and (one == 0).all()
    empty = csr_from_edges(0, np.zeros(0, np.int64), np.zeros(0, np.int64))
    st = K.kappa_refine(dev(empty), torch.zeros(1, dtype=torch.int32, device="cuda"), 4)
    wst = O.refine(empty, np.zeros(0, np.int32), 4)[1]
    assert st.pop("bytes") == 0 and st.pop("init_ticks") == 0 and st.pop("move_ticks") == 0
    assert st == wst
    part = np.random.default_rng(1).integers(0, 4, 64).astype(np.int32)
    check_refine(g, part, 4, max_global=0, what="no global iteration")
    bad = torch.from_numpy(part.copy()).cuda()
    bad[5] = 4
    before = bad.clone()
    with pytest.raises(K.KappaError) as e:
        K.kappa_refine(d, bad, 4)
    assert e.value.status == K.E_RANGE and torch.equal(bad, before)
    p = torch.from_numpy(part).cuda()
    for kw in (dict(alpha_den=0), dict(depth=-1), dict(max_local=0), dict(max_global=-1),
               dict(stop_after=0)):
        with pytest.raises(K.KappaError) as e:
            K.kappa_refine(d, p, 4, **kw)
        assert e.value.status == K.E_ARG, kw
    for k in (0, 257):
        with pytest.raises(K.KappaError) as e:
            K.kappa_refine(d, p, k)
        assert e.value.status == K.E_ARG


@pytest.mark.parametrize("k", [8, 64])
def test_uncoarsen_refined_equals_oracle(k):
    g = rgg(1 << 15, seed=21)
    H = K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 42, 20 * k)
    OH = O.coarsen(g, O.EXPANSION_STAR2, 42, 20 * k)
    assert len(H) == len(OH.levels)
    prm = oracle_params("fast", 3)
    parts, res, stats = O.uncoarsen_refined(OH, k, 1, 3, 100, prm)
    part0, got, gst = K.kappa_uncoarsen_refined(H, k, 1, 3, 100, "fast", 3)
    assert np.array_equal(part0.cpu().numpy(), parts[0])
    for l in range(len(res)):
        assert got[l].as_tuple() == res[l].as_tuple(), l
        assert gst[l].pop("bytes") > 0 or stats[l]["searches"] == 0
        gst[l].pop("init_ticks"), gst[l].pop("move_ticks")
        assert gst[l] == stats[l], l
    say(f"rgg 2^15 k={k}: cut {res[0].cut}, levels {len(res)}")


@pytest.mark.parametrize("qcap", [0, 1, 7, 100])
def test_queue_entries_in_memory(qcap, monkeypatch):
    # the kernel keeps the first queue entries of a search on chip and the rest
    # in memory; a small on-chip capacity sends most entries through memory
    monkeypatch.setenv("KAPPA_REFINE_QCAP", str(qcap))
    for name, g in cases()[:3]:
        for k in (2, 16):
            part = np.random.default_rng(k + qcap).integers(0, k, g.n).astype(np.int32)
            check_refine(g, part, k, "strong", seed=qcap, what=f"{name} k={k} qcap={qcap}")


@pytest.mark.timeout(600)
def test_full_size_refined_way_back_up_equals_oracle():
    # the workload the benchmark times (rgg 2^20, expansion*2 hierarchy, k = 64,
    # preset fast, refinement seed 1): the level-0 partition, every level's
    # cut/balance and every level's search statistics against the oracle's
    # way back up (about 40 s on one host core)
    g = rgg(1 << 20, seed=2)
    H = K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 42, 20 * 64)
    OH = O.coarsen(g, O.EXPANSION_STAR2, 42, 20 * 64)
    parts, res, stats = O.uncoarsen_refined(OH, 64, 1, 3, 100, oracle_params("fast", 1))
    part0, got, gst = K.kappa_uncoarsen_refined(H, 64, 1, 3, 100, "fast", 1)
    assert np.array_equal(part0.cpu().numpy(), parts[0])
    for l in range(len(res)):
        assert got[l].as_tuple() == res[l].as_tuple(), l
        for key in ("bytes", "init_ticks", "move_ticks"):
            gst[l].pop(key)
        assert gst[l] == stats[l], l
    _, plain = K.kappa_uncoarsen(H, 64, 1, 3, 100)
    assert res[0].cut < plain[0].cut // 2
    say(f"rgg 2^20 k=64 fast: cut {plain[0].cut} -> {res[0].cut}, levels {len(res)}, equal to the oracle")


def test_k256_random_partition():
    # the largest k: a random partition makes Q dense (160 colours here) and
    # every block pair small
    g = rgg(4096, seed=31)
    part = np.random.default_rng(5).integers(0, 256, g.n).astype(np.int32)
    check_refine(g, part, 256, "minimal", seed=2, what="k=256 minimal")
    check_refine(g, part, 256, "fast", seed=3, what="k=256 fast")


@pytest.mark.parametrize("name,make,k", [
    ("rmat12", lambda: rmat(12, 16, seed=7, wseed=8, wmax=50), 16),
    ("grid100", lambda: grid2d(100, 100), 8),
])
def test_uncoarsen_refined_strong_equals_oracle(name, make, k):
    # power-law rows (hubs in the searches) and a mesh, with the strong preset
    g = make()
    H = K.kappa_coarsen(dev(g), O.EXPANSION_STAR2, 42, 20 * k)
    OH = O.coarsen(g, O.EXPANSION_STAR2, 42, 20 * k)
    prm = oracle_params("strong", 4)
    parts, res, stats = O.uncoarsen_refined(OH, k, 1, 3, 100, prm)
    part0, got, gst = K.kappa_uncoarsen_refined(H, k, 1, 3, 100, "strong", 4)
    assert np.array_equal(part0.cpu().numpy(), parts[0]), name
    for l in range(len(res)):
        assert got[l].as_tuple() == res[l].as_tuple(), (name, l)
        for key in ("bytes", "init_ticks", "move_ticks"):
            gst[l].pop(key)
        assert gst[l] == stats[l], (name, l)
    say(f"{name} k={k} strong: cut {res[0].cut}")


def test_more_blocks_than_nodes():
    # k > n: most blocks are empty, Q covers only the occupied ones
    g = random_graph(30, 80, seed=12, wmax=5, cmax=3, cmin=0)
    for k in (64, 256):
        part = np.random.default_rng(k).integers(0, k, g.n).astype(np.int32)
        for preset in ("minimal", "strong"):
            check_refine(g, part, k, preset, seed=k, what=f"k={k} {preset}")
