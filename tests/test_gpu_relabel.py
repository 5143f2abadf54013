"""The locality relabelling on the device (kappa_rcb_order, kappa_relabel)
against the oracle's reference (oracle.rcb.rcb_order, oracle.rcb.relabel), and the
whole hierarchy of a device-relabelled graph against the oracle on the host-
relabelled one: the relabelling is exact, so the comparison is bit-exact."""
import sys

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import check_hierarchy, dev, graph_np
from oracle.rcb import rcb_order, relabel
from workloads import grid2d, rgg, rgg_points, rmat, star_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_order(pts, leaf):
    import torch
    xy = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
    return K.kappa_rcb_order(xy, leaf).cpu().numpy()


@pytest.mark.parametrize("n", [0, 1, 2, 5, 33, 1000, 1 << 16])
@pytest.mark.parametrize("leaf", [1, 8, 32, 5000])
def test_rcb_order_equals_host(n, leaf):
    pts = rgg_points(n, 100 + n)
    assert np.array_equal(dev_order(pts, leaf), rcb_order(pts, leaf))


def test_rcb_order_ties_signs_and_size():
    rng = np.random.default_rng(7)
    # many equal coordinates (a lattice), negative values and both zeros
    g = np.stack(np.meshgrid(np.arange(40), np.arange(25), indexing="ij"), -1).reshape(-1, 2)
    pts = np.concatenate([g.astype(np.float64) - 20.0, rng.normal(size=(300, 2)),
                          np.array([[0.0, -0.0], [-0.0, 0.0], [-0.0, -0.0]])])
    pts = pts[rng.permutation(len(pts))]
    for leaf in (1, 3, 16):
        assert np.array_equal(dev_order(pts, leaf), rcb_order(pts, leaf)), leaf
    pts = rgg_points(1 << 20, 2)
    assert np.array_equal(dev_order(pts, 32), rcb_order(pts, 32))


@pytest.mark.parametrize("name,make", [
    ("rgg2^15", lambda: rgg(1 << 15, seed=5)),
    ("rmat12", lambda: rmat(12, 16, seed=6, wseed=7)),
    ("grid30x40", lambda: grid2d(30, 40)),
    ("star500", lambda: star_graph(500)),
])
def test_relabel_equals_host(name, make):
    g = make()
    for s in range(2):
        perm = np.random.default_rng(s).permutation(g.n).astype(np.int32)
        import torch
        got = graph_np(K.kappa_relabel(dev(g), torch.from_numpy(perm).cuda()))
        want = relabel(g, perm)
        assert np.array_equal(got.xadj, want.xadj), name
        assert np.array_equal(got.adj, want.adj), name
        assert np.array_equal(got.ew, want.ew), name
        assert np.array_equal(got.vw, want.vw), name


def test_relabel_rejects_non_permutations():
    import torch
    g = grid2d(10, 10)
    d = dev(g)
    for bad in (np.zeros(100, np.int32), np.arange(1, 101, dtype=np.int32)):
        with pytest.raises(K.KappaError) as e:
            K.kappa_relabel(d, torch.from_numpy(bad).cuda())
        assert e.value.status == K.E_ARG


@pytest.mark.parametrize("rating", [O.EXPANSION_STAR2, O.INNER_OUTER])
def test_device_relabelled_hierarchy_equals_oracle(rating):
    import torch
    n = 1 << 17
    pts = rgg_points(n, 21)
    g = rgg(n, seed=21)
    order = K.kappa_rcb_order(torch.from_numpy(pts).cuda(), 32)
    dr = K.kappa_relabel(dev(g), order)
    host = relabel(O.Graph.of(rgg(n, seed=21)), rcb_order(pts))
    say(f"rgg 2^17: device order equals host: {np.array_equal(order.cpu().numpy(), rcb_order(pts))}")
    check_hierarchy(host, rating, 42, stop_n=20 * 64, k=64, dg=dr)
