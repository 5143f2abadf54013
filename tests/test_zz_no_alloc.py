"""The allocation-free cut/balance entry point against kappa_cut_balance on
the same inputs, two calls in a row on one GPU, the second on a smaller
graph (the shared scratch keeps the first call's contents)."""
import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import dev
from workloads import grid2d, rmat

pytestmark = pytest.mark.gpu


def _both(g, part, k):
    import torch
    dg = dev(g)
    pt = torch.from_numpy(part).to("cuda")
    want, bw_want = K.kappa_cut_balance(dg, pt, k, 3, 100)
    bw = torch.full((k,), -1, dtype=torch.int64, device="cuda")
    got = K.kappa_cut_balance_noalloc(dg, pt, k, 3, 100, block_w=bw)
    torch.cuda.synchronize()
    assert got.as_tuple() == want.as_tuple()
    assert np.array_equal(bw.cpu().numpy(), bw_want.cpu().numpy())
    assert got.as_tuple() == O.cut_balance(g, part, k, 3, 100).as_tuple()
    return got


def test_noalloc_equals_cut_balance_twice_second_smaller():
    rng = np.random.default_rng(7)
    g1 = rmat(14, 16, seed=5, wseed=6)
    p1 = rng.integers(0, 256, size=g1.n).astype(np.int32)
    r1 = _both(g1, p1, 256)
    g2 = grid2d(20, 30)
    p2 = rng.integers(0, 3, size=g2.n).astype(np.int32)
    r2 = _both(g2, p2, 3)
    assert r1.cut != r2.cut


def test_noalloc_block_w_null_and_bad_block_id():
    import torch
    g = grid2d(8, 8)
    part = np.zeros(g.n, dtype=np.int32)
    part[5] = 2
    dg = dev(g)
    got = K.kappa_cut_balance_noalloc(dg, torch.from_numpy(part).to("cuda"), 3, 3, 100)
    assert got.as_tuple() == O.cut_balance(g, part, 3, 3, 100).as_tuple()
    part[7] = 3   # outside [0, k)
    with pytest.raises(K.KappaError):
        K.kappa_cut_balance_noalloc(dg, torch.from_numpy(part).to("cuda"), 3, 3, 100)
    # the next call after the rejected one starts from cleared scratch
    part[7] = 1
    got = K.kappa_cut_balance_noalloc(dg, torch.from_numpy(part).to("cuda"), 3, 3, 100)
    assert got.as_tuple() == O.cut_balance(g, part, 3, 3, 100).as_tuple()
