"""kappa_set_allocator: with torch's caching allocator installed, the
library's device memory comes from torch's pool (it shows in torch's memory
statistics while a hierarchy lives), every result still equals the oracle's,
and switching back returns the memory."""
import sys

import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import compare_hierarchy, dev
from workloads import grid2d, rgg, rmat

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_torch_allocator_backs_library_memory():
    import torch
    g = rgg(30000, seed=31)
    gs = [grid2d(30, 40), rmat(11, 8, seed=2, wseed=3), rgg(2000, seed=4)]
    OH = O.coarsen(g, O.INNER_OUTER, 42, 64, 1, 20, 64)
    OHs = [O.coarsen(x, O.EXPANSION_STAR2, 42, 32, 1, 20, 64) for x in gs]
    dg = dev(g)
    dgs = [dev(x) for x in gs]
    torch.cuda.synchronize()
    K.use_torch_allocator(True)
    try:
        base = torch.cuda.memory_allocated()
        H = K.kappa_coarsen(dg, O.INNER_OUTER, 42, 64)
        held = torch.cuda.memory_allocated()
        say(f"torch-allocated bytes: {base} before, {held} with a hierarchy alive")
        assert held > base   # the arena and the workspace came from torch's pool
        compare_hierarchy(H, OH, check_rounds=False, k=8)
        B = K.kappa_coarsen_graphs(dgs, O.EXPANSION_STAR2, 42, 32)
        for i, oh in enumerate(OHs):
            compare_hierarchy(B.hierarchy(i), oh, check_rounds=False, k=4)
        del H, B
    finally:
        K.use_torch_allocator(False)   # releases the cache through torch's allocator
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= base
    # and the default allocator again
    H = K.kappa_coarsen(dg, O.INNER_OUTER, 42, 64)
    compare_hierarchy(H, OH, check_rounds=False, k=8)


def test_allocator_arguments():
    import ctypes
    L = K.lib()
    st = L.kappa_set_allocator(K._lib._ALLOC_FN(lambda n, s, c: None), K._lib._FREE_FN(), None)
    assert st == K.E_ARG
