"""Two hierarchies of one graph built at the same time, one host thread and
one stream each (the benchmark's step): every level, map and the way back up
must equal the oracle's, as when they run one after the other."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
import paper_0910_2004_amd as K
from gpu_util import compare_hierarchy, dev
from workloads import rgg, rmat

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name,make,stop_n,k", [
    ("rgg2^17", lambda: rgg(1 << 17, seed=41), 1280, 64),
    ("rmat14", lambda: rmat(14, 16, seed=42, wseed=43), 512, 16),
])
def test_two_ratings_on_two_streams(name, make, stop_n, k):
    import torch
    g = make()
    ratings = [O.EXPANSION_STAR2, O.INNER_OUTER]
    OH = {r: O.coarsen(g, r, 42, stop_n, 1, 20, 64, round_stats=True) for r in ratings}
    OP = {r: O.uncoarsen(OH[r], k, 1, 3, 100) for r in ratings}
    dg = dev(g)
    assert K.kappa_validate(dg) == K.OK
    streams = [torch.cuda.Stream() for _ in ratings]
    part0s = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in ratings]
    torch.cuda.synchronize()

    def one(i):
        with torch.cuda.stream(streams[i]):
            H = K.kappa_coarsen(dg, ratings[i], 42, stop_n, 1, 20, 64, trusted=True)
            part, res = K.kappa_uncoarsen(H, k, 1, 3, 100, part0=part0s[i])
            torch.cuda.current_stream().synchronize()
            return H, part.cpu().numpy(), [x.as_tuple() for x in res]

    with ThreadPoolExecutor(max_workers=2) as pool:
        for rep in range(3):
            got = [f.result() for f in [pool.submit(one, i) for i in range(2)]]
            for i, r in enumerate(ratings):
                H, part, res = got[i]
                say(f"{name} rep {rep} rating {r}: levels {len(H)}")
                compare_hierarchy(H, OH[r], check_rounds=True, check_uncoarsen=False)
                oparts, ores = OP[r]
                assert np.array_equal(part, oparts[0]), "level-0 partition differs"
                assert res[0] == ores[0].as_tuple(), f"cut/balance {res[0]} != {ores[0].as_tuple()}"
