"""Writes rmat22_levels.json: SHA-256 digests of the oracle's whole hierarchy
and way back up for the R-MAT workload of scale 22 (2^22 nodes, 16 * 2^22
samples, (a, b, c) = (0.57, 0.19, 0.19), generator seed 3, weights uniform in
[1, 100] with seed 33, unit node weights), expansion*2 with seed 42, stop at
5120 nodes or on the stall rule 1/20, 64 levels at most; stand-in partition
with k = 256 and seed 1, eps = 3/100.

Only the oracle and the seeded generator run here.  The oracle needs about
five minutes on one host core.  Usage: python tests/golden/make_rmat22.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from workloads import rmat  # noqa: E402


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def graph_digest(g):
    return {"n": int(g.n), "nnz": int(g.xadj[-1]) if g.n else 0,
            "xadj": digest(g.xadj, np.int64), "adj": digest(g.adj, np.int32),
            "ew": digest(g.ew, np.uint32), "vw": digest(g.vw, np.uint32)}


def main():
    t0 = time.time()
    g = rmat(22, 16, seed=3, wseed=33)
    k, stop_n = 256, 5120
    H = O.coarsen(g, O.EXPANSION_STAR2, 42, stop_n, 1, 20, 64, round_stats=True)
    parts, res = O.uncoarsen(H, k, 1, 3, 100)
    levels = []
    for l, lv in enumerate(H.levels):
        rec = {"graph": graph_digest(lv.graph), "stop_reason": int(lv.stop_reason)}
        if lv.cmap is not None:
            rec.update({"cmap": digest(lv.cmap, np.int32), "mate": digest(lv.mate, np.int32),
                        "matched": int(lv.matched), "rounds": int(lv.rounds),
                        "round_active": [int(x) for x in lv.round_active],
                        "round_degree": [int(x) for x in lv.round_degree]})
        rec["part"] = digest(parts[l], np.int32)
        rec["cut_balance"] = [int(x) for x in res[l].as_tuple()]
        levels.append(rec)
    out = {"workload": "R-MAT scale 22, edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), seed 3, "
                       "weights [1, 100] seed 33; expansion*2, seed 42, stop 5120, stall 1/20, "
                       "max 64 levels; stand-in partition k = 256 seed 1, eps 3/100",
           "written_by": "tests/golden/make_rmat22.py (oracle only)",
           "input": graph_digest(g), "levels": levels}
    with open(os.path.join(HERE, "rmat22_levels.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{len(levels)} levels in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
