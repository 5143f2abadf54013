"""Measures the library's tuning table (kappa_tuning) on this GPU and writes
it as kappa_tuning.txt, which the library reads when it loads (see
include/kappa.h).

    python -m paper_0910_2004_amd.autotune [--out PATH] [--reps N]

Workloads (seeded, synthetic, built before any timing):
  * rgg 2^20, mean degree 8, expansion*2 and innerOuter, stop 1280 (mesh-like
    and geometric levels: many small rows, long matching tails);
  * R-MAT scale 20, edge factor 16, expansion*2, stop 5120 (power-law levels:
    hubs, handed-back matching levels, the large-row merges);
  * the batched form over 512 uneven graphs (n log-uniform in [1e3, 6.4e4]),
    expansion*2, stop 256 per graph (a union with per-graph stop rules).
Coordinate descent: each field in turn, every candidate value is timed (the
median of `reps` runs of every workload, summed over the workloads) with the
other fields at their best so far, and kept if it beats the current value by
more than 1 %; two sweeps over the fields.  Every timed run is checked
against the compiled defaults' result (level sizes and a checksum of every
level): a table never changes a result, and a mismatch stops the tuner.
"""
from __future__ import annotations

import argparse
import math
import os
import statistics
import sys
import time

from . import _lib as K

CANDIDATES = {
    "bin_small_max": [4, 8, 16],
    "tail_max": [32, 128, 512, 2048],
    "finish_max": [1024, 4096, 16384],
    "finish_max_big": [16, 64, 256],
    "row_small_max": [16, 32, 64],
    "scan_one_block_max": [4096, 16384, 65536],
    "rounds_base": [2, 3, 4],
    "rounds_n0": [1024, 2048, 4096],
    "rounds_growth": [4, 8, 16],
    "rounds_cap": [6, 8, 12],
}
DEFAULTS = {"bin_small_max": 16, "tail_max": 128, "finish_max": 4096, "finish_max_big": 64,
            "row_small_max": 64, "scan_one_block_max": 16384, "rounds_base": 3, "rounds_n0": 2048,
            "rounds_growth": 8, "rounds_cap": 8}


def _signature(H):
    """Level sizes and per-level sums of the CSR arrays (device reductions)."""
    import torch
    out = []
    for l in range(len(H)):
        g = H.level(l).graph
        sig = [int(g.n), int(g.nnz)]
        for t in (g.xadj, g.adj, g.ew, g.vw):
            sig.append(int(t.to(torch.int64).sum().item()) if t.numel() else 0)
        out.append(tuple(sig))
    return out


def _workloads():
    import torch

    from workloads import batch_graphs, rgg, rmat
    t0 = time.time()
    g1 = K.DeviceGraph.from_csr(rgg(1 << 20, seed=2), "cuda")
    g2 = K.DeviceGraph.from_csr(rmat(20, 16, seed=3, wseed=33), "cuda")
    du, off = K.DeviceGraph.union(batch_graphs(512, seed=4, workers=min(16, os.cpu_count() or 1)),
                                  "cuda")
    torch.cuda.synchronize()
    print(f"workloads built in {time.time() - t0:.1f} s", flush=True)

    def batch_sig(B):
        return [B.info(g) for g in range(len(B))] + \
            [_signature(B.hierarchy(g)) for g in range(0, len(B), 64)]

    # (timed call, signature of its result)
    return {"rgg20 expansion*2": (lambda: K.kappa_coarsen(g1, K.EXPANSION_STAR2, 42, 1280,
                                                         trusted=True), _signature),
            "rgg20 innerOuter": (lambda: K.kappa_coarsen(g1, K.INNER_OUTER, 42, 1280,
                                                        trusted=True), _signature),
            "rmat20": (lambda: K.kappa_coarsen(g2, K.EXPANSION_STAR2, 42, 5120, trusted=True),
                       _signature),
            "batch512": (lambda: K.kappa_coarsen_batch(du, off, K.EXPANSION_STAR2, 4, 256),
                         batch_sig)}


def _time(fn, reps):
    import torch
    ts = []
    res = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return statistics.median(ts) * 1e3, res


def tune(reps: int = 5, sweeps: int = 2, log=print):
    import torch
    torch.cuda.set_device(0)
    wl = _workloads()
    K.tuning_set(DEFAULTS)
    want = {}
    for name, (fn, sig) in wl.items():   # warm-up and the reference results
        fn()
        want[name] = sig(fn())

    def measure(table):
        K.tuning_set(table)
        tot, per = 0.0, {}
        for name, (fn, sig) in wl.items():
            ms, res = _time(fn, reps)
            if sig(res) != want[name]:
                raise RuntimeError(f"{name}: result differs under {table}")
            per[name] = round(ms, 3)
            tot += ms
        return tot, per

    best = dict(DEFAULTS)
    best_t, best_per = measure(best)
    log(f"defaults: {best_t:.2f} ms {best_per}")
    history = []
    for sweep in range(sweeps):
        for field, values in CANDIDATES.items():
            for v in values:
                if v == best[field]:
                    continue
                trial = dict(best, **{field: v})
                if trial["rounds_cap"] < trial["rounds_base"]:
                    continue
                t, per = measure(trial)
                history.append((field, v, round(t, 3)))
                log(f"sweep {sweep} {field}={v}: {t:.2f} ms (best {best_t:.2f})")
                if t < best_t * 0.99:
                    best, best_t, best_per = trial, t, per
    # the defaults again, timed after the sweeps, beside the result
    def_t, def_per = measure(DEFAULTS)
    K.tuning_set(best)
    return best, best_t, best_per, def_t, def_per, history


def write_table(path, best, best_t, best_per, def_t, def_per, history):
    import torch
    dev = torch.cuda.get_device_name(0)
    lines = [f"# kappa tuning table, measured by python -m paper_0910_2004_amd.autotune on {dev}",
             f"# ({time.strftime('%Y-%m-%d')}).  Workloads: rgg 2^20 (both ratings), R-MAT scale "
             "20, the batched form over 512 graphs.",
             f"# total {best_t:.2f} ms with this table, {def_t:.2f} ms with the compiled defaults",
             f"# per workload (ms): this table {best_per}",
             f"#                    defaults   {def_per}",
             "# candidates tried (field, value, total ms): " +
             ", ".join(f"{f}={v}:{t}" for f, v, t in history), ""]
    lines += [f"{k} {best[k]}" for k in K.TUNING_FIELDS]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(K.LIB_PATH), "kappa_tuning.txt"))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sweeps", type=int, default=2)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    best, best_t, best_per, def_t, def_per, history = tune(args.reps, args.sweeps)
    write_table(args.out, best, best_t, best_per, def_t, def_per, history)
    print(f"wrote {args.out}: {best} ({best_t:.2f} ms against {def_t:.2f} ms with the defaults)",
          flush=True)
    return 0 if math.isfinite(best_t) else 1


if __name__ == "__main__":
    sys.exit(main())
