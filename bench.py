"""Benchmark of the coarsening hierarchy on one MI355X.

The headline step is one pass of the whole path over the R-MAT power-law
graph of scale 22 (2^22 nodes, 16 * 2^22 samples, (a, b, c) = (0.57, 0.19,
0.19), weights uniform in [1, 100], unit node weights): validation of the
input, then matching + contraction level by level with the expansion*2
rating down to 20*k nodes (k=256) or the stall rule, the coarsest-level
partition, then projection and cut/balance on every level back to level 0.
The graph is resident in HBM before the timed region.  The same line carries,
under "secondary", the random geometric graph workload (n = 2^20, mean degree
8, both ratings, k = 64).

Prints one JSON line: edges/s = (undirected input edges per step) / (time per
step), plus the roofline of the dominant kernel (HIP events on the library's
launch stream, in a second timed pass with per-launch events enabled) and the
oracle's time on the host for a bounded sample (cpu_baseline).
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic bytes (element-granular compulsory traffic) of the kernels with
# an exact per-level model.  D = CSR entries (2|E|), n = nodes of the level.
# ---------------------------------------------------------------------------
def bytes_pick_first(n, D, io):
    # per node: row offsets (8), c(v) (4), best[v] (4) [+ Out(v) (4)]
    # per entry: adj (4), w (4), c(u) (4) [+ Out(u) (4)]
    return (20 if io else 16) * n + (16 if io else 12) * D


def bytes_fill_small(n, D, nc, Dc, matched):
    # per coarse row: rep_of, partner (8), offsets of the representative (16),
    # merged degree written (4); matched rows also read the partner's offsets
    # (16).  Per fine entry: adj, w, cmap of the neighbour (12).  Per merged
    # coarse entry: key and weight written (8).
    return 28 * nc + 16 * matched + 12 * D + 8 * Dc


def bytes_compact(nc, Dc):
    # per row: list entry, two offsets, degree (24); per entry: read 8, write 8
    return 24 * nc + 16 * Dc


def bytes_cut_entries(D):
    # per entry: adj, w, part of both ends
    return 16 * D


def bytes_pick_round(A, Dr):
    # a matching round after the first, pick side, over the A nodes that scan
    # their row again (degree sum Dr): per entry adj, w, the neighbour's
    # attribute and mate (16); per node its two int64 offsets, own attribute,
    # best (24)
    return 16 * Dr + 24 * A


def bytes_mate_round(A):
    # mutual check: per pointing node its choice, the choice's choice, mate (12)
    return 12 * A


def bytes_merge(rows, matched, fine_entries, merged_entries):
    # the merge of a row class (the small-row model): per coarse row rep_of,
    # partner, the representative's offsets, merged degree (28); matched rows
    # also the partner's offsets (16); per fine entry adj, w and cmap of the
    # neighbour (12); per merged entry key and weight written (8)
    return 28 * rows + 16 * matched + 12 * fine_entries + 8 * merged_entries


def bytes_validate(n, D):
    # every entry's neighbour and weight (8) and the row offsets and node
    # weights (12 per node); the reverse entry of an entry is another entry
    return 8 * D + 12 * n


# merge kernels by class of the bound deg(u) + deg(w) - 2 on the merged row
MERGE_CLASSES = (("fill_small", 0, 64), ("fill_mid", 65, 4094),
                 ("fill_big", 4095, 16382), ("fill_large", 16383, 1 << 62))


def merge_class_stats(H):
    """Per merge kernel, summed over the levels of H: coarse rows, matched
    rows, fine entries and merged entries (from the levels' offsets and maps,
    copied to the host)."""
    import numpy as np
    tot = {name: [0, 0, 0, 0] for name, _, _ in MERGE_CLASSES}
    L = len(H)
    prev = None
    for l in range(L):
        lv = H.level(l)
        x = lv.graph.xadj.cpu().numpy()
        if prev is not None:
            deg_f, cmap = prev
            nc = len(x) - 1
            deg_c = np.diff(x)
            sumdeg = np.bincount(cmap, weights=deg_f, minlength=nc).astype(np.int64)
            cnt = np.bincount(cmap, minlength=nc)
            bound = sumdeg - 2 * (cnt == 2)
            for name, lo, hi in MERGE_CLASSES:
                m = (bound >= max(lo, 1)) & (bound <= hi)
                t = tot[name]
                if name == "fill_small":
                    # every coarse row passes the small-row kernel (its header is
                    # read there); the entries of the small rows are merged there
                    m = bound <= hi
                    t[0] += nc
                    t[1] += int((cnt == 2).sum())
                else:
                    t[0] += int(m.sum())
                    t[1] += int((m & (cnt == 2)).sum())
                t[2] += int(sumdeg[m].sum())
                t[3] += int(deg_c[m].sum())
        prev = (np.diff(x), lv.cmap.cpu().numpy()) if lv.cmap is not None else None
    return tot


MODELS = {"pick": "per round r >= 2 run as a grid launch: 16 B per entry of the rows that "
                  "scan again in round r (adj, w, attribute, mate of the neighbour) + 24 B per "
                  "such row (int64 offsets, own attribute, best); rows and degree sum from the "
                  "level's rescan statistics (every pending node, unless long rows are "
                  "chunked: then only those whose choice was matched away)",
          "mate": "per round r >= 2 run as a grid launch: 12 B per pointing node",
          "pick_first": "per level: 16 B/node + 12 B/entry (innerOuter 20 + 16)",
          "fill_small": "per level: 28 B/coarse row + 16 B/matched pair + 12 B/fine entry + 8 B/coarse entry",
          "compact": "per level: 24 B/coarse row + 16 B/coarse entry",
          "cut_entries": "per level: 16 B/entry",
          "validate_entries": "8 B per CSR entry (neighbour, weight) + 12 B per node (offsets, "
                              "node weight)"}
for _name, _lo, _hi in MERGE_CLASSES[1:]:
    MODELS[_name] = (f"per level, over the coarse rows whose merged-row bound is {_lo}.."
                     f"{_hi if _hi < (1 << 60) else 'inf'}: 28 B/row + 16 B/matched row + "
                     "12 B/fine entry + 8 B/merged entry")


def counter_traffic(kernel, tag):
    """HBM bytes per launch of `kernel` on workload `tag` (rmat22, rgg20)
    from the committed counter summary (profiles/<kernel>_<tag>_counters.json:
    FETCH_SIZE and WRITE_SIZE per launch, scaled by a plain copy), or None when
    the kernel's source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{tag}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    srcs = counter_sources(kernel)
    if rec.get("sources") != srcs or rec.get("sources_sha256") != _sources_sha(srcs):
        return None
    return rec["traffic_bytes_per_launch"]


def level_stats(H):
    """Per level: n, entries, |M|, rounds, rounds run as grid launches, the
    per-round (pointing nodes, their degree sum) and the per-round (rows
    scanned again, their degree sum)."""
    out = []
    for l in range(len(H)):
        inf = H.info(l)
        _, p, d = H.round_stats(l)
        _, rr, rd = H.rescan_stats(l)
        out.append((int(inf.n), int(inf.nnz), int(inf.matched), int(inf.rounds),
                    int(inf.grid_rounds), [int(x) for x in p], [int(x) for x in d],
                    [int(x) for x in rr], [int(x) for x in rd]))
    return out


def model_bytes(stats_by_rating, classes=None, n0=0, D0=0):
    """Total model bytes per kernel class over one step.  classes: merge
    class statistics per rating (merge_class_stats), for the merge kernels
    of the larger rows; n0 / D0: the input graph (validation, once)."""
    tot = {k: 0 for k in MODELS}
    tot["validate_entries"] = bytes_validate(n0, D0)
    for cs in (classes or {}).values():
        for name, _, _ in MERGE_CLASSES:
            tot[name] += bytes_merge(*cs[name])
    for rating, lv in stats_by_rating.items():
        io = rating == 1
        for l, (n, D, matched, rounds, grid_rounds, pt, dg, rr, rd) in enumerate(lv):
            tot["cut_entries"] += bytes_cut_entries(D)
            if l + 1 < len(lv):
                nc, Dc = lv[l + 1][0], lv[l + 1][1]
                tot["pick_first"] += bytes_pick_first(n, D, io)
                for r in range(2, min(grid_rounds, len(pt)) + 1):
                    tot["pick"] += bytes_pick_round(rr[r - 1], rd[r - 1])
                    tot["mate"] += bytes_mate_round(pt[r - 1])
                if not classes:
                    tot["fill_small"] += bytes_fill_small(n, D, nc, Dc, matched)
                tot["compact"] += bytes_compact(nc, Dc)
    return tot


# rocprofv3 kernel names (namespace, "void " and arguments stripped) of the
# library's profiler names
KERNEL_SYMBOLS = {"pick": r"pick_k<\d, false, 0, (true|false)>", "mate": r"mate_k<\d, false>",
                  "pick_first": r"pick_k<\d, true, 0, false>", "fill_small": r"fill_small_k",
                  "fill_mid": r"fill_mid_k", "fill_big": r"fill_big_k",
                  "fill_large": r"fill_large_k", "validate_entries": r"validate_entries_k(<(true|false)>)?",
                  "compact": r"compact_k", "cut_entries": r"up_entries_k<(true|false)>",
                  "refine_fm": r"ref_fm_k"}
# the sources a kernel's stored counters depend on (they go stale when these change)
COUNTER_SOURCES = ["paper_0910_2004_amd/csrc/k_level.hip", "paper_0910_2004_amd/csrc/kappa_internal.h",
                   "paper_0910_2004_amd/csrc/k_graph.hip"]
REFINE_COUNTER_SOURCES = ["paper_0910_2004_amd/csrc/k_refine.hip",
                          "paper_0910_2004_amd/csrc/kappa_internal.h"]


def counter_sources(kernel):
    return REFINE_COUNTER_SOURCES if kernel.startswith("refine") else COUNTER_SOURCES
WORKLOAD_RGG = "rgg n=2^20 mean degree 8, both ratings, k=64, stop 1280"
WORKLOAD_RMAT = ("rmat scale 22 edge factor 16 (a, b, c) = (0.57, 0.19, 0.19), weights in "
                 "[1, 100], expansion*2, k=256, stop n<=5120 or stall 1/20, eps=3/100")
WORKLOAD_REFINE = ("the way back up with pairwise refinement (preset fast) on the expansion*2 "
                   "hierarchy of rgg n=2^20 mean degree 8, k=64, stop 1280")


def _short_name(name):
    import re
    return re.sub(r"\(.*", "", name).replace("void ", "").replace("kappa::", "").strip()


def _sources_sha(sources):
    import hashlib
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def summarize_pmc(kernel, fetch_dir, write_dir, bench_cmd, tag="rmat22"):
    """profiles/<kernel>_<tag>_counters.json and .md from the counter-collection CSVs
    of a FETCH_SIZE pass and a WRITE_SIZE pass of the same bench command that
    ended with --copy-calibration: the last three 256 MiB copies give the
    scale from counter KiB to bytes (each copy reads and writes 256 MiB)."""
    import csv
    import glob
    import re
    pat = re.compile("^" + KERNEL_SYMBOLS[kernel] + "$")
    res = {}
    for ctr, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        rows = [r for f in files for r in csv.DictReader(open(f)) if r["Counter_Name"] == ctr]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 65536]
        copies = copies[-3:]
        vals = [float(r["Counter_Value"]) for r in copies]
        scale = (256 * 1024) / (sum(vals) / len(vals))
        ks = [r for r in rows if pat.match(_short_name(r["Kernel_Name"]))]
        tot_kib = sum(float(r["Counter_Value"]) for r in ks)
        res[ctr] = {"copy_kib": vals, "scale": scale, "dispatches": len(ks), "raw_kib_total": tot_kib,
                    "scaled_bytes_per_launch": tot_kib * 1024 * scale / max(len(ks), 1)}
    traffic = res["FETCH_SIZE"]["scaled_bytes_per_launch"] + res["WRITE_SIZE"]["scaled_bytes_per_launch"]
    cmds = [f"cd /tmp && timeout -s KILL 120 rocprofv3 --pmc {c} --kernel-trace -d <out> -o run "
            f"--output-format csv -- python3 <repo>/{bench_cmd}" for c in ("FETCH_SIZE", "WRITE_SIZE")]
    workload = WORKLOAD_REFINE if kernel.startswith("refine") else \
        (WORKLOAD_RMAT if tag == "rmat22" else WORKLOAD_RGG)
    rec = {"kernel": kernel, "tag": tag, "workload": workload, "counters": res,
           "traffic_bytes_per_launch": traffic, "sources": counter_sources(kernel),
           "sources_sha256": _sources_sha(counter_sources(kernel)), "commands": cmds}
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{tag}_counters.json"), "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# HBM traffic of `{kernel}` ({KERNEL_SYMBOLS[kernel]}): {workload}", "",
             "Commands (one counter per run; `<repo>` is the repository root):", ""]
    lines += ["    " + c for c in cmds]
    lines += ["", f"Summarised by `python bench.py --summarize-pmc {kernel} <fetch dir> <write dir> "
              f"--pmc-tag {tag}`.",
              "", "The run ends with three plain 256 MiB device-to-device copies "
              "(`--copy-calibration`), whose counters give the scale from counter KiB to bytes:", "",
              "| counter | copy KiB per 256 MiB | scale | dispatches | scaled MB per launch |",
              "|---|---|---|---|---|"]
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        r = res[ctr]
        lines.append(f"| {ctr} | {', '.join(f'{v:.1f}' for v in r['copy_kib'])} | {r['scale']:.4f} | "
                     f"{r['dispatches']} | {r['scaled_bytes_per_launch'] / 1e6:.3f} |")
    lines += ["", f"Traffic per launch: **{traffic / 1e6:.3f} MB**.  `bench.py` reports it as "
              f"`roofline.traffic` while the SHA-256 of {', '.join(counter_sources(kernel))} equals "
              f"`{rec['sources_sha256'][:16]}…`, and null once they change."]
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{tag}_counters.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    log(f"{kernel}: traffic {traffic / 1e6:.3f} MB per launch "
        f"({res['FETCH_SIZE']['dispatches']} dispatches)")


def summarize_stats(stats_csv, out_md, title, cmd):
    """A kernel-statistics table (rocprofv3 --stats kernel_stats.csv) as markdown."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(int(r["TotalDurationNs"]) for r in rows)
    lines = [f"# {title}", "", "Command (`<repo>` is the repository root):", "", "    " + cmd, "",
             f"Summarised by `python bench.py --summarize-stats <kernel_stats.csv> <out.md>`.", "",
             f"Total kernel time {tot / 1e6:.3f} ms over the whole run.", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{_short_name(r['Name'])}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {int(r['MinNs']) / 1e3:.2f} | "
                     f"{int(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 15 for the single-graph workloads, "
                         "about a second of work that brings a freshly started GPU to its "
                         "steady clocks; 3 otherwise)")
    ap.add_argument("--scale", type=int, default=20, help="log2 of the node count")
    ap.add_argument("--k", type=int, default=64)
    ap.add_argument("--block-bits", type=int, default=None,
                    help="rgg20: match with the two-phase matcher (Section 3.3), blocks of "
                         "2^BLOCK_BITS consecutive ids (0..11); default: local-max rounds")
    ap.add_argument("--serial-ratings", action="store_true",
                    help="rgg20: coarsen the two ratings one after the other on one stream "
                         "(default: concurrently, one stream and host thread per rating)")
    ap.add_argument("--order", default="generation", choices=["generation", "rcb", "rcb-device"],
                    help="rgg20: node ids in point generation order, or renumbered in "
                         "recursive coordinate bisection order (locality of a geometric "
                         "prepartition) on the device before the timed steps "
                         "(kappa_rcb_order + kappa_relabel, timed apart; rcb and rcb-device "
                         "are the same)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-out", default=None)
    ap.add_argument("--no-secondary", action="store_true",
                    help="rmat22: skip the random geometric graph summary in the same line")
    ap.add_argument("--workload", default="rmat22",
                    choices=["rgg20", "rmat22", "batch4096", "serve", "refine"],
                    help="rmat22: the headline single-graph workload (R-MAT scale 22); rgg20: "
                         "the random geometric graph of 2^20 nodes; batch4096: the batched "
                         "form on 4096 uneven graphs, against a loop of single calls; serve: "
                         "the served form on a Poisson request stream, against FIFO single "
                         "calls; refine: the way back up with pairwise refinement (Section 5) "
                         "on the rgg20 hierarchy")
    ap.add_argument("--preset", default="fast", choices=["minimal", "fast", "strong"],
                    help="refine: the refinement preset of Table 2")
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--serve-split", type=int, default=1 << 18,
                    help="serve: level-0 entries above which requests step in engines of their "
                         "own (0: one engine per rating)")
    ap.add_argument("--uploaders", type=int, default=2, help="serve: upload threads of the "
                                                             "level-granular server")
    ap.add_argument("--persistent", action="store_true",
                    help="run a level's matching rounds after the first in one cooperative launch "
                         "(kappa_persistent_enable; the library's default is a launch per round)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay repeated launch sequences as HIP graphs (kappa_graphs_enable; "
                         "the library's default is direct launches)")
    ap.add_argument("--no-plain-loop", action="store_true",
                    help="batch4096: skip the loop of single calls")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (3x) so that HBM byte counters "
                         "can be scaled against a kernel of known traffic")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("KERNEL", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/<kernel>_<tag>_counters.json/.md from two rocprofv3 --pmc runs "
                         "(no GPU work)")
    ap.add_argument("--pmc-tag", default="rmat22", help="workload of the --pmc runs (rmat22, rgg20)")
    ap.add_argument("--pmc-command", default="bench.py --steps 1 --warmup 1 --no-cpu-baseline "
                                             "--no-secondary --copy-calibration",
                    help="the bench command the --pmc runs profiled (recorded in the summary)")
    ap.add_argument("--summarize-stats", nargs=2, metavar=("STATS_CSV", "OUT_MD"),
                    help="write a markdown table from rocprofv3 --stats kernel_stats.csv (no GPU work)")
    ap.add_argument("--stats-title", default=f"Kernel statistics: {WORKLOAD_RMAT}")
    ap.add_argument("--stats-command", default="cd /tmp && rocprofv3 --kernel-trace --stats -d <out> -o run "
                                               "--output-format csv -- python3 <repo>/bench.py --steps 3 "
                                               "--warmup 1 --no-cpu-baseline --no-secondary")
    args = ap.parse_args()
    if args.warmup is None:
        args.warmup = 15 if args.workload in ("rmat22", "rgg20") else 3
    if args.summarize_pmc:
        return summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.summarize_pmc[2],
                             args.pmc_command, args.pmc_tag)
    if args.summarize_stats:
        return summarize_stats(args.summarize_stats[0], args.summarize_stats[1], args.stats_title,
                               args.stats_command)
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0910_2004_amd as K
    from workloads import rgg

    if args.graphs or args.persistent:
        import paper_0910_2004_amd as K
        K.graphs_enable(args.graphs)
        K.persistent_enable(args.persistent)
    if args.workload == "batch4096":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "refine":
        return bench_refine(args)

    out = single_graph(args, args.workload == "rmat22", primary=True)
    if args.workload == "rmat22" and not args.no_secondary:
        out["secondary"] = single_graph(args, False, primary=False)
    print(json.dumps(out), flush=True)


def single_graph(args, rmat_mode, primary):
    """One single-graph workload: rmat_mode the R-MAT of scale 22, else the
    random geometric graph.  primary: also the per-launch profile, the
    roofline object and the oracle baseline (the headline line); otherwise a
    short summary for the same JSON line."""
    import numpy as np
    import torch

    import paper_0910_2004_amd as K
    from workloads import rgg
    n = 1 << args.scale
    k = args.k
    stop_n = 20 * k
    eps = (3, 100)
    seed, part_seed = 42, 1
    ratings = [K.EXPANSION_STAR2, K.INNER_OUTER]
    if rmat_mode:
        # R-MAT of scale 22, edge factor 16, weights in [1, 100]; expansion*2,
        # k = 256, stop at 5120 nodes (or on the stall rule)
        if args.order != "generation" or args.block_bits is not None:
            print("bench.py: --workload rmat22 has no point coordinates and runs the default "
                  "matcher", file=sys.stderr)
            sys.exit(2)
        k, stop_n, ratings = 256, 5120, [K.EXPANSION_STAR2]

    t0 = time.time()
    if rmat_mode:
        from workloads import rmat
        g = rmat(22, 16, seed=3, wseed=33)
        log(f"generated rmat scale 22 n={g.n} |E|={g.m} in {time.time() - t0:.1f}s")
    else:
        g = rgg(n, seed=2)
        log(f"generated rgg n={g.n} |E|={g.m} in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    dg = K.DeviceGraph.from_csr(g, "cuda:0")
    relabel_ms = None
    if args.order != "generation" and not rmat_mode:
        # the points' RCB order and the renumbered graph, on the device
        from workloads import rgg_points
        xy = torch.from_numpy(rgg_points(n, 2)).to("cuda:0")
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t_a = time.perf_counter()
            order = K.kappa_rcb_order(xy, 32)
            dr = K.kappa_relabel(dg, order)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t_a) * 1e3)
        relabel_ms = round(min(ts), 3)
        log(f"device relabelling: {relabel_ms} ms (best of 3)")
        dg = dr
    # one stream (default priority) and one level-0 partition buffer per rating
    streams = [torch.cuda.Stream(device="cuda:0") for _ in ratings]
    part0s = [torch.empty(g.n, dtype=torch.int32, device="cuda:0") for _ in ratings]
    torch.cuda.synchronize()
    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=len(ratings))

    def hierarchy(i):
        # the whole hierarchy of rating i and the way back up, on stream i
        with torch.cuda.stream(streams[i]):
            H = K.kappa_coarsen(dg, ratings[i], seed, stop_n, 1, 20, 64, trusted=True,
                                block_bits=args.block_bits)
            _, res = K.kappa_uncoarsen(H, k, part_seed, eps[0], eps[1], part0=part0s[i])
            out = (level_stats(H), res[0].as_tuple())
            del H
        return out

    def step(serial=False):
        # the input is validated once per step (synchronous), then coarsened
        # with each rating: concurrently, one host thread and stream each
        # (independent hierarchies of the same graph), or one after the other
        st = K.kappa_validate(dg)
        if st != K.OK:
            raise RuntimeError(f"kappa_validate: {st}")
        if serial or args.serial_ratings:
            res = [hierarchy(i) for i in range(len(ratings))]
        else:
            res = [f.result() for f in [pool.submit(hierarchy, i) for i in range(len(ratings))]]
        return {r: res[i] for i, r in enumerate(ratings)}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the host's cyclic garbage collector paused a timed step now and then
    # (about 40 ms once per run, Python-side work, not the library's): collect
    # first and hold it off while timing, as timeit does
    gc.collect()
    gc.disable()
    t1 = time.perf_counter()
    marks = [t1]
    for _ in range(args.steps):
        stats = step()          # every call inside returns after its stream is synchronised
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gc.enable()
    ms_step = (t2 - t1) * 1e3 / args.steps
    med_ms = float(np.median(np.diff(marks))) * 1e3
    log("step times (ms): " + " ".join(f"{x * 1e3:.1f}" for x in np.diff(marks)))
    edges_step = g.m * len(ratings)
    value = edges_step / (ms_step / 1e3)
    # all levels' edges (sum over the hierarchy of |E_l|) per second
    level_edges = sum(x[1] // 2 for r in ratings for x in stats[r][0])
    wl_name = WORKLOAD_RMAT if rmat_mode else WORKLOAD_RGG
    log(f"{wl_name}: {ms_step:.3f} ms per step, {value:.4g} edges/s")
    if not primary:
        return {"workload": wl_name, "value": round(value, 1), "unit": "edges/s",
                "ms_per_step": round(ms_step, 3), "median_ms_per_step": round(med_ms, 3),
                "steps": args.steps, "warmup": args.warmup, "n": g.n, "m": g.m,
                "edges_per_step": edges_step, "ratings_concurrent": not args.serial_ratings}
    # merge classes of every level (for the merge kernels' byte models), from
    # one more hierarchy per rating, untimed
    classes = {}
    for i, r in enumerate(ratings):
        H = K.kappa_coarsen(dg, r, seed, stop_n, 1, 20, 64, trusted=True, block_bits=args.block_bits)
        classes[r] = merge_class_stats(H)
        del H

    # second timed pass with per-launch HIP events, the ratings one after the
    # other (a launch's events then bracket that launch alone)
    K.profile_reset()
    K.profile_enable(True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        pstats = step(serial=True)   # level statistics incl. rescans (recorded while profiling)
    torch.cuda.synchronize()
    K.profile_enable(False)
    prof = K.profile_read()
    K.profile_reset()

    lv = {r: pstats[r][0] for r in ratings}
    mb = model_bytes(lv, classes, g.n, g.nnz)
    total_ms = sum(ms for _, ms in prof.values()) / args.steps
    kern = sorted(prof.items(), key=lambda kv: -kv[1][1])
    log("kernel time per step (ms), launches per step:")
    for name, (cnt, ms) in kern:
        log(f"  {name:20s} {ms / args.steps:8.3f} ms  {cnt / args.steps:7.1f}")
    dom = kern[0][0]
    # the dominant kernel with a byte model (the roofline object reports it)
    cand = [name for name, _ in kern if name in mb]
    rk = cand[0] if cand else None
    roof = None
    if rk:
        cnt, ms = prof[rk]
        per_launch_bytes = mb[rk] / (cnt / args.steps)
        avg_s = ms / cnt / 1e3
        achieved = per_launch_bytes / avg_s / 1e9
        # the stored counters were taken on this workload in generation order
        traffic = counter_traffic(rk, "rmat22" if rmat_mode else "rgg20") \
            if args.order == "generation" and args.block_bits is None else None
        roof = {"bound": "hbm", "kernel": rk, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                "avg_launch_us": round(avg_s * 1e6, 2), "bytes_per_launch": int(per_launch_bytes),
                "model": MODELS[rk], "time_share": round(ms / args.steps / total_ms, 3),
                "dominant_kernel": dom}
        cc = copy_ceiling_gbs(torch)
        roof["copy_ceiling_gbs"] = cc
        roof["frac_of_copy"] = round(achieved / cc, 4)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        if rmat_mode:
            # the full scale-22 hierarchy takes the oracle minutes: the same
            # generator at scale 19 (an eighth of the edges; about 10-15 s on
            # one host thread), whole hierarchy
            from workloads import rmat
            gs = rmat(19, 16, seed=3, wseed=33)
            sample = f"R-MAT scale 19 (|E|={gs.m}), same generator and parameters, whole " \
                     "hierarchy and way back up on one host thread"
        else:
            gs = g
            if args.order != "generation":   # the same renumbered graph, by the oracle's reference
                from oracle.rcb import rcb_order, relabel
                from workloads import rgg_points
                gs = relabel(O.Graph.of(g), rcb_order(rgg_points(n, 2)))
            sample = "one full step (both ratings) of the same workload on one host thread"
        t3 = time.perf_counter()
        for r in ratings:
            OH = O.coarsen(gs, r, seed, stop_n, 1, 20, 64, block_bits=args.block_bits)
            O.uncoarsen(OH, k, part_seed, eps[0], eps[1])
        t4 = time.perf_counter()
        cpu = {"value": round(gs.m * len(ratings) / (t4 - t3), 1), "unit": "edges/s", "cores": 1,
               "kind": "oracle", "sample": f"{sample}; {t4 - t3:.2f} s",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}

    levels = {("expansion*2" if r == 0 else "innerOuter"): [x[0] for x in lv[r]] for r in ratings}
    lv_json = {str(r): [list(x[:5]) for x in lv[r]] for r in ratings}
    out = {
        "metric": "coarsening edges/s per GPU (full hierarchy)",
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "median_ms_per_step": round(med_ms, 3),
        "all_levels_edges_per_s": round(level_edges / (ms_step / 1e3), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 (exact integer; 128-bit rating compares)",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_RMAT if rmat_mode else
                               f"rgg n=2^{args.scale} mean degree 8, unit weights, both ratings "
                               f"(expansion*2, innerOuter), k={k}, stop n<={stop_n}, eps=3/100"
                               + ("" if args.order == "generation" else
                                  ", node ids in recursive coordinate bisection order"
                                  + (" (renumbered on the device before the timed steps)"
                                     if args.order != "generation" else ""))
                               + ("" if args.block_bits is None else
                                  f", two-phase matcher with blocks of 2^{args.block_bits}"),
                   "node_order": args.order, "block_bits": args.block_bits,
                   "relabel_ms": relabel_ms,
                   "ratings_concurrent": not args.serial_ratings, "graph_replay": bool(args.graphs),
                   "persistent_rounds": bool(args.persistent),
                   "n": g.n, "m": g.m, "edges_per_step": edges_step, "k": k, "stop_n": stop_n,
                   "seed": seed, "graph_seed": (3, 33) if rmat_mode else 2, "levels_n": levels},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {name: round(ms / args.steps, 4) for name, (cnt, ms) in kern},
        "path_model_gbs": round(sum(mb.values()) / (ms_step / 1e3) / 1e9, 1),
    }
    if args.copy_calibration:
        a = torch.ones(64 << 20, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {a.numel() * 4} bytes read and written")
    if args.profile_out:
        with open(args.profile_out, "w") as f:
            json.dump({"prof": prof, "model_bytes": mb, "levels": lv_json, "classes": classes},
                      f, indent=1)
    return out


def copy_ceiling_gbs(torch, mib=1024, reps=5):
    """Context for the roofline: a plain device-to-device copy of `mib` MiB,
    timed with events; read + written bytes per second (GB/s)."""
    a = torch.ones(mib << 18, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(gbs, 1)


def bench_batch(args):
    import numpy as np
    """The batched form on 4096 graphs of uneven size (n log-uniform in
    [1e3, 6.4e4]; half grids with 10 % of edges removed, half random
    geometric graphs of mean degree 8; weights uniform in [1, 16];
    expansion*2, stop at 256 nodes per graph).  A step is one
    kappa_coarsen_batch call on the union (validation and every level of
    every graph).  The same graphs coarsened one kappa_coarsen call at a time
    (the plain path) are timed once beside it."""
    import torch

    import paper_0910_2004_amd as K
    from workloads import batch_graphs

    t0 = time.time()
    graphs = batch_graphs(4096, seed=4, workers=min(16, os.cpu_count() or 1))
    torch.cuda.set_device(0)
    du, off = K.DeviceGraph.union(graphs, "cuda:0")
    edges = du.nnz // 2
    log(f"generated {len(graphs)} graphs, n={du.n} |E|={edges} in {time.time() - t0:.1f}s")
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        B = K.kappa_coarsen_batch(du, off, 0, 4, 256)
        del B
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()   # no host garbage-collector pause inside the timed steps
    t1 = time.perf_counter()
    for _ in range(args.steps):
        B = K.kappa_coarsen_batch(du, off, 0, 4, 256)
        levels = [B.info(g)[0] for g in range(len(graphs))]
        del B
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / args.steps
    gc.enable()
    plain = None
    if not args.no_plain_loop:
        plain = plain_loop(K, graphs, torch)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = batch_cpu_baseline(graphs)
    out = {
        "metric": "coarsening edges/s per GPU (batched form, 4096 graphs)",
        "value": round(edges / (ms / 1e3), 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 (exact integer; 128-bit rating compares)",
        "data": "synthetic",
        "config": {"workload": "4096 graphs, n log-uniform [1e3, 6.4e4], half grids minus 10% "
                               "of edges, half rgg mean degree 8, weights uniform [1, 16], "
                               "expansion*2, stop n<=256 per graph",
                   "graphs": len(graphs), "n": du.n, "m": edges, "seed": 4,
                   "graph_replay": bool(args.graphs), "persistent_rounds": bool(args.persistent),
                   "levels_max": int(max(levels)), "levels_mean": round(float(np.mean(levels)), 2)},
        "plain_loop": None if plain is None else
        {"ms": round(plain, 1), "value": round(edges / (plain / 1e3), 1), "unit": "edges/s",
         "kind": "one kappa_coarsen call per graph"},
        "speedup_vs_plain_loop": None if plain is None else round(plain / ms, 2),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_refine(args):
    """The way back up with pairwise refinement (Section 5) on the hierarchy
    of the rgg20 workload (n = 2^scale, mean degree 8, expansion*2, k = 64,
    stop at 20 k nodes), built once before the timed steps.  A step is one
    kappa_uncoarsen_refined call: the stand-in coarsest partition, then per
    level projection, refinement (Table 2 preset) and cut/balance.  The
    plain way back up (projection only) is timed beside it."""
    import numpy as np
    import torch

    import paper_0910_2004_amd as K
    from workloads import rgg

    n, k = 1 << args.scale, args.k
    stop_n, eps, seed, part_seed, rseed = 20 * k, (3, 100), 42, 1, 1
    t0 = time.time()
    g = rgg(n, seed=2)
    torch.cuda.set_device(0)
    dg = K.DeviceGraph.from_csr(g, "cuda:0")
    H = K.kappa_coarsen(dg, K.EXPANSION_STAR2, seed, stop_n)
    part0 = torch.empty(n, dtype=torch.int32, device="cuda:0")
    log(f"rgg n={n} |E|={g.m}, {len(H)} levels in {time.time() - t0:.1f}s")

    def step():
        return K.kappa_uncoarsen_refined(H, k, part_seed, eps[0], eps[1], args.preset, rseed,
                                         part0=part0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()   # no host garbage-collector pause inside the timed steps
    t1 = time.perf_counter()
    for _ in range(args.steps):
        _, res, st = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / args.steps
    tp = time.perf_counter()
    for _ in range(args.steps):
        _, plain = K.kappa_uncoarsen(H, k, part_seed, eps[0], eps[1])
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - tp) * 1e3 / args.steps
    gc.enable()

    K.profile_reset()
    K.profile_enable(True)
    torch.cuda.synchronize()
    step()
    torch.cuda.synchronize()
    K.profile_enable(False)
    prof = K.profile_read()
    K.profile_reset()
    kern = sorted(prof.items(), key=lambda kv: -kv[1][1])
    log("kernel time per step (ms), launches per step:")
    for name, (cnt, kms) in kern:
        log(f"  {name:20s} {kms:8.3f} ms  {cnt:7.0f}")
    total_ms = sum(kms for _, kms in prof.values())
    cnt, fm_ms = prof.get("refine_fm", (0, 0.0))
    fm_bytes = sum(x["bytes"] for x in st)
    moves = sum(x["moves"] for x in st)
    roof = None
    if cnt:
        avg_s = fm_ms / cnt / 1e3
        achieved = fm_bytes / cnt / avg_s / 1e9
        traffic = counter_traffic("refine_fm", "rgg20") if (args.scale, k, args.preset) == (20, 64, "fast") \
            else None
        roof = {"bound": "hbm", "kernel": "refine_fm", "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": None if traffic is None else int(traffic),
                "avg_launch_us": round(avg_s * 1e6, 2),
                "bytes_per_launch": int(fm_bytes / cnt),
                "model": "per local search 40 B per node of the two blocks + 12 B per row entry; "
                         "per move 17 B per queued node scanned + 25 B per entry of the moved "
                         "node's row; 12 B per kept move (counted by the kernel)",
                "time_share": round(fm_ms / total_ms, 3),
                "dominant_kernel": kern[0][0],
                "us_per_move_step": round(fm_ms * 1e3 / max(1, moves / 2), 3)}
        cc = copy_ceiling_gbs(torch)
        roof["copy_ceiling_gbs"] = cc
        roof["frac_of_copy"] = round(achieved / cc, 5)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        gs = rgg(1 << 16, seed=2)
        OH = O.coarsen(gs, O.EXPANSION_STAR2, seed, stop_n)
        prm = O.RefineParams(seed=rseed, **K.REFINE_PRESETS[args.preset])
        t3 = time.perf_counter()
        O.uncoarsen_refined(OH, k, part_seed, eps[0], eps[1], prm)
        t4 = time.perf_counter()
        cpu = {"value": round(gs.m / (t4 - t3), 1), "unit": "edges/s", "cores": 1,
               "kind": "oracle",
               "sample": f"rgg n=2^16 (|E|={gs.m}), same generator, k={k}, the way back up with "
                         f"refinement on one host thread; {t4 - t3:.2f} s",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    out = {
        "metric": "refined uncoarsening edges/s per GPU (level-0 edges)",
        "value": round(g.m / (ms / 1e3), 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64 gains, exact integer balance",
        "data": "synthetic",
        "config": {"workload": f"rgg n=2^{args.scale} mean degree 8, unit weights, expansion*2 "
                               f"hierarchy (stop n<={stop_n}), k={k}, eps=3/100, pairwise "
                               f"refinement preset {args.preset}",
                   "n": g.n, "m": g.m, "levels": len(H), "preset": args.preset,
                   "params": K.REFINE_PRESETS[args.preset]},
        "cut_refined": int(res[0].cut), "cut_projected": int(plain[0].cut),
        "feasible": bool(res[0].feasible), "max_block": int(res[0].max_block),
        "plain_uncoarsen_ms": round(plain_ms, 3),
        "refine_stats": {key: sum(x[key] for x in st) for key in st[0]},
        "refine_levels": [[H.info(l).n, x["searches"], x["moves"], round(x["init_ticks"] / 1e5, 1),
                           round(x["move_ticks"] / 1e5, 1)] for l, x in enumerate(st)],
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {name: round(kms, 4) for name, (c, kms) in kern},
    }
    if args.copy_calibration:
        a = torch.ones(64 << 20, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {a.numel() * 4} bytes read and written")
    print(json.dumps(out), flush=True)


def plain_loop(K, graphs, torch):
    """The plain path on the batch's graphs: one kappa_coarsen call per
    graph, graphs resident beforehand; milliseconds for all of them."""
    sub = [K.DeviceGraph.from_csr(g, "cuda:0") for g in graphs]
    torch.cuda.synchronize()
    for dg in sub[:64]:
        H = K.kappa_coarsen(dg, 0, 4, 256)
        del H
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for dg in sub:
        H = K.kappa_coarsen(dg, 0, 4, 256)
        del H
    torch.cuda.synchronize()
    return (time.perf_counter() - t2) * 1e3


def _oracle_one(args):
    import oracle as O
    g, seed, stop_n = args
    O.coarsen(g, 0, seed, stop_n, 1, 20, 64)
    return int(g.m)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batch_cpu_baseline(graphs, sample=256):
    """The oracle on a sample of the batch's graphs (every 16th): one host
    thread, then all host cores with the graphs split over processes."""
    from concurrent.futures import ProcessPoolExecutor
    sub = graphs[::max(1, len(graphs) // sample)][:sample]
    work = [(g, 4, 256) for g in sub]
    t0 = time.perf_counter()
    edges = sum(_oracle_one(w) for w in work)
    one = time.perf_counter() - t0
    cores = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_oracle_one, work, chunksize=4))
    many = time.perf_counter() - t0
    return {"value": round(edges / one, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sub)} of the {len(graphs)} graphs (every {len(graphs) // len(sub)}th), "
                      f"{edges} edges, {one:.2f} s on one thread",
            "all_cores": {"value": round(edges / many, 1), "cores": cores, "s": round(many, 2)},
            "cpu_model": cpu_model()}


def bench_serve(args):
    """The served form: `--requests` requests of the served mix (|E|
    log-uniform in [1e3, 4e6]; grids, random geometric graphs and R-MAT;
    rating, k in {2, 8, 32, 64}, stop at 20 k, eps 3/100), generated before
    the clock starts.  Three services: the plain path (one request at a time,
    kappa_coarsen), request-granular batches (BatchServer: kappa_coarsen_graphs
    per batch, two workers) and level-granular continuous batching
    (LevelServer: kappa_server_*, one engine per rating).  The plain path is
    first run with every request present to find its sustainable rate; then
    every service serves the same Poisson arrival trace at 0.7 of that rate.
    Latency is completion minus scheduled arrival; edges/s is all edges over
    first arrival to last completion.  The saturated figures serve every
    request at once (all present at the start).  `value` is the
    level-granular server's."""
    import numpy as np
    import torch

    import paper_0910_2004_amd as K
    from paper_0910_2004_amd.serve import (BatchServer, LevelServer, Request, latency_stats,
                                           serve_plain)
    from workloads import serve_requests

    t0 = time.time()
    mix = serve_requests(args.requests, seed=5, workers=min(16, os.cpu_count() or 1))
    log(f"generated {len(mix)} requests, |E| total {sum(g.m for g, _, _ in mix)} "
        f"in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    reqs = [Request(i, g, rating, k) for i, (g, rating, k) in enumerate(mix)]
    last = {}

    def level_run(rs):
        last["level"] = LevelServer(split_entries=args.serve_split if args.serve_split > 0
                                    else 1 << 62, uploaders=args.uploaders)
        return last["level"].run(rs)

    def level_profile():   # per engine: steps, mean step time, mean active requests
        out = {}
        for (rating, seed, big), p in sorted(last["level"].profile.items()):
            steps = max(p["steps"], 1)
            out[f"rating{rating}_{'large' if big else 'small'}"] = {
                "steps": p["steps"], "step_ms": round(1e3 * p["step_s"] / steps, 3),
                "admit_ms": round(1e3 * p["admit_s"] / steps, 3),
                "active": round(p["active_sum"] / steps, 2)}
        return out

    services = {"batch": lambda rs: BatchServer(workers=2).run(rs), "level": level_run}
    serve_plain(reqs[:32])   # warm up
    for run in services.values():
        run(reqs[:32])
    total_edges = sum(int(r.graph.m) for r in reqs)
    t1 = time.perf_counter()
    serve_plain(reqs)
    plain_s = time.perf_counter() - t1
    rate = len(reqs) / plain_s
    saturated = {"plain_edges_per_s": round(total_edges / plain_s, 1), "plain_s": round(plain_s, 3)}
    log(f"saturated plain: {plain_s:.2f} s")
    def clean():   # every service starts from an empty device cache
        torch.cuda.synchronize()
        K.kappa_cache_release()
        torch.cuda.empty_cache()

    for name, run in services.items():   # every request present at once
        clean()
        t1 = time.perf_counter()
        res = run(reqs)
        sec = time.perf_counter() - t1
        saturated[f"{name}_edges_per_s"] = round(total_edges / sec, 1)
        saturated[f"{name}_s"] = round(sec, 3)
        saturated[f"{name}_speedup"] = round(plain_s / sec, 2)
        saturated[f"{name}_mean_batch"] = round(float(np.mean([r.batch for r in res])), 2)
        log(f"saturated {name}: {sec:.2f} s")
        if name == "level":
            saturated["level_engines"] = level_profile()
    log(f"saturated: {saturated}")
    lam = 0.7 * rate
    gaps = np.random.default_rng(5).exponential(1.0 / lam, size=len(reqs))
    arrivals = np.cumsum(gaps) - gaps[0]
    trace = [Request(r.rid, r.graph, r.rating, r.k, arrival=float(arrivals[i]))
             for i, r in enumerate(reqs)]
    log(f"plain path sustains {rate:.1f} req/s; trace at {lam:.1f} req/s")
    stats = {"plain": latency_stats(trace, serve_plain(trace))}
    log(f"plain: {stats['plain']}")
    for name, run in services.items():
        clean()
        stats[name] = latency_stats(trace, run(trace))
        if name == "level":
            stats[name]["engines"] = level_profile()
        log(f"{name}: {stats[name]}")
    served = stats["level"]
    out = {
        "metric": "served coarsening: aggregate edges/s per GPU, p50/p99 latency",
        "value": served["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(served["span_s"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 (exact integer; 128-bit rating compares)",
        "data": "synthetic",
        "config": {"workload": "served mix: |E| log-uniform [1e3, 4e6], grid/rgg/rmat, "
                               "expansion*2 or innerOuter, k in {2,8,32,64}, stop 20k, "
                               "eps 3/100, Poisson arrivals at 0.7 x the plain path's rate",
                   "requests": len(trace), "rate_req_s": round(lam, 2), "seed": 5,
                   "server": "level-granular (kappa_server_*), one engine per rating" +
                             (f" and size class (split at {args.serve_split} entries)"
                              if args.serve_split > 0 else ""),
                   "uploaders": args.uploaders},
        "served": served,
        "batch_granular": stats["batch"],
        "plain": stats["plain"],
        "saturated": saturated,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
