"""CPU oracle for the coarsening hierarchy (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never does.

The arithmetic lives in ``kappa_oracle.c`` (plain sequential C); this module
marshals numpy arrays to it and writes the level loop of the multilevel scheme
(Section 2, "contraction phase") and the way back up (projection, cut and
balance) in plain Python, so the loop can be read against the paper.

A graph is any object with attributes ``n``, ``xadj`` (int64[n+1]),
``adj`` (int32[nnz]), ``ew`` (uint32[nnz]) and ``vw`` (uint32[n]).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# Rating selectors (Section 3.1), same numbering as the library.
EXPANSION_STAR2 = 0
INNER_OUTER = 1
WEIGHT = 2
EXPANSION = 3
EXPANSION_STAR = 4
RATINGS = {"expansion*2": EXPANSION_STAR2, "innerOuter": INNER_OUTER, "weight": WEIGHT,
           "expansion": EXPANSION, "expansion*": EXPANSION_STAR}

# Stop reasons of the level loop.
STOP_NONE, STOP_SIZE, STOP_EMPTY, STOP_STALL, STOP_MAXLEVEL = 0, 1, 2, 3, 4

OK, E_ARG, E_GRAPH, E_RANGE = 0, -1, -2, -3

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        L.orc_mix64.argtypes = [u64]
        L.orc_mix64.restype = u64
        L.orc_splitmix64_next.argtypes = [P]
        L.orc_splitmix64_next.restype = u64
        L.orc_validate.argtypes = [i32, i64, P, P, P, P]
        L.orc_validate.restype = ctypes.c_int
        L.orc_out.argtypes = [i32, P, P, P]
        L.orc_out.restype = None
        L.orc_rate.argtypes = [i32, P, P, P, P, ctypes.c_int, P, P]
        L.orc_rate.restype = ctypes.c_int
        L.orc_match_greedy.argtypes = [i32, i64, P, P, P, P, ctypes.c_int, u64, P]
        L.orc_match_greedy.restype = i64
        L.orc_match_rounds.argtypes = [i32, i64, P, P, P, P, ctypes.c_int, u64, P, P, P, P, i32]
        L.orc_match_rounds.restype = i32
        L.orc_match_two_phase.argtypes = [i32, i64, P, P, P, P, ctypes.c_int, u64, i32, P, P, P, P]
        L.orc_match_two_phase.restype = i64
        L.orc_contract.argtypes = [i32, i64, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_contract.restype = i32
        L.orc_initial_partition.argtypes = [i32, i32, u64, P]
        L.orc_initial_partition.restype = None
        L.orc_project.argtypes = [i32, P, P, P]
        L.orc_project.restype = None
        L.orc_cut_balance.argtypes = [i32, P, P, P, P, P, i32, u32, u32, P, P]
        L.orc_cut_balance.restype = ctypes.c_int
        L.orc_greedy_certificate.argtypes = [i32, P, P, P, P, ctypes.c_int, u64, P]
        L.orc_greedy_certificate.restype = i64
        L.orc_quotient_colouring.argtypes = [i32, P, P, P, i32, P, P, P, P]
        L.orc_quotient_colouring.restype = i32
        L.orc_fm_pair.argtypes = [i32, P, P, P, P, P, i32, i32, i32, u32, u32, u64, u32, u32, i32,
                                  P, P]
        L.orc_fm_pair.restype = ctypes.c_int
        L.orc_run_seed.argtypes = [u64, i32, i32, i32, i32, i32]
        L.orc_run_seed.restype = u64
        L.orc_refine.argtypes = [i32, P, P, P, P, P, i32, u32, u32, u64, u32, u32, i32, i32, i32,
                                 i32, P]
        L.orc_refine.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """Symmetric CSR of G = (V, E, c, w) (Section 2)."""
    n: int
    xadj: np.ndarray
    adj: np.ndarray
    ew: np.ndarray
    vw: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.xadj[self.n])

    @staticmethod
    def of(g) -> "Graph":
        return Graph(int(g.n), np.ascontiguousarray(g.xadj, dtype=np.int64),
                     np.ascontiguousarray(g.adj, dtype=np.int32),
                     np.ascontiguousarray(g.ew, dtype=np.uint32),
                     np.ascontiguousarray(g.vw, dtype=np.uint32))


def mix64(x: int) -> int:
    return int(lib().orc_mix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def splitmix64_stream(state: int, count: int) -> List[int]:
    s = ctypes.c_uint64(state)
    return [int(lib().orc_splitmix64_next(ctypes.byref(s))) for _ in range(count)]


def level_seed(seed: int, level: int) -> int:
    """Per-level tie-break seed: mix64(seed + level)."""
    return mix64((seed + level) & 0xFFFFFFFFFFFFFFFF)


def validate(g) -> int:
    g = Graph.of(g)
    return int(lib().orc_validate(g.n, g.nnz, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw)))


def out_weights(g) -> np.ndarray:
    g = Graph.of(g)
    out = np.zeros(max(g.n, 1), dtype=np.uint64)
    lib().orc_out(g.n, _p(g.xadj), _p(g.ew), _p(out))
    return out[:g.n]


def rate(g, rating: int):
    g = Graph.of(g)
    num = np.zeros(max(g.nnz, 1), dtype=np.uint64)
    den = np.zeros(max(g.nnz, 1), dtype=np.uint64)
    st = lib().orc_rate(g.n, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw), rating, _p(num), _p(den))
    if st != OK:
        raise ValueError(f"oracle rate failed: {st}")
    return num[:g.nnz], den[:g.nnz]


def match_greedy(g, rating: int, seed_l: int):
    g = Graph.of(g)
    mate = np.empty(max(g.n, 1), dtype=np.int32)
    m = lib().orc_match_greedy(g.n, g.nnz, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw),
                               rating, ctypes.c_uint64(seed_l), _p(mate))
    return mate[:g.n], int(m)


def match_rounds(g, rating: int, seed_l: int, max_rounds: int = 1 << 16):
    """Synchronous local-max rounds.  Returns (mate, |M|, rounds, active[], degree[])."""
    g = Graph.of(g)
    mate = np.empty(max(g.n, 1), dtype=np.int32)
    act = np.zeros(max_rounds, dtype=np.int64)
    deg = np.zeros(max_rounds, dtype=np.int64)
    matched = ctypes.c_int64(0)
    r = lib().orc_match_rounds(g.n, g.nnz, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw),
                               rating, ctypes.c_uint64(seed_l), _p(mate), ctypes.byref(matched),
                               _p(act), _p(deg), max_rounds)
    k = min(r, max_rounds)
    return mate[:g.n], int(matched.value), int(r), act[:k].copy(), deg[:k].copy()


def match_two_phase(g, rating: int, seed_l: int, block_bits: int):
    """The two-phase matcher of Section 3.3 (blocks of 2^block_bits
    consecutive ids; Greedy inside blocks, then Greedy on the gap graph).
    Returns (mate, |M|, block matching, gap-graph edges, gap edges matched)."""
    if not 0 <= block_bits <= 31:
        raise ValueError("block_bits must be in [0, 31]")
    g = Graph.of(g)
    mate = np.empty(max(g.n, 1), dtype=np.int32)
    loc = np.empty(max(g.n, 1), dtype=np.int32)
    ge, gm = ctypes.c_int64(0), ctypes.c_int64(0)
    m = lib().orc_match_two_phase(g.n, g.nnz, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw),
                                  rating, ctypes.c_uint64(seed_l), block_bits, _p(mate), _p(loc),
                                  ctypes.byref(ge), ctypes.byref(gm))
    return mate[:g.n], int(m), loc[:g.n], int(ge.value), int(gm.value)


def contract(g, mate: np.ndarray):
    """Returns (cmap, coarse Graph)."""
    g = Graph.of(g)
    mate = np.ascontiguousarray(mate, dtype=np.int32)
    n1 = max(g.n, 1)
    cmap = np.empty(n1, dtype=np.int32)
    cvw = np.empty(n1, dtype=np.uint32)
    cxadj = np.empty(n1 + 1, dtype=np.int64)
    cadj = np.empty(max(g.nnz, 1), dtype=np.int32)
    cew = np.empty(max(g.nnz, 1), dtype=np.uint32)
    cnnz = ctypes.c_int64(0)
    nc = lib().orc_contract(g.n, g.nnz, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw), _p(mate),
                            _p(cmap), _p(cvw), _p(cxadj), _p(cadj), _p(cew), ctypes.byref(cnnz))
    m = int(cnnz.value)
    coarse = Graph(int(nc), cxadj[:nc + 1].copy(), cadj[:m].copy(), cew[:m].copy(), cvw[:nc].copy())
    return cmap[:g.n].copy(), coarse


def initial_partition(n: int, k: int, seed: int) -> np.ndarray:
    part = np.empty(max(n, 1), dtype=np.int32)
    lib().orc_initial_partition(n, k, ctypes.c_uint64(seed), _p(part))
    return part[:n]


def project(cmap: np.ndarray, part_coarse: np.ndarray) -> np.ndarray:
    cmap = np.ascontiguousarray(cmap, dtype=np.int32)
    part_coarse = np.ascontiguousarray(part_coarse, dtype=np.int32)
    out = np.empty(max(len(cmap), 1), dtype=np.int32)
    lib().orc_project(len(cmap), _p(cmap), _p(part_coarse), _p(out))
    return out[:len(cmap)]


@dataclass
class CutBalance:
    cut: int
    total: int
    max_block: int
    max_node: int
    lmax_num: int
    lmax_den: int
    imb_num: int
    bal_num: int
    bal_den: int
    feasible: bool
    block_w: np.ndarray

    def as_tuple(self):
        return (self.cut, self.total, self.max_block, self.max_node, self.lmax_num,
                self.lmax_den, self.imb_num, self.bal_num, self.bal_den, int(self.feasible))


def cut_balance(g, part: np.ndarray, k: int, eps_num: int = 3, eps_den: int = 100) -> CutBalance:
    g = Graph.of(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    bw = np.zeros(max(k, 1), dtype=np.uint64)
    res = np.zeros(10, dtype=np.uint64)
    st = lib().orc_cut_balance(g.n, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw), _p(part), k,
                               eps_num, eps_den, _p(bw), _p(res))
    if st != OK:
        raise ValueError(f"oracle cut_balance failed: {st}")
    r = [int(x) for x in res]
    return CutBalance(r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], r[8], bool(r[9]), bw[:k].copy())


def cut_balance_status(g, part, k, eps_num, eps_den) -> int:
    g = Graph.of(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    bw = np.zeros(max(k, 1), dtype=np.uint64)
    res = np.zeros(10, dtype=np.uint64)
    return int(lib().orc_cut_balance(g.n, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw), _p(part), k,
                                     eps_num, eps_den, _p(bw), _p(res)))


def greedy_certificate(g, rating: int, seed_l: int, mate: np.ndarray) -> int:
    g = Graph.of(g)
    mate = np.ascontiguousarray(mate, dtype=np.int32)
    return int(lib().orc_greedy_certificate(g.n, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw),
                                            rating, ctypes.c_uint64(seed_l), _p(mate)))


# ---------------------------------------------------------------------------
# The multilevel loop (Section 2 and the stop rule of Section 4)
# ---------------------------------------------------------------------------
@dataclass
class Level:
    graph: Graph
    cmap: Optional[np.ndarray] = None      # fine -> coarse map to the next level
    mate: Optional[np.ndarray] = None
    matched: int = 0
    rounds: int = 0
    round_active: Optional[np.ndarray] = None
    round_degree: Optional[np.ndarray] = None
    stop_reason: int = STOP_NONE           # set on the coarsest level only


@dataclass
class Hierarchy:
    levels: List[Level] = field(default_factory=list)

    @property
    def stop_reason(self) -> int:
        return self.levels[-1].stop_reason


def coarsen_levels(g, rating: int = EXPANSION_STAR2, seed: int = 42, stop_n: int = 256,
                   stall_num: int = 1, stall_den: int = 20, max_levels: int = 64,
                   cross_check: bool = False, round_stats: bool = False,
                   block_bits: Optional[int] = None):
    """Contract until small (Section 2, contraction phase), one level at a time.

    Yields each level once it is final: with its matching, cmap and |M| if it
    was contracted, or with its stop reason if it is the coarsest.

    Level l is matched with the tie-break seed mix64(seed + l) using Greedy
    (Section 3.2), which under the strict edge order equals the parallel
    local-max scheme of Section 3.3.  ``cross_check`` also runs the round
    formulation and asserts that both give the same matching; ``round_stats``
    records the round statistics (from the round formulation).

    With ``block_bits`` set, every level is matched by the two-phase scheme
    of Section 3.3 instead (match_two_phase, blocks of 2^block_bits
    consecutive ids of that level); round statistics are then not recorded.

    Stop rules: before matching level l, stop if n_l <= stop_n (SIZE) or
    l == max_levels (MAXLEVEL); if the matching is empty, stop (EMPTY); after
    contracting, keep level l+1 and stop if it removed fewer than
    stall_num/stall_den of the nodes (STALL).
    """
    cur = Level(Graph.of(g))
    l = 0
    while True:
        G = cur.graph
        if G.n <= stop_n:
            cur.stop_reason = STOP_SIZE
            yield cur
            return
        if l == max_levels:
            cur.stop_reason = STOP_MAXLEVEL
            yield cur
            return
        s = level_seed(seed, l)
        if block_bits is not None:
            mate, m = match_two_phase(G, rating, s, block_bits)[:2]
        else:
            mate, m = match_greedy(G, rating, s)
        if block_bits is None and (cross_check or round_stats):
            mate_b, m_b, r, act, deg = match_rounds(G, rating, s)
            if cross_check:
                assert m_b == m and np.array_equal(mate_b, mate), "Greedy != local-max rounds"
            cur.rounds, cur.round_active, cur.round_degree = r, act, deg
        cur.mate, cur.matched = mate, m
        if m == 0:
            cur.stop_reason = STOP_EMPTY
            yield cur
            return
        cmap, coarse = contract(G, mate)
        cur.cmap = cmap
        yield cur
        nxt = Level(coarse)
        l += 1
        if (G.n - coarse.n) * stall_den < stall_num * G.n:
            nxt.stop_reason = STOP_STALL
            yield nxt
            return
        cur = nxt


def coarsen(g, rating: int = EXPANSION_STAR2, seed: int = 42, stop_n: int = 256,
            stall_num: int = 1, stall_den: int = 20, max_levels: int = 64,
            cross_check: bool = False, round_stats: bool = False,
            block_bits: Optional[int] = None) -> Hierarchy:
    """The whole hierarchy of coarsen_levels (same arguments)."""
    return Hierarchy(list(coarsen_levels(g, rating, seed, stop_n, stall_num, stall_den, max_levels,
                                         cross_check, round_stats, block_bits)))


def uncoarsen(H: Hierarchy, k: int, part_seed: int = 1, eps_num: int = 3, eps_den: int = 100):
    """Coarsest partition (stand-in), then projection and cut/balance per level.

    Returns (parts, results) with parts[l] / results[l] for every level l.
    """
    L = len(H.levels) - 1
    parts = [None] * (L + 1)
    res = [None] * (L + 1)
    parts[L] = initial_partition(H.levels[L].graph.n, k, part_seed)
    res[L] = cut_balance(H.levels[L].graph, parts[L], k, eps_num, eps_den)
    for l in range(L - 1, -1, -1):
        parts[l] = project(H.levels[l].cmap, parts[l + 1])
        res[l] = cut_balance(H.levels[l].graph, parts[l], k, eps_num, eps_den)
    return parts, res


# ---------------------------------------------------------------------------
# Pairwise refinement (Section 5); the readings are listed in kappa_oracle.c.
# ---------------------------------------------------------------------------

@dataclass
class RefineParams:
    """Parameters of the refinement (Table 2 names the presets)."""
    seed: int = 1
    alpha_num: int = 5          # FM patience alpha = alpha_num / alpha_den
    alpha_den: int = 100
    depth: int = 5              # BFS search depth
    max_local: int = 3          # local iterations
    max_global: int = 15        # max. global iterations
    stop_after: int = 1         # global iterations in a row without change that end it

    @staticmethod
    def preset(name: str) -> "RefineParams":
        """Table 2: minimal, fast, strong."""
        return {"minimal": RefineParams(alpha_num=1, depth=1, max_local=1, max_global=1),
                "fast": RefineParams(),
                "strong": RefineParams(alpha_num=20, depth=20, max_local=5, stop_after=2)}[name]


def quotient_colouring(g, part: np.ndarray, k: int):
    """Q's edges (a < b, ascending) with their greedy colours; returns
    (pairs int32[m, 2], colour int32[m], number of colours)."""
    g = Graph.of(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    cap = k * k // 2 + 1
    pa, pb, pc = (np.zeros(cap, np.int32) for _ in range(3))
    m = ctypes.c_int32(0)
    nc = lib().orc_quotient_colouring(g.n, _p(g.xadj), _p(g.adj), _p(part), k, _p(pa), _p(pb),
                                      _p(pc), ctypes.byref(m))
    m = m.value
    return np.stack([pa[:m], pb[:m]], 1), pc[:m].copy(), int(nc)


def run_seed(seed: int, g: int, a: int, b: int, t: int, r: int) -> int:
    return int(lib().orc_run_seed(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), g, a, b, t, r))


def fm_pair(g, part: np.ndarray, k: int, a: int, b: int, run_seed_: int, alpha_num: int = 5,
            alpha_den: int = 100, depth: int = 5, eps_num: int = 3, eps_den: int = 100):
    """One two-block local search (Section 5.2) on blocks a < b.  Returns
    (moves int32[made], dict) with the start/end (imbalance, cut) and the
    number of moves kept after the rollback; part is not changed."""
    g = Graph.of(g)
    part = np.ascontiguousarray(part, dtype=np.int32)
    moves = np.zeros(max(g.n, 1), np.int32)
    res = np.zeros(6, np.int64)
    st = lib().orc_fm_pair(g.n, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw), _p(part), k, a, b,
                           eps_num, eps_den, ctypes.c_uint64(run_seed_), alpha_num, alpha_den,
                           depth, _p(moves), _p(res))
    if st != OK:
        raise ValueError(f"oracle fm_pair failed: {st}")
    r = [int(x) for x in res]
    return moves[:r[4]].copy(), {"start": (r[0], r[1]), "end": (r[2], r[3]), "made": r[4],
                                 "kept": r[5]}


def refine(g, part: np.ndarray, k: int, eps_num: int = 3, eps_den: int = 100,
           params: Optional[RefineParams] = None):
    """Pairwise refinement of one level (Section 5).  Returns (new part,
    stats dict); the input array is not changed."""
    p = params or RefineParams()
    g = Graph.of(g)
    out = np.array(part, dtype=np.int32, copy=True)
    st = np.zeros(6, np.int64)
    rc = lib().orc_refine(g.n, _p(g.xadj), _p(g.adj), _p(g.ew), _p(g.vw), _p(out), k, eps_num,
                          eps_den, ctypes.c_uint64(p.seed), p.alpha_num, p.alpha_den, p.depth,
                          p.max_local, p.max_global, p.stop_after, _p(st))
    if rc != OK:
        raise ValueError(f"oracle refine failed: {rc}")
    keys = ("global_iterations", "searches", "moves", "kept", "adoptions", "colours")
    return out, dict(zip(keys, (int(x) for x in st)))


def uncoarsen_refined(H: Hierarchy, k: int, part_seed: int = 1, eps_num: int = 3,
                      eps_den: int = 100, params: Optional[RefineParams] = None):
    """The way back up with refinement: coarsest partition (stand-in), then
    per level from the coarsest down: project, refine, cut/balance.  The
    refinement seed of level l is mix64(params.seed + l).  Returns (parts,
    results, stats) per level."""
    p = params or RefineParams()
    L = len(H.levels) - 1
    parts, res, stats = [None] * (L + 1), [None] * (L + 1), [None] * (L + 1)
    for l in range(L, -1, -1):
        g = H.levels[l].graph
        start = (initial_partition(g.n, k, part_seed) if l == L
                 else project(H.levels[l].cmap, parts[l + 1]))
        pl = RefineParams(**{**p.__dict__, "seed": level_seed(p.seed, l)})
        parts[l], stats[l] = refine(g, start, k, eps_num, eps_den, pl)
        res[l] = cut_balance(g, parts[l], k, eps_num, eps_den)
    return parts, res, stats
