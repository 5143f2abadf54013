// k_level.hip -- one level of the multilevel loop (Section 2): matching
// (Section 3.3) and contraction, driven entirely by device-resident state.
//
// Every kernel reads its level's graph from the level descriptor and checks
// the level's phase, so the host enqueues whole levels without reading
// anything back: a level whose stop rule fired (or that does not exist yet)
// turns every later kernel into a no-op.  Allocation of the next level's
// arrays is a device-side bump in one arena.
//
// Matching: rounds as in the paper's parallel scheme.  Every free node that
// still has a free neighbour points at its best edge to a free neighbour
// (the strict order of kappa.h); edges that are best at both ends are
// matched; repeat until no free node has a free neighbour.  Under a strict
// total order this is exactly the Greedy matching of Section 3.2.
//   pick kernel  -- node-centric argmax over the row, nodes binned by degree:
//                   bin 0 (deg <= 16) 4 lanes per node, bin 1 (deg <= 1024)
//                   one wave per node, bin 2 one block per node.  A pending
//                   node whose previous choice is still free keeps it (free
//                   sets only shrink, so it is still the maximum).
//   mate kernel  -- mutual check best[best[v]] == v, matched pairs written,
//                   survivors appended (block-aggregated) to the next lists.
//   finisher     -- one 1024-thread workgroup runs the remaining rounds with
//                   workgroup barriers once few nodes remain.
//
// Contraction: each matched pair {u, v} becomes one coarse node x with
// c(x) = c(u) + c(v); the rows of u and v are merged (neighbours renamed to
// coarse ids, the contracted edge dropped, parallel edges summed).  Coarse
// ids: representatives (unmatched nodes and the smaller end of each matched
// edge) numbered in ascending fine id by a device scan.
//   1. scan of representative flags; its apply writes the whole coarse node
//      (cmap of both ends, rep_of, partner, c(x)); the epilogue allocates the
//      next level's node arrays
//   2. merge of each coarse row, staged in the slots of its two fine rows
//      (deg(u) + deg(v) - 2 entries at most), by class of that bound:
//        small (<= 64 entries): 16 lanes per row, rank sort in LDS
//        mid (<= 4094):         one block per row, bitonic sort in LDS
//        large:                 dense per-slot accumulator + bitmap, read
//                               back in ascending id order
//   3. scan of the merged degrees -> coarse row offsets; the epilogue
//      allocates the next level's edge arrays and checks the stall rule
//   4. compact: copy merged rows into the exact-size coarse arrays
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "kappa_internal.h"

namespace kappa {

// ===========================================================================
// Common
// ===========================================================================
__device__ __forceinline__ bool load_level(const LevelDesc *L, int32_t want, DevGraph &g) {
    if (L->phase != want) return false;
    g.n = L->n; g.nnz = L->nnz; g.xadj = L->xadj; g.adj = L->adj; g.ew = L->ew; g.vw = L->vw;
    g.gid = L->gid; g.noff = L->noff;
    return true;
}

// Batched form: is v's graph still coarsening?
__device__ __forceinline__ bool graph_active(const Ctx &c, const DevGraph &g, int64_t v) {
    return !g.gid || c.b.active[g.gid[v]];
}

__device__ __forceinline__ int bin_of(const Ctx &c, int64_t deg) {
    return deg <= c.t.bin_small_max ? 0 : (deg <= BIN_MID_MAX ? 1 : 2);
}


// Node id read from a pending list: -1 (and a control flag) if out of range.
// Valid state never trips this; it keeps a broken state from indexing memory.
__device__ __forceinline__ int32_t checked_node(int32_t v, int32_t n, Control *ctrl) {
    if ((uint32_t)v < (uint32_t)n) return v;
    atomicOr(&ctrl->flags, (uint32_t)CF_STATE);
    return -1;
}

// ===========================================================================
// Level start (first kernel of a level): stop rules (Section 2 threshold,
// Section 4), state resets.  Every block takes the same decision from the
// same inputs; block 0 writes it (the only fields it changes are read as
// "this level goes on" either way, or end the level for every block).
// ===========================================================================
__device__ __forceinline__ bool level_gate(const Ctx &c, int l, bool stop_rules, bool writer) {
    Control *ctrl = c.ctrl;
    LevelDesc *L = c.lv + l;
    if (ctrl->done || ctrl->nlevels != l + 1) return false;
    const int32_t ph = L->phase;
    if (ph != PH_IDLE && ph != PH_MATCH) return false;
    int32_t stop = KAPPA_STOP_NONE;
    if (stop_rules && L->n <= ctrl->stop_n) stop = KAPPA_STOP_SIZE;
    else if (stop_rules && l >= ctrl->max_levels) stop = KAPPA_STOP_MAXLEVEL;
    if (stop != KAPPA_STOP_NONE || !L->mate || !L->cmap) {
        if (writer) {
            L->stop = stop;
            L->phase = PH_STOPPED;
            ctrl->done = 1;
        }
        return false;
    }
    if (writer) L->phase = PH_MATCH;
    return true;
}

// ===========================================================================
// Matching
// ===========================================================================
// Pending nodes of a round live in lists per degree bin, stored as three
// arrays: the node, its current choice (-1: none yet) and its degree.  Round
// r reads parity (r-1)&1 (round 1: every node for bin 0, the init lists for
// bins 1 and 2) and writes parity r&1.
struct PList {
    int32_t *v, *b, *d;
};
__device__ __forceinline__ PList plist(const MatchScratch &ms, int32_t n, int par, int bin) {
    const int64_t off = (int64_t)(par * 3 + bin) * n;
    return PList{ms.lv + off, ms.lb + off, ms.ld + off};
}

// The rating's node attribute: c(v), or Out(v) for innerOuter (weight uses
// neither).  Round 1 reads it from the graph; later rounds from the packed
// node record {attribute, mate}, one 8-byte gather per neighbour.
template <int R>
__device__ __forceinline__ uint32_t attr_src(const DevGraph &g, const uint32_t *out, int32_t v) {
    return R == KAPPA_INNER_OUTER ? out[v] : (R == KAPPA_WEIGHT ? 0u : g.vw[v]);
}

// Two-phase matcher (Section 3.3): the edges its gap rounds may match.
// F = 0: every edge; F = 1: gap edges only -- {v,u} with v and u in
// different blocks (blocks of 2^bb consecutive ids) and above, in the strict
// order, the edge the block phase matched at v and the one at u.
struct GapView {
    int32_t bb;
    const int32_t *loc;
    const LocKey *key;
};
__device__ __forceinline__ GapView gap_view(const Ctx &c) {
    return GapView{c.block_bits, c.ms.loc, c.ms.lkey};
}
// The block edge at x as a candidate incident to x (u = -1: none).
__device__ __forceinline__ Cand loc_cand(const GapView &gv, int32_t x) {
    Cand k = cand_none();
    k.u = gv.loc[x];
    if (k.u >= 0) {
        const LocKey q = gv.key[x];
        k.num = q.num;
        k.den = q.den;
        k.h = q.h;
    }
    return k;
}
__device__ __forceinline__ bool cross_block(const GapView &gv, int32_t v, int32_t u) {
    return (v >> gv.bb) != (u >> gv.bb);
}
// cd: a candidate {v, cd.u} between two blocks; kv: loc_cand(gv, v).
__device__ __forceinline__ bool above_block_edges(const GapView &gv, const Cand &cd, int32_t v,
                                                  const Cand &kv) {
    if (!cand_better(cd, kv, v)) return false;
    Cand cu = cd;   // the same edge seen from u
    cu.u = v;
    return cand_better(cu, loc_cand(gv, cd.u), cd.u);
}

// Best edge from v to a free neighbour over the entries sub, sub+G, ... of
// [b, e).  A lane keeps SCAN_UNROLL entries in flight: their loads, then
// their neighbours' records, are issued before the first comparison.
constexpr int SCAN_UNROLL = 4;
template <int R, int G, bool FIRST, int F = 0>
__device__ __forceinline__ Cand scan_range(const DevGraph &g, int32_t v, uint32_t av, int sub,
                                           int64_t b, int64_t e, const int2 *nrec,
                                           const uint32_t *out, uint64_t seed, int32_t base,
                                           const GapView &gv) {
    Cand best = cand_none();
    const Cand kv = F ? loc_cand(gv, v) : cand_none();
    for (int64_t j0 = b + sub; j0 < e; j0 += (int64_t)G * SCAN_UNROLL) {
        int32_t u[SCAN_UNROLL];
        uint32_t w[SCAN_UNROLL], au[SCAN_UNROLL];
        bool ok[SCAN_UNROLL];
#pragma unroll
        for (int t = 0; t < SCAN_UNROLL; ++t) {
            const int64_t j = j0 + (int64_t)t * G;
            ok[t] = j < e;
            u[t] = ok[t] ? g.adj[j] : 0;
            w[t] = ok[t] ? g.ew[j] : 0u;
        }
#pragma unroll
        for (int t = 0; t < SCAN_UNROLL; ++t) {
            if (F) ok[t] = ok[t] && cross_block(gv, v, u[t]);
            if (FIRST) {
                au[t] = ok[t] ? attr_src<R>(g, out, u[t]) : 0u;   // round 1: every node is free
            } else {
                const int2 rec = ok[t] ? nrec[u[t]] : make_int2(0, 0);
                ok[t] = ok[t] && rec.y < 0;
                au[t] = (uint32_t)rec.x;
            }
        }
#pragma unroll
        for (int t = 0; t < SCAN_UNROLL; ++t) {
            if (!ok[t]) continue;
            Cand cd;
            rate<R>(w[t], au[t], av, au[t], av, cd.num, cd.den);
            cd.h = mix64(seed ^ edge_id_local(v, u[t], base));
            cd.u = u[t];
            if (F && !above_block_edges(gv, cd, v, kv)) continue;
            if (cand_better(cd, best, v)) best = cd;
        }
    }
    return best;
}
template <int R, int G, bool FIRST, int F = 0>
__device__ __forceinline__ Cand scan_row(const DevGraph &g, int32_t v, uint32_t av, int sub,
                                         const int2 *nrec, const uint32_t *out, uint64_t seed,
                                         int32_t base, const GapView &gv) {
    return scan_range<R, G, FIRST, F>(g, v, av, sub, g.xadj[v], g.xadj[v + 1], nrec, out, seed,
                                      base, gv);
}

// The same over a row of at most BIN_SMALL_MAX entries [b, e): every load of
// a lane's entries is issued before the first comparison.
template <int R, int G, bool FIRST, int F = 0>
__device__ __forceinline__ Cand scan_row_small(const DevGraph &g, int32_t v, uint32_t av, int sub,
                                               int64_t b, int64_t e, const int2 *nrec,
                                               const uint32_t *out, uint64_t seed, int32_t base,
                                               const GapView &gv) {
    constexpr int T = BIN_SMALL_MAX / G;
    int32_t u[T];
    uint32_t w[T], au[T];
    bool ok[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t j = b + sub + (int64_t)t * G;
        ok[t] = j < e;
        u[t] = ok[t] ? g.adj[j] : 0;
        w[t] = ok[t] ? g.ew[j] : 0u;
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (F) ok[t] = ok[t] && cross_block(gv, v, u[t]);
        if (FIRST) {
            au[t] = ok[t] ? attr_src<R>(g, out, u[t]) : 0u;
        } else {
            const int2 rec = ok[t] ? nrec[u[t]] : make_int2(0, 0);
            ok[t] = ok[t] && rec.y < 0;
            au[t] = (uint32_t)rec.x;
        }
    }
    Cand best = cand_none();
    const Cand kv = F ? loc_cand(gv, v) : cand_none();
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (!ok[t]) continue;
        Cand cd;
        rate<R>(w[t], au[t], av, au[t], av, cd.num, cd.den);
        cd.h = mix64(seed ^ edge_id_local(v, u[t], base));
        cd.u = u[t];
        if (F && !above_block_edges(gv, cd, v, kv)) continue;
        if (cand_better(cd, best, v)) best = cd;
    }
    return best;
}

template <int G>
__device__ __forceinline__ Cand group_reduce(Cand cd, int32_t v) {
    for (int off = G / 2; off > 0; off >>= 1) {
        Cand o = cand_shfl_xor(cd, off, G);
        if (cand_better(o, cd, v)) cd = o;
    }
    return cd;
}

// Whole-block argmax (all threads call; contains barriers).
__device__ __forceinline__ Cand block_reduce_cand(Cand cd, int32_t v, Cand *sh) {
    cd = group_reduce<WAVE>(cd, v);
    int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    if (lane_id() == 0) sh[w] = cd;
    __syncthreads();
    Cand r = sh[0];
    for (int i = 1; i < nw; ++i)
        if (cand_better(sh[i], r, v)) r = sh[i];
    __syncthreads();
    return r;
}

// A pending node keeps its choice while that neighbour is still free (free
// sets only shrink, so it is still the maximum).
__device__ __forceinline__ bool keeps_choice(int32_t bp, int32_t n, const int2 *nrec) {
    return bp >= 0 && bp < n && nrec[bp].y < 0;
}

__device__ __forceinline__ uint64_t level_seed(const Ctx &c, int l) {
    return c.seed_direct ? c.seed : mix64(c.seed + (uint64_t)l);
}

// The tie-break seed of v's graph: in a served step every graph carries the
// seed of its own hierarchy level, which differs from the union's level.
__device__ __forceinline__ uint64_t row_seed(const Ctx &c, const DevGraph &g, int32_t v,
                                             uint64_t seed) {
    return (c.b.gseed && g.gid) ? c.b.gseed[g.gid[v]] : seed;
}

// Block-aggregated append of up to MK entries per thread into the three bin
// lists `ol` (bin < 0: none); counters cnt[3] may be global or LDS.  Every
// thread of the block calls it; sh: BLOCK/WAVE + 1 (blockDim.x/WAVE + 1)
// int64, sbase: 3 int32 of LDS.  Order inside a list is not deterministic;
// no consumer depends on it.
constexpr int MK = 8;
// Where the chunk records of appended bin-2 entries go (rec == nullptr: none;
// the one-workgroup finisher scans long rows whole).  cnt: the record counter.
// kfirst (round 1 only): each row's first record is also kept by node.
struct HubOut {
    int2 *rec;
    int32_t *first;
    int32_t *cnt;
    int64_t cap;
    int32_t *kfirst;
};
__device__ __forceinline__ HubOut hub_out(const Ctx &c, int32_t n, int par, int32_t *cnt3) {
    HubOut h{nullptr, nullptr, nullptr, 0, nullptr};
    if (!c.ms.hub.rec) return h;
    h.rec = c.ms.hub.rec + (int64_t)par * c.ms.hub.cap;
    h.first = c.ms.hub.first + (int64_t)par * n;
    h.cnt = cnt3 + 3;
    h.cap = c.ms.hub.cap;
    h.kfirst = c.ms.hub.kfirst;
    return h;
}
__device__ __forceinline__ int32_t hub_chunks_of(int64_t deg) {
    return (int32_t)((deg + HUB_CHUNK - 1) / HUB_CHUNK);
}
// Records {p, 0 .. k-1} for the bin-2 entry (node v) at list position p of
// degree d.
__device__ __forceinline__ void hub_emit(const HubOut &h, int32_t p, int32_t v, int32_t d,
                                         Control *ctrl) {
    const int32_t k = hub_chunks_of(d);
    const int32_t base = atomicAdd(h.cnt, k);
    if ((int64_t)base + k > h.cap) {   // cannot happen: the capacity bounds every level
        atomicOr(&ctrl->flags, (uint32_t)CF_STATE);
        h.first[p] = -1;
        if (h.kfirst) h.kfirst[v] = -1;
        return;
    }
    h.first[p] = base;
    if (h.kfirst) h.kfirst[v] = base;
    for (int32_t q = 0; q < k; ++q) h.rec[base + q] = make_int2(p, q);
}
__device__ __forceinline__ void block_append_mk(const int bin[MK], const int32_t v[MK],
                                                const int32_t b[MK], const int32_t d[MK],
                                                const PList ol[3], int32_t *cnt, int64_t *sh,
                                                int32_t *sbase, const HubOut &ho = HubOut{},
                                                Control *ctrl = nullptr) {
    constexpr int64_t M = 0x1fffff;   // 21 bits per bin: at most 1024 * MK entries per block
    int64_t packed = 0;
#pragma unroll
    for (int k = 0; k < MK; ++k)
        if (bin[k] >= 0) packed += (int64_t)1 << (21 * bin[k]);
    int64_t tot;
    const int64_t pre = block_excl_scan(packed, sh, &tot);
    if (threadIdx.x < 3) {
        const int32_t t = (int32_t)((tot >> (21 * threadIdx.x)) & M);
        sbase[threadIdx.x] = t ? atomicAdd(&cnt[threadIdx.x], t) : 0;
    }
    __syncthreads();
    int32_t p0 = sbase[0] + (int32_t)(pre & M), p1 = sbase[1] + (int32_t)((pre >> 21) & M),
            p2 = sbase[2] + (int32_t)((pre >> 42) & M);
#pragma unroll
    for (int k = 0; k < MK; ++k) {
        if (bin[k] < 0) continue;
        int32_t p;
        PList o;
        if (bin[k] == 0) { p = p0++; o = ol[0]; }
        else if (bin[k] == 1) { p = p1++; o = ol[1]; }
        else { p = p2++; o = ol[2]; }
        o.v[p] = v[k];
        o.b[p] = b[k];
        o.d[p] = d[k];
        if (bin[k] == 2 && ho.rec) hub_emit(ho, p, v[k], d[k], ctrl);
    }
    __syncthreads();   // sbase is reused by the next call
}

// --- phases of the per-round kernels --------------------------------------

// mate = best = -1; nodes of bins 1 and 2 go to the round-1 lists (parity 0).
// Loads of a thread's MK entries are issued before its stores.
// bid / nb: this block and the number of blocks sharing the work; cnt: the
// three list counters (global, or LDS when one block does all the work).
__device__ __forceinline__ void init_phase(const Ctx &c, const DevGraph &g, LevelDesc *L,
                                           int64_t *sh, int32_t *sbase, unsigned bid, unsigned nb,
                                           int32_t *cnt, bool grid) {
    int32_t *mate = L->mate, *best = c.ms.best;
    const PList ol[3] = {plist(c.ms, g.n, 0, 0), plist(c.ms, g.n, 0, 1), plist(c.ms, g.n, 0, 2)};
    // chunk records only for the grid rounds (a one-workgroup caller scans
    // long rows whole, and its counters have no chunk slot)
    const HubOut ho = grid ? hub_out(c, g.n, 0, cnt) : HubOut{};
    // pass p, slot k of block b covers entries ((p * MK + k) * nb + b) * blockDim.x + t:
    // small inputs spread over every block first
    const int64_t row = (int64_t)nb * blockDim.x, per_pass = row * MK;
    for (int64_t base = 0; base < g.n; base += per_pass) {   // block-uniform
        const int64_t first = base + (int64_t)bid * blockDim.x + threadIdx.x;
        int bin[MK];
        int32_t vv[MK], bb[MK], dd[MK];
        int64_t deg[MK];
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            const int64_t i = first + (int64_t)k * row;
            deg[k] = i < g.n ? g.xadj[i + 1] - g.xadj[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            const int64_t i = first + (int64_t)k * row;
            vv[k] = (int32_t)i;
            bb[k] = -1;
            dd[k] = (int32_t)deg[k];
            const int bn = bin_of(c, deg[k]);
            bin[k] = i < g.n && bn > 0 && graph_active(c, g, i) ? bn : -1;
            if (i < g.n) {
                mate[i] = -1;
                best[i] = -1;
            }
        }
        block_append_mk(bin, vv, bb, dd, ol, cnt, sh, sbase, ho, c.ctrl);
    }
}

// Inputs of round r: lists and their sizes (round 1: bin 0 is every node),
// and the chunk records of the bin-2 list (grid rounds only).
struct RoundIn {
    PList in[3];
    int32_t cn[3];
    int32_t nrec;
    const int2 *rec;
    const int32_t *first;
    // rounds >= 2 with a preparation launch: the rows to rescan
    const int2 *scan[2];
    int32_t scn[2];
};
template <bool FIRST>
__device__ __forceinline__ RoundIn round_inputs(const Ctx &c, const DevGraph &g, int r,
                                                const int32_t *cnt3) {
    RoundIn ri;
    const int par = FIRST ? 0 : ((r - 1) & 1);
    for (int b = 0; b < 3; ++b) {
        ri.in[b] = plist(c.ms, g.n, par, b);
        ri.cn[b] = min(cnt3[b], g.n);
    }
    if (FIRST) ri.cn[0] = g.n;
    ri.nrec = 0;
    ri.rec = nullptr;
    ri.first = nullptr;
    ri.scan[0] = ri.scan[1] = nullptr;
    ri.scn[0] = ri.scn[1] = 0;
    if (c.ms.hub.rec) {
        // round 1: records of every bin-2 row (the init lists); later rounds:
        // records and scan lists of the rows the preparation found to rescan
        const int32_t *sc = FIRST ? cnt3 : c.ms.state->scnt[r & 3];
        ri.nrec = (int32_t)min<int64_t>(sc[3], c.ms.hub.cap);
        ri.rec = c.ms.hub.rec + (int64_t)par * c.ms.hub.cap;
        ri.first = c.ms.hub.first + (int64_t)par * g.n;
        if (!FIRST) {
            for (int b = 0; b < 2; ++b) {
                ri.scan[b] = c.ms.hub.scan + (int64_t)b * g.n;
                ri.scn[b] = min(sc[b], g.n);
            }
        }
    }
    return ri;
}

// bin 0: SMALL_G lanes per node
template <int R, bool FIRST, int F = 0>
__device__ __forceinline__ void pick_bin0(const Ctx &c, const DevGraph &g, uint64_t seed,
                                          const RoundIn &ri, unsigned bid, unsigned nb) {
    const GapView gv = gap_view(c);
    const int G = SMALL_G;
    int32_t *best = c.ms.best;
    const int2 *nrec = c.ms.nrec;
    const uint32_t *out = c.ms.out;
    const int sub = threadIdx.x & (G - 1);
    const int64_t gi = (int64_t)bid * (blockDim.x / G) + threadIdx.x / G;
    const int64_t gs = (int64_t)nb * (blockDim.x / G);
    const int64_t cnt = ri.cn[0];
    const int64_t lim = (cnt + gs - 1) / gs * gs;   // uniform trip count (group shuffles)
    for (int64_t i = gi; i < lim; i += gs) {
        int32_t v = -1;
        bool act = false;
        uint32_t av = 0;
        int64_t rb = 0, re = 0;
        if (i < cnt) {
            if (FIRST) {
                v = (int32_t)i;
                rb = g.xadj[v];
                re = g.xadj[v + 1];
                act = re - rb >= 1 && re - rb <= c.t.bin_small_max && graph_active(c, g, v);
                if (act) av = attr_src<R>(g, out, v);
            } else {
                v = checked_node(ri.in[0].v[i], g.n, c.ctrl);
                if (v >= 0 && !keeps_choice(ri.in[0].b[i], g.n, nrec)) {
                    act = true;
                    av = (uint32_t)nrec[v].x;
                    rb = g.xadj[v];
                    re = g.xadj[v + 1];
                    if (re - rb > BIN_SMALL_MAX) re = rb + BIN_SMALL_MAX;   // valid lists never
                }
            }
        }
        Cand cd = act ? scan_row_small<R, G, FIRST, F>(g, v, av, sub, rb, re, nrec, out,
                                                       row_seed(c, g, v, seed),
                                                       local_base(g, v), gv)
                      : cand_none();
        cd = group_reduce<G>(cd, v);
        if (act && sub == 0) {
            best[v] = cd.u;
            if (!FIRST) ri.in[0].b[i] = cd.u;
        }
    }
}

// bin 1: one wave per node
template <int R, bool FIRST, int F = 0>
__device__ __forceinline__ void pick_bin1(const Ctx &c, const DevGraph &g, uint64_t seed,
                                          const RoundIn &ri, unsigned bid, unsigned nb) {
    const GapView gv = gap_view(c);
    int32_t *best = c.ms.best;
    const int2 *nrec = c.ms.nrec;
    const uint32_t *out = c.ms.out;
    const int64_t gi = (int64_t)bid * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t gs = (int64_t)nb * (blockDim.x / WAVE);
    for (int64_t i = gi; i < ri.cn[1]; i += gs) {
        const int32_t v = checked_node(ri.in[1].v[i], g.n, c.ctrl);
        if (v < 0 || (!FIRST && keeps_choice(ri.in[1].b[i], g.n, nrec))) continue;   // wave-uniform
        const uint32_t av = FIRST ? attr_src<R>(g, out, v) : (uint32_t)nrec[v].x;
        Cand cd = scan_row<R, WAVE, FIRST, F>(g, v, av, lane_id(), nrec, out, row_seed(c, g, v, seed),
                                              local_base(g, v),
                                              gv);
        cd = group_reduce<WAVE>(cd, v);
        if (lane_id() == 0) {
            best[v] = cd.u;
            ri.in[1].b[i] = cd.u;
        }
    }
}

// bin 2: one block per node (blockDim.x lanes, a multiple of 64)
template <int R, bool FIRST, int NT, int F = 0>
__device__ __forceinline__ void pick_bin2(const Ctx &c, const DevGraph &g, uint64_t seed,
                                          const RoundIn &ri, unsigned bid, unsigned nb, Cand *sh) {
    const GapView gv = gap_view(c);
    int32_t *best = c.ms.best;
    const int2 *nrec = c.ms.nrec;
    const uint32_t *out = c.ms.out;
    for (int64_t i = bid; i < ri.cn[2]; i += nb) {
        const int32_t v = checked_node(ri.in[2].v[i], g.n, c.ctrl);
        if (v < 0 || (!FIRST && keeps_choice(ri.in[2].b[i], g.n, nrec))) continue;   // block-uniform
        const uint32_t av = FIRST ? attr_src<R>(g, out, v) : (uint32_t)nrec[v].x;
        Cand cd = scan_row<R, NT, FIRST, F>(g, v, av, threadIdx.x, nrec, out, row_seed(c, g, v, seed),
                                            local_base(g, v), gv);
        cd = block_reduce_cand(cd, v, sh);
        if (threadIdx.x == 0) {
            best[v] = cd.u;
            ri.in[2].b[i] = cd.u;
        }
    }
}

// Rounds >= 2 after a preparation: bins 0 and 1 over the rows to rescan
// ({node, list position}); the list's choice field is updated for the mutual
// check.
template <int R>
__device__ __forceinline__ void pick_scan0(const Ctx &c, const DevGraph &g, uint64_t seed,
                                           const RoundIn &ri, unsigned bid, unsigned nb) {
    const GapView gv = gap_view(c);
    const int G = SMALL_G;
    int32_t *best = c.ms.best;
    const int2 *nrec = c.ms.nrec;
    const int sub = threadIdx.x & (G - 1);
    const int64_t gi = (int64_t)bid * (blockDim.x / G) + threadIdx.x / G;
    const int64_t gs = (int64_t)nb * (blockDim.x / G);
    const int64_t cnt = ri.scn[0];
    const int64_t lim = (cnt + gs - 1) / gs * gs;   // uniform trip count (group shuffles)
    for (int64_t i = gi; i < lim; i += gs) {
        int2 e = make_int2(-1, -1);
        bool act = false;
        uint32_t av = 0;
        int64_t rb = 0, re = 0;
        if (i < cnt) {
            e = ri.scan[0][i];
            act = (uint32_t)e.x < (uint32_t)g.n && (uint32_t)e.y < (uint32_t)ri.cn[0];
            if (act) {
                av = (uint32_t)nrec[e.x].x;
                rb = g.xadj[e.x];
                re = g.xadj[e.x + 1];
                if (re - rb > BIN_SMALL_MAX) re = rb + BIN_SMALL_MAX;   // valid lists never
            }
        }
        Cand cd = act ? scan_row_small<R, G, false>(g, e.x, av, sub, rb, re, nrec, nullptr,
                                                    row_seed(c, g, e.x, seed),
                                                    local_base(g, e.x), gv)
                      : cand_none();
        cd = group_reduce<G>(cd, e.x);
        if (act && sub == 0) {
            best[e.x] = cd.u;
            ri.in[0].b[e.y] = cd.u;
        }
    }
}
template <int R>
__device__ __forceinline__ void pick_scan1(const Ctx &c, const DevGraph &g, uint64_t seed,
                                           const RoundIn &ri, unsigned bid, unsigned nb) {
    const GapView gv = gap_view(c);
    int32_t *best = c.ms.best;
    const int2 *nrec = c.ms.nrec;
    const int64_t gi = (int64_t)bid * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t gs = (int64_t)nb * (blockDim.x / WAVE);
    for (int64_t i = gi; i < ri.scn[1]; i += gs) {   // wave-uniform
        const int2 e = ri.scan[1][i];
        if ((uint32_t)e.x >= (uint32_t)g.n || (uint32_t)e.y >= (uint32_t)ri.cn[1]) continue;
        const uint32_t av = (uint32_t)nrec[e.x].x;
        Cand cd = scan_row<R, WAVE, false>(g, e.x, av, lane_id(), nrec, nullptr, row_seed(c, g, e.x, seed),
                                           local_base(g, e.x), gv);
        cd = group_reduce<WAVE>(cd, e.x);
        if (lane_id() == 0) {
            best[e.x] = cd.u;
            ri.in[1].b[e.y] = cd.u;
        }
    }
}

// bin 2 in the grid rounds: one block per chunk of HUB_CHUNK entries.  A row
// of one chunk gets its choice at once; longer rows keep one maximum per
// chunk in hub.part, at the row's round-1 records (hub.kfirst) for the whole
// level, for hub_reduce_k.  Records exist only for rows that scan this round
// (round 1: every row; later rounds: the rows whose choice was matched away,
// found by prep_k).  In a later round a chunk whose kept maximum is still
// free, or that had no free neighbour, keeps it without a scan: the free
// set only shrinks, so that maximum is still the chunk's best free
// neighbour.  r: the round (statistics).
template <int R, bool FIRST>
__device__ __forceinline__ void pick_bin2_chunks(const Ctx &c, const DevGraph &g, uint64_t seed,
                                                 const RoundIn &ri, unsigned bid, unsigned nb,
                                                 Cand *sh, int r) {
    constexpr int T = HUB_CHUNK / BLOCK;
    static_assert(T * BLOCK == HUB_CHUNK, "a chunk is T entries per thread");
    int32_t *best = c.ms.best;
    const int2 *nrec = c.ms.nrec;
    const uint32_t *out = c.ms.out;
    int64_t scanned = 0;   // entries scanned by this block (thread 0)
    for (int64_t q = bid; q < ri.nrec; q += nb) {   // block-uniform
        const int2 rc = ri.rec[q];
        if ((uint32_t)rc.x >= (uint32_t)ri.cn[2]) continue;   // valid records never
        const int32_t v = checked_node(ri.in[2].v[rc.x], g.n, c.ctrl);
        if (v < 0) continue;
        const int64_t rb = g.xadj[v], re = g.xadj[v + 1];
        const int32_t kc = hub_chunks_of(re - rb);
        const int32_t kf = kc > 1 ? c.ms.hub.kfirst[v] : 0;
        if (kc > 1 && (kf < 0 || (int64_t)kf + kc > c.ms.hub.cap)) {   // valid records never
            if (threadIdx.x == 0) atomicOr(&c.ctrl->flags, (uint32_t)CF_STATE);
            continue;
        }
        if (!FIRST && kc > 1) {
            const int32_t ku = c.ms.hub.part[kf + rc.y].u;
            if (ku < 0 || nrec[ku].y < 0) continue;
        }
        const int64_t j0 = rb + (int64_t)rc.y * HUB_CHUNK;
        const int64_t j1 = min(re, j0 + HUB_CHUNK);
        scanned += j1 - j0;
        const uint32_t av = FIRST ? attr_src<R>(g, out, v) : (uint32_t)nrec[v].x;
        const int32_t base = local_base(g, v);
        const uint64_t sv = row_seed(c, g, v, seed);
        // T entries per thread, strided by the block for coalesced row loads
        int32_t u[T];
        uint32_t w[T], au[T];
        bool ok[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int64_t j = j0 + (int64_t)t * BLOCK + threadIdx.x;
            ok[t] = j < j1;
            u[t] = ok[t] ? g.adj[j] : 0;
            w[t] = ok[t] ? g.ew[j] : 0u;
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            if (FIRST) {
                au[t] = ok[t] ? attr_src<R>(g, out, u[t]) : 0u;
            } else {
                const int2 rec = ok[t] ? nrec[u[t]] : make_int2(0, 0);
                ok[t] = ok[t] && rec.y < 0;
                au[t] = (uint32_t)rec.x;
            }
        }
        Cand cd = cand_none();
#pragma unroll
        for (int t = 0; t < T; ++t) {
            if (!ok[t]) continue;
            Cand e;
            rate<R>(w[t], au[t], av, au[t], av, e.num, e.den);
            e.h = mix64(sv ^ edge_id_local(v, u[t], base));
            e.u = u[t];
            if (cand_better(e, cd, v)) cd = e;
        }
        cd = block_reduce_cand(cd, v, sh);
        if (threadIdx.x == 0) {
            if (kc == 1) {
                best[v] = cd.u;
                ri.in[2].b[rc.x] = cd.u;
            } else {
                c.ms.hub.part[kf + rc.y] = cd;
            }
        }
    }
    if (!FIRST && c.rescan_stats && threadIdx.x == 0 && scanned > 0) {
        const int ri_ = r - 1 < STAT_ROUNDS ? r - 1 : STAT_ROUNDS - 1;
        atomicAdd((unsigned long long *)&c.ms.state->sstat[ri_][4][shard_of_block()],
                  (unsigned long long)scanned);
    }
}

// Mutual check of round r; matched pairs written (mate and the node
// record), survivors appended to the output lists (counters ocnt[3]).
// Round 1 also writes every node's record {attribute, mate}.  A thread's MK
// entries are loaded first, then their partners' choices, then stored.
template <int R, bool FIRST>
__device__ __forceinline__ void mate_phase(const Ctx &c, const DevGraph &g, LevelDesc *L, int r,
                                           const RoundIn &ri, int32_t *ocnt, unsigned bid,
                                           unsigned nb, int64_t *sh, int32_t *sbase) {
    MatchState *st = c.ms.state;
    int32_t *mate = L->mate;
    const int32_t *best = c.ms.best;
    int2 *nrec = c.ms.nrec;
    const uint32_t *out = c.ms.out;
    const int32_t n = g.n, c0 = ri.cn[0], c1 = ri.cn[1];
    const int64_t total = FIRST ? (int64_t)n : (int64_t)c0 + c1 + ri.cn[2];
    const int opar = r & 1;
    const PList ol[3] = {plist(c.ms, n, opar, 0), plist(c.ms, n, opar, 1), plist(c.ms, n, opar, 2)};
    int64_t point = 0, degs = 0, pairs = 0;
    int64_t scanned = 0, sdeg = 0;   // later rounds without chunked rows: every entry rescanned
    bool bad = false;
    // pass p, slot k of block b covers entries ((p * MK + k) * nb + b) * blockDim.x + t
    const int64_t row = (int64_t)nb * blockDim.x, per_pass = row * MK;
    for (int64_t base = 0; base < total; base += per_pass) {   // block-uniform
        const int64_t first = base + (int64_t)bid * blockDim.x + threadIdx.x;
        int bin[MK];
        int32_t vv[MK], bb[MK], dd[MK], bq[MK];
        uint32_t av[MK];
        // 1. the entries: node, choice, degree (and the attribute in round 1)
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            const int64_t i = first + (int64_t)k * row;
            vv[k] = -1;
            bb[k] = -1;
            dd[k] = 0;
            av[k] = 0;
            if (i >= total) continue;
            if (FIRST) {
                vv[k] = (int32_t)i;
                bb[k] = best[i];
                dd[k] = (int32_t)(g.xadj[i + 1] - g.xadj[i]);
                av[k] = attr_src<R>(g, out, (int32_t)i);
            } else {
                PList src;
                int64_t j;
                if (i < c0) { src = ri.in[0]; j = i; }
                else if (i < (int64_t)c0 + c1) { src = ri.in[1]; j = i - c0; }
                else { src = ri.in[2]; j = i - c0 - c1; }
                vv[k] = src.v[j];
                bb[k] = src.b[j];
                dd[k] = src.d[j];
            }
        }
        // 2. range checks (valid state never fails them), partners' choices
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            if ((uint32_t)vv[k] >= (uint32_t)n) {
                bad = bad || vv[k] != -1;
                vv[k] = -1;
            }
            if (vv[k] < 0 || (uint32_t)bb[k] >= (uint32_t)n) {
                bad = bad || (vv[k] >= 0 && bb[k] >= n);
                bb[k] = -1;
            }
            bq[k] = bb[k] >= 0 ? best[bb[k]] : -2;
        }
        // 3. decide and store
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            bin[k] = -1;
            const int32_t v = vv[k], b = bb[k];
            if (v < 0) continue;
            ++scanned;
            sdeg += dd[k];
            int32_t m = -1;
            if (b >= 0) {
                ++point;
                degs += dd[k];
                if (bq[k] == v) {
                    m = b;
                    if (v < b) ++pairs;
                } else {
                    bin[k] = bin_of(c, dd[k]);
                }
            }
            if (FIRST) {
                nrec[v] = make_int2((int32_t)av[k], m);
                if (m >= 0) mate[v] = m;
            } else if (m >= 0) {
                mate[v] = m;
                nrec[v].y = m;
            }
        }
        block_append_mk(bin, vv, bb, dd, ol, ocnt, sh, sbase);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&c.ctrl->flags, (uint32_t)CF_STATE);
    // with the rows this round's pick scanned, where it scans every pending
    // row (with chunked rows the preparation counts the rows that rescan),
    // while the profiler asks for them
    int64_t sums[5] = {point, degs, pairs, scanned, sdeg};
    if (c.rescan_stats) {
        block_sum_n<5>(sums, sh);
    } else {
        block_sum3(sums[0], sums[1], sums[2], sh);
        sums[3] = 0;
    }
    const int ri_ = r - 1 < STAT_ROUNDS ? r - 1 : STAT_ROUNDS - 1, sd = shard_of_block();
    if (threadIdx.x == 0 && sums[0] > 0) {
        atomicAdd((unsigned long long *)&st->sstat[ri_][0][sd], (unsigned long long)sums[0]);
        atomicAdd((unsigned long long *)&st->sstat[ri_][1][sd], (unsigned long long)sums[1]);
        if (sums[2]) atomicAdd((unsigned long long *)&st->sstat[ri_][2][sd], (unsigned long long)sums[2]);
        atomicMax(&st->sround[sd], r);
    }
    if (!FIRST && !c.ms.hub.rec && threadIdx.x == 0 && sums[3] > 0) {
        atomicAdd((unsigned long long *)&st->sstat[ri_][3][sd], (unsigned long long)sums[3]);
        atomicAdd((unsigned long long *)&st->sstat[ri_][4][sd], (unsigned long long)sums[4]);
    }
}

// --- per-round kernels -----------------------------------------------------
// The level's first kernel: gate, then mate = best = -1 and the round-1
// lists.  Block 0 also resets the matching state (read by later kernels).
// The list counters and round statistics are zero on entry (reset by the
// previous level's finisher, or by the host before level 0).
// lists = 0 (two-phase matcher): gate and resets only; the block phase
// writes mate, best, the node records and the lists.
__global__ void __launch_bounds__(BLOCK) match_init_k(Ctx c, int l, int stop_rules, int lists) {
    __shared__ int64_t sh[BLOCK / WAVE + 1];
    __shared__ int32_t sbase[3];
    __shared__ int go;
    if (threadIdx.x == 0) go = level_gate(c, l, stop_rules != 0, blockIdx.x == 0);
    __syncthreads();
    if (!go) return;
    LevelDesc *L = c.lv + l;
    DevGraph g;
    g.n = L->n; g.nnz = L->nnz; g.xadj = L->xadj; g.adj = L->adj; g.ew = L->ew; g.vw = L->vw;
    g.gid = L->gid; g.noff = L->noff;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the round statistics are zero on entry (the previous level's
        // finisher, or the host before level 0, cleared them)
        c.ms.state->handoff = -1;
        L->matched = 0;
        L->rounds = 0;
    }
    if (lists) init_phase(c, g, L, sh, sbase, blockIdx.x, gridDim.x, &c.ms.state->cnt[0][0], true);
}

struct PickGrid {
    unsigned b0, b1, b2;  // blocks per bin
};

// SCAN (rounds >= 2, long rows in chunks): the rows prep_k found to rescan.
template <int R, bool FIRST, int F = 0, bool SCAN = false>
__global__ void __launch_bounds__(BLOCK) pick_k(Ctx c, int l, int r, PickGrid pg) {
    __shared__ Cand sh[BLOCK / WAVE];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_MATCH, g)) return;
    MatchState *st = c.ms.state;
    if (st->handoff != -1) return;
    const RoundIn ri = round_inputs<FIRST>(c, g, r, st->cnt[FIRST ? 0 : (r - 1) & 3]);
    if (!FIRST) {
        const int64_t total = (int64_t)ri.cn[0] + ri.cn[1] + ri.cn[2];
        if (total == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&st->handoff, -1, -2);
            return;
        }
        if (total <= c.t.tail_max) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&st->handoff, -1, r - 1);
            return;
        }
    }
    const uint64_t seed = level_seed(c, l);
    unsigned bid = blockIdx.x;
    if (SCAN) {
        if (bid < pg.b0) { pick_scan0<R>(c, g, seed, ri, bid, pg.b0); return; }
        bid -= pg.b0;
        if (bid < pg.b1) { pick_scan1<R>(c, g, seed, ri, bid, pg.b1); return; }
        bid -= pg.b1;
        pick_bin2_chunks<R, false>(c, g, seed, ri, bid, pg.b2, sh, r);
        return;
    }
    if (bid < pg.b0) { pick_bin0<R, FIRST, F>(c, g, seed, ri, bid, pg.b0); return; }
    bid -= pg.b0;
    if (bid < pg.b1) { pick_bin1<R, FIRST, F>(c, g, seed, ri, bid, pg.b1); return; }
    bid -= pg.b1;
    if (F == 0 && ri.rec)
        pick_bin2_chunks<R, FIRST>(c, g, seed, ri, bid, pg.b2, sh, r);
    else
        pick_bin2<R, FIRST, BLOCK, F>(c, g, seed, ri, bid, pg.b2, sh);
}

// Preparation of round r >= 2 (long rows in chunks): every pending entry
// whose choice was matched away in round r - 1 must rescan its row.  Rows of
// bins 0 and 1 go to the scan lists ({node, list position}); bin-2 rows get
// their chunk records (first = the row's first record, -1 for a row that
// keeps its choice).  Also applies the hand-over tests of the round (nothing
// pending, or few enough for the finisher).  A thread's MK entries are loaded
// together.
__global__ void __launch_bounds__(BLOCK) prep_k(Ctx c, int l, int r) {
    __shared__ int64_t sh[5 * (BLOCK / WAVE) + 1];
    __shared__ int32_t sbase[2];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_MATCH, g)) return;
    MatchState *st = c.ms.state;
    if (st->handoff != -1 || !c.ms.hub.rec) return;
    const RoundIn ri = round_inputs<false>(c, g, r, st->cnt[(r - 1) & 3]);
    const int32_t c0 = ri.cn[0], c1 = ri.cn[1];
    const int64_t total = (int64_t)c0 + c1 + ri.cn[2];
    if (total == 0 || total <= c.t.tail_max) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicCAS(&st->handoff, -1, total == 0 ? -2 : r - 1);
        return;
    }
    int32_t *sc = st->scnt[r & 3];
    int2 *const scan0 = c.ms.hub.scan, *const scan1 = c.ms.hub.scan + g.n;
    const int par = (r - 1) & 1;
    const HubOut ho{c.ms.hub.rec + (int64_t)par * c.ms.hub.cap,
                    c.ms.hub.first + (int64_t)par * g.n, sc + 3, c.ms.hub.cap, nullptr};
    const int2 *nrec = c.ms.nrec;
    const int64_t row = (int64_t)gridDim.x * blockDim.x, per_pass = row * MK;
    int64_t rrows = 0, rdeg = 0;   // the round's rescanning rows and their degrees
    for (int64_t base = 0; base < total; base += per_pass) {   // block-uniform
        const int64_t first = base + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        int32_t vv[MK], bb[MK], dd[MK], jj[MK], bin[MK];
        bool resc[MK];
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            const int64_t i = first + (int64_t)k * row;
            bin[k] = -1;
            vv[k] = bb[k] = -1;
            dd[k] = 0;
            jj[k] = 0;
            if (i >= total) continue;
            PList src;
            if (i < c0) { src = ri.in[0]; jj[k] = (int32_t)i; bin[k] = 0; }
            else if (i < (int64_t)c0 + c1) { src = ri.in[1]; jj[k] = (int32_t)(i - c0); bin[k] = 1; }
            else { src = ri.in[2]; jj[k] = (int32_t)(i - c0 - c1); bin[k] = 2; }
            vv[k] = src.v[jj[k]];
            bb[k] = src.b[jj[k]];
            dd[k] = src.d[jj[k]];
        }
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            const bool live = bin[k] >= 0 && (uint32_t)vv[k] < (uint32_t)g.n;
            resc[k] = live && !keeps_choice(bb[k], g.n, nrec);
            if (bin[k] >= 0 && !live) bin[k] = -1;   // valid lists never
            if (resc[k]) {
                ++rrows;
                if (bin[k] < 2) rdeg += dd[k];   // chunked rows: the pick counts what it scans
            }
        }
        // rows of bins 0 and 1 that rescan: block-aggregated append
        int64_t packed = 0;
#pragma unroll
        for (int k = 0; k < MK; ++k)
            if (resc[k] && bin[k] < 2) packed += (int64_t)1 << (21 * bin[k]);
        int64_t tot;
        const int64_t pre = block_excl_scan(packed, sh, &tot);
        if (threadIdx.x < 2) {
            const int32_t t = (int32_t)((tot >> (21 * threadIdx.x)) & 0x1fffff);
            sbase[threadIdx.x] = t ? atomicAdd(&sc[threadIdx.x], t) : 0;
        }
        __syncthreads();
        int32_t p0 = sbase[0] + (int32_t)(pre & 0x1fffff);
        int32_t p1 = sbase[1] + (int32_t)((pre >> 21) & 0x1fffff);
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            if (bin[k] == 2) {
                if (resc[k]) hub_emit(ho, jj[k], vv[k], dd[k], c.ctrl);
                else ho.first[jj[k]] = -1;
            } else if (resc[k]) {
                if (bin[k] == 0) scan0[p0++] = make_int2(vv[k], jj[k]);
                else scan1[p1++] = make_int2(vv[k], jj[k]);
            }
        }
        __syncthreads();   // sbase is reused by the next pass
    }
    if (!c.rescan_stats) return;
    int64_t none = 0;
    block_sum3(rrows, rdeg, none, sh);
    if (threadIdx.x == 0 && rrows > 0) {
        const int ri_ = r - 1 < STAT_ROUNDS ? r - 1 : STAT_ROUNDS - 1, sd = shard_of_block();
        atomicAdd((unsigned long long *)&st->sstat[ri_][3][sd], (unsigned long long)rrows);
        atomicAdd((unsigned long long *)&st->sstat[ri_][4][sd], (unsigned long long)rdeg);
    }
}

// The choices of bin-2 rows of more than one chunk: the best of their
// chunks' maxima (one wave per row).  Runs between the pick and the mate
// launches of a grid round, under the same gates.
template <bool FIRST>
__global__ void __launch_bounds__(BLOCK) hub_reduce_k(Ctx c, int l, int r) {
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_MATCH, g)) return;
    MatchState *st = c.ms.state;
    if (st->handoff != -1 || !c.ms.hub.rec) return;
    const RoundIn ri = round_inputs<FIRST>(c, g, r, st->cnt[FIRST ? 0 : (r - 1) & 3]);
    int32_t *best = c.ms.best;
    const int64_t gi = (int64_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE;
    const int64_t gs = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t i = gi; i < ri.cn[2]; i += gs) {   // wave-uniform
        const int32_t f = ri.first[i];   // -1: the row keeps its choice (prep_k)
        if (f < 0) continue;
        const int32_t v = ri.in[2].v[i];
        if ((uint32_t)v >= (uint32_t)g.n) continue;   // flagged by the pick
        const int32_t k = hub_chunks_of(g.xadj[v + 1] - g.xadj[v]);
        if (k <= 1) continue;
        const int32_t kf = c.ms.hub.kfirst[v];   // the row's chunk maxima for the level
        if (kf < 0 || (int64_t)kf + k > c.ms.hub.cap) continue;   // flagged by the pick
        Cand cd = cand_none();
        for (int32_t q = lane_id(); q < k; q += WAVE) {
            const Cand o = c.ms.hub.part[kf + q];
            if (cand_better(o, cd, v)) cd = o;
        }
        cd = group_reduce<WAVE>(cd, v);
        if (lane_id() == 0) {
            best[v] = cd.u;
            ri.in[2].b[i] = cd.u;
        }
    }
}

template <int R, bool FIRST>
__global__ void __launch_bounds__(BLOCK) mate_k(Ctx c, int l, int r) {
    __shared__ int64_t sh[5 * (BLOCK / WAVE) + 1];
    __shared__ int32_t sbase[3];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_MATCH, g)) return;
    MatchState *st = c.ms.state;
    if (st->handoff != -1) return;
    const RoundIn ri = round_inputs<FIRST>(c, g, r, st->cnt[FIRST ? 0 : (r - 1) & 3]);
    // the counters of round r + 2 were last read by round r - 1 (list sizes)
    // and round r - 2 (rescan counts)
    if (blockIdx.x == 0 && threadIdx.x < 4) {
        st->cnt[(r + 2) & 3][threadIdx.x] = 0;
        st->scnt[(r + 2) & 3][threadIdx.x] = 0;
    }
    mate_phase<R, FIRST>(c, g, L, r, ri, st->cnt[r & 3], blockIdx.x, gridDim.x, sh, sbase);
}

// Rounds r0+1, r0+2, ... of level L in one workgroup of NT threads, with
// workgroup barriers, until no node is pending; s_cnt[r0 & 1] holds the list
// sizes round r0 left.  Every round that has a pointing node matches at least
// one pair, so at most n/2 + 1 rounds remain; returns true only if that cap
// was hit (broken state).
template <int R, int NT, int F = 0>
__device__ bool wg_rounds(const Ctx &c, const DevGraph &g, LevelDesc *L, uint64_t seed, int r0,
                          int32_t (*s_cnt)[4], Cand *shc, int64_t *sh, int32_t *sbase) {
    const int64_t r_cap = (int64_t)r0 + 2 + g.n;
    for (int r = r0 + 1; r <= r_cap; ++r) {
        const RoundIn ri = round_inputs<false>(c, g, r, s_cnt[(r - 1) & 1]);
        if ((int64_t)ri.cn[0] + ri.cn[1] + ri.cn[2] == 0) return false;
        pick_bin0<R, false, F>(c, g, seed, ri, 0, 1);
        pick_bin1<R, false, F>(c, g, seed, ri, 0, 1);
        __syncthreads();
        pick_bin2<R, false, NT, F>(c, g, seed, ri, 0, 1, shc);
        if (threadIdx.x < 3) s_cnt[r & 1][threadIdx.x] = 0;
        __syncthreads();
        mate_phase<R, false>(c, g, L, r, ri, s_cnt[r & 1], 0, 1, sh, sbase);
        __syncthreads();
    }
    return true;
}

// Closes level L's matching in one workgroup of NT threads: sums the round
// statistics over the rounds used (one wave per statistic) and leaves them,
// the list counters and the contraction counters zero; records |M|, the
// round count and how many rounds ran as grid launches (grid_r0: rounds up to
// grid_r0 did, -2: all did); ends the level loop on an empty matching.
// defer (the gap rounds of the two-phase matcher): the level moves to
// PH_MERGE instead, where the merged matching decides.
template <int NT>
__device__ void close_matching(const Ctx &c, LevelDesc *L, bool capped, int grid_r0,
                               int64_t *s_acc, bool defer = false) {
    MatchState *st = c.ms.state;
    __syncthreads();
    if (threadIdx.x < WAVE) {
        const int32_t rr = wave_max(st->sround[lane_id()]);
        st->sround[lane_id()] = 0;
        if (lane_id() == 0) {
            s_acc[0] = 0;
            s_acc[1] = rr;
        }
    }
    __syncthreads();
    {
        const int w = threadIdx.x / WAVE, nw = NT / WAVE;
        const int slots = (int)min<int64_t>(s_acc[1], STAT_ROUNDS);
        for (int q = w; q < slots * 5; q += nw) {
            const int i = q / 5, f = q % 5;
            int64_t *p = &st->sstat[i][f][lane_id()];
            const int64_t v = wave_sum(*p);
            *p = 0;
            if (lane_id() == 0) {
                if (f < 2) L->stat[i][f] = v;
                else if (f == 2) {
                    if (v) atomicAdd((unsigned long long *)&s_acc[0], (unsigned long long)v);
                } else {
                    L->stat[i][f - 1] = v;
                }
            }
        }
    }
    if (threadIdx.x < 8) c.cs.row_cnt[threadIdx.x] = 0;
    if (threadIdx.x < 4 && c.cs.hg_cnt) c.cs.hg_cnt[threadIdx.x] = 0;
    if (threadIdx.x < 4) c.cs.totals[threadIdx.x] = 0;
    __syncthreads();   // every read of st->cnt is done
    if (threadIdx.x < 16) {   // next level's lists
        st->cnt[threadIdx.x >> 2][threadIdx.x & 3] = 0;
        st->scnt[threadIdx.x >> 2][threadIdx.x & 3] = 0;
    }
    if (threadIdx.x == 0) {
        int64_t m = s_acc[0];
        const int32_t used = (int32_t)s_acc[1];
        st->handoff = -2;
        L->matched = m;
        L->rounds = used;
        L->grid_rounds = grid_r0 < 0 ? used : min(grid_r0, used);
        if (capped) c.ctrl->flags |= CF_ROUNDS;
        if (defer && !capped) {
            L->phase = PH_MERGE;
        } else if (m == 0 || capped) {
            L->stop = KAPPA_STOP_EMPTY;
            L->phase = PH_STOPPED;
            c.ctrl->done = 1;
        } else {
            L->phase = PH_CONTRACT;
        }
    }
    __syncthreads();
}

// Finisher: one workgroup runs the remaining rounds (from the handoff point,
// or after round r_last) with workgroup barriers, then closes the level's
// matching.
template <int R, int F = 0>
__global__ void __launch_bounds__(FINISH_THREADS) finish_k(Ctx c, int l, int r_last) {
    __shared__ Cand shc[FINISH_THREADS / WAVE];
    __shared__ int64_t sh[5 * (FINISH_THREADS / WAVE) + 1];
    __shared__ int32_t s_cnt[2][4];
    __shared__ int32_t sbase[3];
    __shared__ int64_t s_acc[2];
    __shared__ int32_t s_r0;
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_MATCH, g)) return;
    MatchState *st = c.ms.state;
    const uint64_t seed = level_seed(c, l);
    if (threadIdx.x == 0) {
        int h = st->handoff;
        if (h == -1) h = r_last;   // every round up to r_last ran: take over from there
        s_r0 = h;
    }
    __syncthreads();
    const int r0 = s_r0;
    bool capped = false;
    if (r0 >= 0) {
        if (threadIdx.x < 3) {
            s_cnt[r0 & 1][threadIdx.x] = st->cnt[r0 & 3][threadIdx.x];
            s_cnt[(r0 + 1) & 1][threadIdx.x] = 0;
        }
        __syncthreads();
        // the launched grid rounds ran out with many nodes pending (graphs
        // whose matching needs more rounds than the host planned, such as
        // power-law graphs): one workgroup would crawl through them, so the
        // level goes back to the host for more grid rounds.  The level stays
        // in PH_MATCH; `done` ends this batch of levels.
        const int32_t pend = s_cnt[r0 & 1][0] + s_cnt[r0 & 1][1] + s_cnt[r0 & 1][2];
        if (F == 0 && st->handoff == -1 && r0 == r_last &&
            (pend > c.t.finish_max || s_cnt[r0 & 1][2] > c.t.finish_max_big)) {
            if (threadIdx.x == 0) {
                c.ctrl->ext_level = l;
                c.ctrl->ext_round = r_last;
                c.ctrl->flags |= CF_EXTEND;
                c.ctrl->done = 1;
            }
            return;
        }
        capped = wg_rounds<R, FINISH_THREADS, F>(c, g, L, seed, r0, s_cnt, shc, sh, sbase);
    }
    // r0 = -2: the round kernels found nothing left, so they ran every round
    close_matching<FINISH_THREADS>(c, L, capped, r0, s_acc, F != 0);
}

// ===========================================================================
// Two-phase matcher (Section 3.3)
// ===========================================================================
// Block phase.  One workgroup matches the nodes of one block [v0, v0 + nb)
// of 2^bb consecutive ids: local-max rounds over the edges inside the block,
// the block's state in LDS and workgroup barriers between rounds.  Under the
// strict order this is Greedy on the block's edges, the sequential matcher
// the paper runs per processor.  Then, per node: the block partner (loc),
// the key of that edge (written by the node's last choice), the node record
// {attribute, free} and mate = best = -1 for the gap rounds; a node with an
// edge to another block above its own block edge enters the gap rounds'
// first lists (a node without one has no gap edge: every gap edge is above
// the block edges at both ends).
constexpr int BM_MAX = 1 << BM_BITS_MAX;
constexpr int BM_STAGE = 8192;   // CSR entries of a block staged in LDS (more: rows read from HBM)
static_assert(MK * BM_THREADS >= BM_MAX, "the list step covers a block in one pass");
static_assert(BM_MAX <= 32768 && BM_STAGE <= 32768, "local indices are 16-bit");

// The rows of a block are contiguous in the CSR: entry j of the block is
// entry e0 + j of the graph.  Staged blocks keep, per entry, the neighbour's
// local index (-1: another block) and the weight in LDS, and the row
// offsets relative to e0.
struct BlockRows {
    int64_t e0;
    bool staged;
    const int16_t *nbr;
    const uint32_t *w;
    const int32_t *roff;
};
__device__ __forceinline__ void block_row(const DevGraph &g, const BlockRows &br, int32_t v,
                                          int i, int64_t &rb, int64_t &re) {
    if (br.staged) {
        rb = br.roff[i];
        re = br.roff[i + 1];
    } else {
        rb = g.xadj[v] - br.e0;
        re = g.xadj[v + 1] - br.e0;
    }
}

// v's best free neighbour inside the block over the entries sub, sub+G, ...
// of [rb, re) (block-relative).  s_mate: LDS state; s_attr: attributes.
template <int R, int G, bool STAGED>
__device__ __forceinline__ Cand block_scan(const DevGraph &g, const BlockRows &br, int32_t v,
                                           int32_t v0, int32_t nb, uint32_t av, int64_t rb,
                                           int64_t re, int sub, const int16_t *s_mate,
                                           const uint32_t *s_attr, uint64_t seed) {
    Cand best = cand_none();
    for (int64_t j = rb + sub; j < re; j += G) {
        int32_t iu;
        uint32_t w;
        if (STAGED) {
            iu = br.nbr[j];
            if (iu < 0) continue;   // another block
            w = br.w[j];
        } else {
            iu = g.adj[br.e0 + j] - v0;
            if ((uint32_t)iu >= (uint32_t)nb) continue;
            w = g.ew[br.e0 + j];
        }
        if (s_mate[iu] >= 0) continue;   // taken
        Cand cd;
        rate<R>(w, s_attr[iu], av, s_attr[iu], av, cd.num, cd.den);
        cd.u = v0 + iu;
        cd.h = mix64(seed ^ edge_id(v, cd.u));
        if (cand_better(cd, best, v)) best = cd;
    }
    return best;
}

// Is some edge from v to another block above kv (v's block edge, or none)?
// Over the entries sub, sub+G, ... of [rb, re).
template <int R, int G>
__device__ __forceinline__ bool block_gap_any(const DevGraph &g, const BlockRows &br, int32_t v,
                                              int32_t v0, int32_t nb, uint32_t av, int64_t rb,
                                              int64_t re, int sub, const Cand &kv,
                                              const uint32_t *out, uint64_t seed) {
    bool any = false;
    for (int64_t j = rb + sub; j < re && !any; j += G) {
        if (br.staged && br.nbr[j] >= 0) continue;
        const int32_t u = g.adj[br.e0 + j];
        if ((uint32_t)(u - v0) < (uint32_t)nb) continue;
        const uint32_t au = attr_src<R>(g, out, u);
        Cand cd;
        rate<R>(br.staged ? br.w[j] : g.ew[br.e0 + j], au, av, au, av, cd.num, cd.den);
        cd.u = u;
        cd.h = mix64(seed ^ edge_id(v, u));
        any = cand_better(cd, kv, v);
    }
    return any;
}

template <int G>
__device__ __forceinline__ bool group_any(bool x) {
    int a = x ? 1 : 0;
    for (int off = G / 2; off > 0; off >>= 1) a |= __shfl_xor(a, off, G);
    return a != 0;
}

// two workgroups per CU (LDS allows two; registers are held to 128)
template <int R>
__global__ void __launch_bounds__(BM_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
block_match_k(Ctx c, int l) {
    // s_best: local index of the current choice; -1 none yet, -2 no free
    // neighbour inside the block left (free sets only shrink).  After the
    // rounds it holds the gap-list flag.
    __shared__ int16_t s_mate[BM_MAX], s_best[BM_MAX], s_big[BM_MAX];
    __shared__ uint32_t s_attr[BM_MAX];
    __shared__ int32_t s_roff[BM_MAX + 1];
    __shared__ int16_t s_nbr[BM_STAGE];
    __shared__ uint32_t s_w[BM_STAGE];
    __shared__ int32_t s_nbig, s_pt[2];
    __shared__ int64_t sh[BM_THREADS / WAVE + 1];
    __shared__ int32_t sbase[3];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_MATCH, g)) return;
    const int bb = c.block_bits;
    const uint64_t seed = level_seed(c, l);
    const uint32_t *out = c.ms.out;
    const int64_t nblocks = ((int64_t)g.n + ((int64_t)1 << bb) - 1) >> bb;
    const PList ol[3] = {plist(c.ms, g.n, 0, 0), plist(c.ms, g.n, 0, 1), plist(c.ms, g.n, 0, 2)};
    constexpr int G = SMALL_G, GS = BM_THREADS / G;
    const int sub = threadIdx.x & (G - 1);
    for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {   // block-uniform
        const int32_t v0 = (int32_t)(blk << bb);
        const int32_t nb = (int32_t)min<int64_t>((int64_t)1 << bb, (int64_t)g.n - v0);
        BlockRows br;
        br.e0 = g.xadj[v0];
        const int64_t ne = g.xadj[v0 + nb] - br.e0;
        br.staged = ne <= BM_STAGE;   // block-uniform
        br.nbr = s_nbr;
        br.w = s_w;
        br.roff = s_roff;
        if (threadIdx.x == 0) {
            s_nbig = 0;
            s_pt[0] = 0;
            s_pt[1] = 0;
            if (br.staged) s_roff[nb] = (int32_t)ne;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += BM_THREADS) {
            const int32_t v = v0 + i;
            const int64_t rb = g.xadj[v], deg = g.xadj[v + 1] - rb;
            if (br.staged) s_roff[i] = (int32_t)(rb - br.e0);
            s_mate[i] = -1;
            s_best[i] = deg == 0 ? -2 : -1;
            s_attr[i] = attr_src<R>(g, out, v);
            if (deg > BIN_SMALL_MAX) s_big[atomicAdd(&s_nbig, 1)] = (int16_t)i;
        }
        if (br.staged) {
            for (int64_t j = threadIdx.x; j < ne; j += BM_THREADS) {
                const int32_t iu = g.adj[br.e0 + j] - v0;
                s_nbr[j] = (uint32_t)iu < (uint32_t)nb ? (int16_t)iu : (int16_t)-1;
                s_w[j] = g.ew[br.e0 + j];
            }
        }
        __syncthreads();
        const int nbig = s_nbig;
        // every round with a pointing node matches the top pair among them,
        // so at most nb/2 + 1 rounds run
        for (int r = 0;; ++r) {   // block-uniform
            const int par = r & 1;
            {   // small rows: G lanes per node
                const int lim = (nb + GS - 1) / GS * GS;   // uniform trip count (group shuffles)
                for (int i = threadIdx.x / G; i < lim; i += GS) {
                    bool act = false;
                    int64_t rb = 0, re = 0;
                    const int32_t v = v0 + i;
                    if (i < nb && s_mate[i] < 0) {
                        const int b = s_best[i];
                        if (b >= 0 && s_mate[b] < 0) {   // keeps its choice: still the best
                            if (sub == 0) s_pt[par] = 1;
                        } else if (b != -2) {
                            block_row(g, br, v, i, rb, re);
                            act = re - rb <= BIN_SMALL_MAX;
                        }
                    }
                    Cand cd = cand_none();
                    if (act)
                        cd = br.staged ? block_scan<R, G, true>(g, br, v, v0, nb, s_attr[i], rb, re,
                                                                sub, s_mate, s_attr, seed)
                                       : block_scan<R, G, false>(g, br, v, v0, nb, s_attr[i], rb, re,
                                                                 sub, s_mate, s_attr, seed);
                    cd = group_reduce<G>(cd, v);
                    if (act && sub == 0) {
                        if (cd.u >= 0) {
                            s_best[i] = (int16_t)(cd.u - v0);
                            c.ms.lkey[v] = LocKey{cd.num, cd.den, cd.h};
                            s_pt[par] = 1;
                        } else {
                            s_best[i] = -2;
                        }
                    }
                }
            }
            {   // larger rows: one wave per node
                const int w = threadIdx.x / WAVE, nw = BM_THREADS / WAVE;
                for (int q = w; q < nbig; q += nw) {
                    const int i = s_big[q];
                    const int b = s_best[i];
                    if (s_mate[i] >= 0 || b == -2) continue;   // wave-uniform
                    if (b >= 0 && s_mate[b] < 0) {
                        if (lane_id() == 0) s_pt[par] = 1;
                        continue;
                    }
                    const int32_t v = v0 + i;
                    int64_t rb, re;
                    block_row(g, br, v, i, rb, re);
                    Cand cd = br.staged ? block_scan<R, WAVE, true>(g, br, v, v0, nb, s_attr[i], rb,
                                                                    re, lane_id(), s_mate, s_attr,
                                                                    seed)
                                        : block_scan<R, WAVE, false>(g, br, v, v0, nb, s_attr[i],
                                                                     rb, re, lane_id(), s_mate,
                                                                     s_attr, seed);
                    cd = group_reduce<WAVE>(cd, v);
                    if (lane_id() == 0) {
                        if (cd.u >= 0) {
                            s_best[i] = (int16_t)(cd.u - v0);
                            c.ms.lkey[v] = LocKey{cd.num, cd.den, cd.h};
                            s_pt[par] = 1;
                        } else {
                            s_best[i] = -2;
                        }
                    }
                }
            }
            __syncthreads();
            const bool go = s_pt[par] != 0;
            if (go) {   // pairs that chose each other
                for (int i = threadIdx.x; i < nb; i += BM_THREADS) {
                    const int b = s_best[i];
                    if (s_mate[i] < 0 && b >= 0 && s_best[b] == i) s_mate[i] = (int16_t)b;
                }
            }
            if (threadIdx.x == 0) s_pt[par ^ 1] = 0;   // read again only after the barrier
            __syncthreads();
            if (!go) break;
            if (r > nb / 2 + 2) {   // cannot happen on valid state
                if (threadIdx.x == 0) atomicOr(&c.ctrl->flags, (uint32_t)CF_ROUNDS);
                break;
            }
        }
        // gap-list flags (into s_best): an edge to another block above the
        // node's block edge
        {
            const int lim = (nb + GS - 1) / GS * GS;
            for (int i = threadIdx.x / G; i < lim; i += GS) {
                bool act = false;
                int64_t rb = 0, re = 0;
                const int32_t v = v0 + i;
                Cand kv = cand_none();
                if (i < nb) {
                    block_row(g, br, v, i, rb, re);
                    act = re - rb <= BIN_SMALL_MAX;
                    if (act && s_mate[i] >= 0) {
                        const LocKey q = c.ms.lkey[v];
                        kv.num = q.num;
                        kv.den = q.den;
                        kv.h = q.h;
                        kv.u = v0 + s_mate[i];
                    }
                }
                const bool any = group_any<G>(
                    act && block_gap_any<R, G>(g, br, v, v0, nb, s_attr[i], rb, re, sub, kv, out,
                                               seed));
                if (act && sub == 0) s_best[i] = any ? 1 : 0;
            }
            const int w = threadIdx.x / WAVE, nw = BM_THREADS / WAVE;
            for (int q = w; q < nbig; q += nw) {
                const int i = s_big[q];
                const int32_t v = v0 + i;
                int64_t rb, re;
                block_row(g, br, v, i, rb, re);
                Cand kv = cand_none();
                if (s_mate[i] >= 0) {
                    const LocKey k = c.ms.lkey[v];
                    kv.num = k.num;
                    kv.den = k.den;
                    kv.h = k.h;
                    kv.u = v0 + s_mate[i];
                }
                const bool any = __ballot(block_gap_any<R, WAVE>(g, br, v, v0, nb, s_attr[i], rb, re,
                                                                 lane_id(), kv, out, seed)) != 0;
                if (lane_id() == 0) s_best[i] = any ? 1 : 0;
            }
        }
        __syncthreads();
        // the block matching, the gap rounds' state and their first lists
        int bin[MK];
        int32_t vv[MK], bq[MK], dd[MK];
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            const int i = threadIdx.x + k * BM_THREADS;   // MK * BM_THREADS >= BM_MAX
            bin[k] = -1;
            vv[k] = v0 + i;
            bq[k] = -1;
            dd[k] = 0;
            if (i >= nb) continue;
            const int32_t v = v0 + i;
            const int m = s_mate[i];
            c.ms.loc[v] = m >= 0 ? v0 + m : -1;
            L->mate[v] = -1;
            c.ms.best[v] = -1;
            c.ms.nrec[v] = make_int2((int32_t)s_attr[i], -1);
            if (s_best[i] == 1) {
                const int64_t deg = g.xadj[v + 1] - g.xadj[v];
                dd[k] = (int32_t)deg;
                bin[k] = bin_of(c, deg);
            }
        }
        block_append_mk(bin, vv, bq, dd, ol, &c.ms.state->cnt[0][0], sh, sbase);
        __syncthreads();   // LDS is reused by the next block
    }
}

// Merge: a gap edge replaces the block edges at its ends; a node whose
// block partner took a gap edge stays unmatched.  Gap partners are read from
// the node records (their mate field), block partners from loc.
__global__ void __launch_bounds__(BLOCK) merge_k(Ctx c, int l) {
    __shared__ int64_t sh[5 * (BLOCK / WAVE) + 1];
    LevelDesc *L = c.lv + l;
    if (L->phase != PH_MERGE) return;
    const int32_t n = L->n;
    const int2 *nrec = c.ms.nrec;
    int64_t pairs = 0, z0 = 0, z1 = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t m = nrec[i].y;
        if (m < 0) {
            const int32_t lc = c.ms.loc[i];
            if (lc >= 0 && nrec[lc].y < 0) m = lc;
        }
        L->mate[i] = m;
        pairs += m > i;
    }
    block_sum3(pairs, z0, z1, sh);
    if (threadIdx.x == 0 && pairs)
        atomicAdd((unsigned long long *)&c.ms.state->spairs[shard_of_block()],
                  (unsigned long long)pairs);
}

// |M| of the merged matching; ends the level loop if it is empty.
__global__ void __launch_bounds__(WAVE) merge_close_k(Ctx c, int l) {
    LevelDesc *L = c.lv + l;
    if (L->phase != PH_MERGE) return;
    int64_t *p = &c.ms.state->spairs[lane_id()];
    const int64_t m = wave_sum(*p);
    *p = 0;
    if (lane_id() == 0) {
        L->matched = m;
        if (m == 0) {
            L->stop = KAPPA_STOP_EMPTY;
            L->phase = PH_STOPPED;
            c.ctrl->done = 1;
        } else {
            L->phase = PH_CONTRACT;
        }
    }
}

// ===========================================================================
// Contraction
// ===========================================================================
constexpr uint32_t INVALID_KEY = 0xffffffffu;
constexpr int SM_ROWS = BLOCK / ROW_SMALL_G;      // 16 small rows per block
// entries incl. the dropped edge, rounded to whole 16-byte reads
constexpr int SM_CAP = (ROW_SMALL_MAX + 2 + 3) / 4 * 4;
constexpr int MID_P = 4096;

// --- 1. coarse ids: scan of representative flags; the apply writes the whole
//        coarse node (cmap of both ends, rep_of, partner, c(x)) ----------------
struct RepF {
    Ctx c;
    int l;
    __device__ int64_t size() const {
        const LevelDesc *L = c.lv + l;
        return L->phase == PH_CONTRACT ? L->n : -1;
    }
    // representatives: unmatched nodes and the smaller end of each pair (the
    // nodes of a stopped graph in a batch are none: they leave the union)
    __device__ int64_t operator()(int64_t i) const {
        const LevelDesc *L = c.lv + l;
        const int32_t m = L->mate[i];
        if (L->gid && !c.b.active[L->gid[i]]) return 0;
        return (m < 0 || i < m) ? 1 : 0;
    }
    __device__ void post(int64_t nc) const {
        LevelDesc *L = c.lv + l, *N = c.lv + l + 1;
        if (L->phase != PH_CONTRACT) return;
        const bool batch = L->gid != nullptr;
        const uint64_t b4 = (uint64_t)nc * 4;
        const uint64_t bytes[6] = {b4, (uint64_t)(nc + 1) * 8, b4, b4, batch ? b4 : 0,
                                   batch ? (uint64_t)(c.b.count + 1) * 4 : 0};
        void *p[6];
        const bool ok = arena_alloc_k<6>(c.ctrl, bytes, p);
        N->n = (int32_t)nc;
        N->vw = (uint32_t *)p[0];
        N->xadj = (int64_t *)p[1];
        N->mate = (int32_t *)p[2];
        N->cmap = (int32_t *)p[3];
        N->gid = batch ? (int32_t *)p[4] : nullptr;
        N->noff = batch ? (int32_t *)p[5] : nullptr;
        N->adj = nullptr;
        N->ew = nullptr;
        N->phase = PH_IDLE;
        N->stop = KAPPA_STOP_NONE;
        if (!ok) {
            L->phase = PH_STOPPED;
            c.ctrl->done = 1;
        }
    }
};
struct RepW {
    Ctx c;
    int l;
    struct Pre {
        int32_t w;
        uint32_t cw;
        int32_t gid;
    };
    struct Bound {
        const int32_t *mate;
        const uint32_t *vw;
        int32_t *cmap, *rep_of, *partner;
        uint32_t *cvw;
        // batched form (null otherwise)
        const int32_t *gid;
        int32_t *cgid, *excl;
        __device__ Pre prefetch(int64_t i, int64_t v) const {
            Pre p{-1, 0u, 0};
            p.w = mate[i];
            if (!v) return p;
            p.cw = vw[i] + (p.w >= 0 ? vw[p.w] : 0u);
            if (gid) p.gid = gid[i];
            return p;
        }
        __device__ void operator()(int64_t i, int64_t pre, int64_t v, const Pre &p) const {
            if (excl) excl[i] = (int32_t)pre;
            if (!v) {
                if (p.w < 0) cmap[i] = -1;   // a stopped graph's node: not carried over
                return;
            }
            const int32_t x = (int32_t)pre;
            cmap[i] = x;
            if (p.w >= 0) cmap[p.w] = x;
            rep_of[x] = (int32_t)i;
            partner[x] = p.w;
            cvw[x] = p.cw;
            if (cgid) cgid[x] = p.gid;
        }
    };
    __device__ Bound bind() const {
        const LevelDesc *L = c.lv + l, *N = c.lv + l + 1;
        const bool batch = L->gid != nullptr;
        return Bound{L->mate,   L->vw,  L->cmap,  c.cs.rep_of,
                     c.cs.partner, N->vw, L->gid, batch ? N->gid : nullptr,
                     batch ? c.b.excl : nullptr};
    }
};

// --- 3. scan of the merged degrees -> coarse row offsets; then the next
//        level's edge arrays and the stall rule ---------------------------------
struct DegF {
    Ctx c;
    int l;
    // post() moves the level to PH_COMPACT before the apply kernel runs
    __device__ int64_t size() const {
        int32_t ph = c.lv[l].phase;
        return (ph == PH_CONTRACT || ph == PH_COMPACT) ? c.lv[l + 1].n + 1 : -1;
    }
    __device__ int64_t operator()(int64_t i) const {
        return i < c.lv[l + 1].n ? c.cs.cdeg[i] : 0;
    }
    __device__ void post(int64_t nnzc) const {
        Control *ctrl = c.ctrl;
        LevelDesc *L = c.lv + l, *N = c.lv + l + 1;
        // everything read here is loaded before the first decision
        const int32_t phase = L->phase;
        const uint32_t flags = ctrl->flags, stall_num = ctrl->stall_num,
                       stall_den = ctrl->stall_den;
        const int64_t n = L->n, nc = N->n;
        if (phase != PH_CONTRACT) return;
        if (flags & CF_HUBS) {   // rows were left unmerged: stop, the host retries
            L->phase = PH_STOPPED;
            ctrl->done = 1;
            return;
        }
        const uint64_t bytes[2] = {(uint64_t)nnzc * 4, (uint64_t)nnzc * 4};
        void *p[2];
        const bool ok = arena_alloc_k<2>(ctrl, bytes, p);
        N->nnz = nnzc;
        N->adj = (int32_t *)p[0];
        N->ew = (uint32_t *)p[1];
        N->maxdeg = 0;   // not tracked below level 0
        if (!ok) {
            L->phase = PH_STOPPED;
            ctrl->done = 1;
            return;
        }
        L->phase = PH_COMPACT;
        ctrl->nlevels = l + 2;
        ctrl->last_n = (int32_t)nc;
        if (stall_num > 0 && (uint64_t)(n - nc) * stall_den < (uint64_t)stall_num * (uint64_t)n) {
            N->stop = KAPPA_STOP_STALL;
            N->phase = PH_STOPPED;
            ctrl->done = 1;
        }
    }
};
struct CoarseOffW {
    Ctx c;
    int l;
    struct Pre {};
    struct Bound {
        int64_t *xadj;
        __device__ Pre prefetch(int64_t, int64_t) const { return Pre{}; }
        __device__ void operator()(int64_t i, int64_t pre, int64_t, const Pre &) const { xadj[i] = pre; }
    };
    __device__ Bound bind() const { return Bound{c.lv[l + 1].xadj}; }
};

// The coarse-id scan of level l in the calling workgroup (the tail).
__device__ __noinline__ void ids_one_block(const Ctx &c, int l) {
    __shared__ int64_t sh[ONE_SCAN_THREADS / WAVE + 1];
    __shared__ int go;
    scan_one_block(RepF{c, l}, RepW{c, l}, c.cs.totals + 0, sh, &go);
    __syncthreads();
}

// The fine entries of coarse row x: row u, then row w (partner), each
// without the contracted edge.  t-th entry -> (coarse key, weight);
// INVALID_KEY for the contracted edge.  The merged row is staged in the same
// two fine rows' slots (it has at most deg(u) + deg(w) - 2 entries): merged
// position p lives at xadj[u] + p while p < deg(u), then at xadj[w] + p - deg(u).
struct RowSrc {
    int32_t u, w;
    int64_t bu, du, bw;
    int64_t tot;
};
__device__ __forceinline__ RowSrc row_src(const DevGraph &g, const Ctx &c, int32_t x) {
    RowSrc r;
    r.u = c.cs.rep_of[x];
    r.w = c.cs.partner[x];
    r.bu = g.xadj[r.u];
    r.du = g.xadj[r.u + 1] - r.bu;
    r.bw = 0;
    int64_t dw = 0;
    if (r.w >= 0) {
        r.bw = g.xadj[r.w];
        dw = g.xadj[r.w + 1] - r.bw;
    }
    r.tot = r.du + dw;
    return r;
}
__device__ __forceinline__ int64_t row_bound(const RowSrc &r) {
    return r.w >= 0 ? r.tot - 2 : r.tot;
}
__device__ __forceinline__ int64_t staged_at(const RowSrc &r, int64_t p) {
    return p < r.du ? r.bu + p : r.bw + (p - r.du);
}
__device__ __forceinline__ void row_entry(const DevGraph &g, const int32_t *cmap, const RowSrc &r,
                                          int64_t t, uint32_t &key, uint32_t &wt) {
    int32_t nb;
    if (t < r.du) {
        nb = g.adj[r.bu + t];
        wt = g.ew[r.bu + t];
        key = nb == r.w ? INVALID_KEY : (uint32_t)cmap[nb];
    } else {
        int64_t j = r.bw + (t - r.du);
        nb = g.adj[j];
        wt = g.ew[j];
        key = nb == r.u ? INVALID_KEY : (uint32_t)cmap[nb];
    }
}

// Merge classes by the bound on the merged row: 0 small (16 lanes), 1 one
// wave, 3 one block, 2 large (hub accumulators); -1 empty.
__device__ __forceinline__ int row_class(int64_t bound, int32_t small_max) {
    if (bound == 0) return -1;
    if (bound <= small_max) return 0;
    if (bound <= ROW_WAVE_MAX) return 1;
    if (bound <= ROW_MID_MAX) return 3;
    return bound <= ROW_BIG_MAX ? 4 : 2;
}
__device__ __forceinline__ int32_t *class_list(const ContractScratch &cs, int32_t n, int cls) {
    const int slot = cls == 3 ? 0 : (cls == 1 ? 1 : (cls == 2 ? 2 : 3));
    return cs.rows + (int64_t)slot * n;
}

// A large row of a level whose next level has nc nodes is merged by key
// buckets (fill_huge_*) rather than by the dense hub accumulators.
__device__ __forceinline__ bool huge_row(int64_t nc, int64_t tot) {
    return nc <= HUGE_NC_MAX && tot <= HUGE_ROW_MAX;
}

// Orders the LDS traffic of one wave (all lanes of the wave call it).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Class-list appends through a per-wave LDS buffer: a wave writes its list
// entries out WBUF_FLUSH or more at a time with one atomic on the list's
// counter, instead of one (returning) atomic per loop iteration; those
// atomics all hit one address and serialise across the chip.  n is
// wave-uniform.
constexpr int WBUF_FLUSH = 32;
constexpr int WBUF_CAP = WBUF_FLUSH + WAVE;
__device__ __forceinline__ void wbuf_flush(int32_t *buf, int &n, int32_t *list, int32_t *counter) {
    if (n == 0) return;
    wave_sync_lds();
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, n);
    base = __shfl(base, 0, WAVE);
    for (int t = lane_id(); t < n; t += WAVE) list[base + t] = buf[t];
    n = 0;
    wave_sync_lds();   // the buffer is refilled next
}
__device__ __forceinline__ void wbuf_add(bool pred, int32_t val, int32_t *buf, int &n,
                                         int32_t *list, int32_t *counter) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    if (pred) buf[n + (int)__popcll(mask & lanemask_lt())] = val;
    n += (int)__popcll(mask);
    if (n >= WBUF_FLUSH) wbuf_flush(buf, n, list, counter);
}

// --- 2a. small rows: 16 lanes per row, rank sort; every coarse row passes
//         here (empty rows get degree 0, bigger rows go to the class lists) --
// The contraction phases below are written for `nb` blocks of NT threads
// (block `bid`): the kernels run them over their grid; the tail kernel runs
// them in one workgroup.
// BIG: rows of the big class get their own list (false: they join the large rows).
// BUF: class-list appends through per-wave LDS buffers (wbuf_add).
template <int NT, bool BIG = true, bool BUF = false>
__device__ __forceinline__ void fill_small_body(const Ctx &c, int l, unsigned bid, unsigned nb) {
    constexpr int ROWS = NT / ROW_SMALL_G;
    __shared__ __align__(16) uint32_t sk[ROWS][SM_CAP];   // renamed entries
    __shared__ __align__(16) uint32_t sr[ROWS][SM_CAP];   // first occurrences only (others INVALID_KEY)
    __shared__ uint32_t sw[ROWS][SM_CAP];   // weights; a first occurrence collects its duplicates'
    __shared__ int32_t wb[BUF ? NT / WAVE : 1][4][BUF ? WBUF_CAP : 1];
    int wn[4] = {0, 0, 0, 0};
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    const int32_t *cmap = L->cmap;
    const int grp = threadIdx.x / ROW_SMALL_G, sub = threadIdx.x % ROW_SMALL_G;
    const int64_t count = c.lv[l + 1].n;
    int32_t *lists1 = class_list(c.cs, g.n, 1), *lists2 = class_list(c.cs, g.n, 2),
            *lists3 = class_list(c.cs, g.n, 3), *lists4 = class_list(c.cs, g.n, 4);
    const int64_t gs = (int64_t)nb * ROWS;
    const int64_t lim = (count + gs - 1) / gs * gs;   // uniform trip count
    bool need_hubs = false;
    for (int64_t i = (int64_t)bid * ROWS + grp; i < lim; i += gs) {
        const bool live = i < count;
        const int32_t x = live ? (int32_t)i : 0;
        RowSrc r;
        r.tot = 0;
        r.w = -1;
        int cls = -1;
        if (live) {
            r = row_src(g, c, x);
            cls = row_class(row_bound(r), c.t.row_small_max);
            // rows of 4095..16382 entries take the key buckets where those
            // apply (groups of a few hundred entries, sorted a wave each),
            // else a 1024-thread block each (fill_big_k)
            if (cls == 4 && (!BIG || !c.big_rows || (c.huge && huge_row(count, r.tot)))) cls = 2;
            if (cls == 2 && !c.cs.hub_acc && !(BIG && c.huge && huge_row(count, r.tot)))
                need_hubs = true;
        }
        if constexpr (BUF) {
            int32_t(*b)[WBUF_CAP] = wb[threadIdx.x / WAVE];
            wbuf_add(sub == 0 && cls == 1, x, b[0], wn[0], lists1, &c.cs.row_cnt[1]);
            wbuf_add(sub == 0 && cls == 2, x, b[1], wn[1], lists2, &c.cs.row_cnt[2]);
            wbuf_add(sub == 0 && cls == 3, x, b[2], wn[2], lists3, &c.cs.row_cnt[3]);
            wbuf_add(sub == 0 && cls == 4, x, b[3], wn[3], lists4, &c.cs.row_cnt[4]);
        } else {
            wave_append(sub == 0 && cls == 1, x, lists1, &c.cs.row_cnt[1]);
            wave_append(sub == 0 && cls == 2, x, lists2, &c.cs.row_cnt[2]);
            wave_append(sub == 0 && cls == 3, x, lists3, &c.cs.row_cnt[3]);
            wave_append(sub == 0 && cls == 4, x, lists4, &c.cs.row_cnt[4]);
        }
        const int tot = cls == 0 ? (int)r.tot : 0;
        {
            constexpr int U = (SM_CAP + ROW_SMALL_G - 1) / ROW_SMALL_G;   // entries per lane
            uint32_t kk[U], ww[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = sub + u * ROW_SMALL_G;
                kk[u] = INVALID_KEY;
                ww[u] = 0;
                if (t < tot) row_entry(g, cmap, r, t, kk[u], ww[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = sub + u * ROW_SMALL_G;
                if (t < tot) {
                    sk[grp][t] = kk[u];
                    sw[grp][t] = ww[u];
                }
            }
        }
        wave_sync_lds();
        // the first occurrence of a key leads; a later one adds its weight
        // to it (only leaders receive, only non-leaders send)
        // (keys read four at a time; slots past the row are masked)
        for (int t = sub; t < tot; t += ROW_SMALL_G) {
            const uint32_t k = sk[grp][t];
            int first = -1;   // the first earlier occurrence of k
            if (k != INVALID_KEY) {
                for (int q0 = 0; q0 < t; q0 += 4) {
                    const uint4 x = *reinterpret_cast<const uint4 *>(&sk[grp][q0]);
                    if (x.x == k) { first = q0; break; }
                    if (q0 + 1 < t && x.y == k) { first = q0 + 1; break; }
                    if (q0 + 2 < t && x.z == k) { first = q0 + 2; break; }
                    if (q0 + 3 < t && x.w == k) { first = q0 + 3; break; }
                }
            }
            const bool lead = k != INVALID_KEY && first < 0;
            sr[grp][t] = lead ? k : INVALID_KEY;
            if (first >= 0) atomicAdd(&sw[grp][first], sw[grp][t]);
        }
        wave_sync_lds();
        int nl = 0;
        for (int t = sub; t < tot; t += ROW_SMALL_G) {
            const uint32_t k = sr[grp][t];
            if (k == INVALID_KEY) continue;
            int rank = 0;   // distinct keys below k
            for (int q0 = 0; q0 < tot; q0 += 4) {
                const uint4 x = *reinterpret_cast<const uint4 *>(&sr[grp][q0]);
                rank += (x.x < k ? 1 : 0) + (q0 + 1 < tot && x.y < k ? 1 : 0) +
                        (q0 + 2 < tot && x.z < k ? 1 : 0) + (q0 + 3 < tot && x.w < k ? 1 : 0);
            }
            int64_t at = staged_at(r, rank);
            c.cs.tmp_adj[at] = (int32_t)k;
            c.cs.tmp_ew[at] = sw[grp][t];
            ++nl;
        }
        for (int o = ROW_SMALL_G / 2; o > 0; o >>= 1) nl += __shfl_xor(nl, o, ROW_SMALL_G);
        if (live && sub == 0 && cls <= 0) c.cs.cdeg[x] = nl;
        wave_sync_lds();
    }
    if constexpr (BUF) {
        int32_t(*b)[WBUF_CAP] = wb[threadIdx.x / WAVE];
        wbuf_flush(b[0], wn[0], lists1, &c.cs.row_cnt[1]);
        wbuf_flush(b[1], wn[1], lists2, &c.cs.row_cnt[2]);
        wbuf_flush(b[2], wn[2], lists3, &c.cs.row_cnt[3]);
        wbuf_flush(b[3], wn[3], lists4, &c.cs.row_cnt[4]);
    }
    if (__ballot(need_hubs) && lane_id() == 0) atomicOr(&c.ctrl->flags, (uint32_t)CF_HUBS);
}
// BUF: graphs with long rows (many rows for the class lists) append through
// the per-wave buffers; others (few list rows) directly.
template <bool BUF>
__global__ void __launch_bounds__(BLOCK) fill_small_k(Ctx c, int l) {
    fill_small_body<BLOCK, true, BUF>(c, l, blockIdx.x, gridDim.x);
}

// Sorted arrays in LDS are left in a padded layout: position p lives in
// slot p + p / 32.  A thread that writes (or reads) E consecutive positions
// with E in {1, 2, 4, 8, 16} then touches distinct banks across its half-wave,
// where the plain layout would put every lane of a half-wave on a handful of
// banks (stride E * 8 bytes).
__host__ __device__ constexpr int lds_padded(int p) { return p + p / 32; }
__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 5); }

// One compare-exchange stage (block size k, distance j) of a bitonic sort of
// s[lo, lo + 2 * npairs): pair p pairs element t (bit j clear) with t | j and
// orders them ascending when bit k of t is clear.  The caller's threads take
// pairs first, first + stride, ...; each thread loads up to BS_BATCH pairs
// before it stores any (the pairs of a stage are disjoint).
constexpr int BS_BATCH = 8;
template <class T>
__device__ __forceinline__ void bitonic_stage(T *s, int lo, int npairs, int k, int j, int first,
                                              int stride) {
    const int lj = __ffs(j) - 1;
    for (int p0 = first; p0 < npairs; p0 += stride * BS_BATCH) {
        T a[BS_BATCH], b[BS_BATCH];
        int t[BS_BATCH];
#pragma unroll
        for (int q = 0; q < BS_BATCH; ++q) {
            const int p = p0 + q * stride;
            t[q] = lo + (((p >> lj) << (lj + 1)) | (p & (j - 1)));
            if (p < npairs) {
                a[q] = s[t[q]];
                b[q] = s[t[q] | j];
            }
        }
#pragma unroll
        for (int q = 0; q < BS_BATCH; ++q) {
            const int p = p0 + q * stride;
            if (p >= npairs) continue;
            const bool up = (t[q] & k) == 0;
            if ((a[q] > b[q]) == up) {
                s[t[q]] = b[q];
                s[t[q] | j] = a[q];
            }
        }
    }
}

// Bitonic sort of P = E * NT values held in registers, E per thread: thread
// `tid` holds positions tid * E + e.  Stages whose partner distance j is
// below E pair two registers of one thread; below E * WAVE, the partner is
// lane ^ (j / E) of the same wave (shuffles); wider stages exchange through
// LDS s (P entries, stored slot e * NT + tid so that a wave's accesses hit
// consecutive slots) between block barriers.  Every loop has a constant trip
// count and unrolls, so j, k and the register indices are constants.
__device__ __forceinline__ uint64_t shfl_xor_v(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, WAVE);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, WAVE);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl_xor_v(uint32_t v, int m) {
    return (uint32_t)__shfl_xor((int)v, m, WAVE);
}
// T: uint64_t, or uint32_t (one shuffle, one compare and one select per
// exchange).  An exchange compares once and flips the result by the
// direction: written as a minimum and a maximum, a 64-bit pair compiles to
// two compares and six selects.
template <int E, int NT, class T>
__device__ __forceinline__ void reg_bitonic(T (&v)[E], int tid, T *s) {
    constexpr int P = E * NT;
    constexpr int LOGP = __builtin_ctz(P);
    static_assert((E & (E - 1)) == 0 && (NT & (NT - 1)) == 0 && NT >= WAVE, "sort shape");
#pragma unroll
    for (int lk = 1; lk <= LOGP; ++lk) {
        const int k = 1 << lk;
#pragma unroll
        for (int lj = lk - 1; lj >= 0; --lj) {
            const int j = 1 << lj;
            if (j < E) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if ((e & j) != 0) continue;
                    const bool up = (((tid * E + e) & k) == 0);
                    const T a = v[e], b = v[e | j];
                    if (sizeof(T) == 4 && k < E) {   // direction fixed at compile time
                        const T lo = a < b ? a : b, hi = a < b ? b : a;
                        v[e] = up ? lo : hi;
                        v[e | j] = up ? hi : lo;
                    } else {   // one compare; swapped where out of order for the direction
                        const bool sw = (b < a) == up;
                        v[e] = sw ? b : a;
                        v[e | j] = sw ? a : b;
                    }
                }
            } else if (j < E * WAVE) {
                const int m = j / E;
                const bool lower = (tid & m) == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const bool up = (((tid * E + e) & k) == 0);
                    const T o = shfl_xor_v(v[e], m);
                    const bool take_min = lower == up;
                    v[e] = ((o < v[e]) == take_min) ? o : v[e];
                }
            } else {
                const int m = j / E;
                const bool lower = (tid & m) == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) s[e * NT + tid] = v[e];
                __syncthreads();
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const bool up = (((tid * E + e) & k) == 0);
                    const T o = s[e * NT + (tid ^ m)];
                    const bool take_min = lower == up;
                    v[e] = ((o < v[e]) == take_min) ? o : v[e];
                }
                __syncthreads();
            }
        }
    }
}

// Sorts s[0, P) (P = E * NT, every thread of the block calling) through
// registers: slot tid + e * NT is read as position tid * E + e (any initial
// placement sorts), and the sorted positions are written back in the padded
// layout (s holds lds_padded(P) entries).
template <int E, int NT, class T = uint64_t>
__device__ __forceinline__ void block_sort_regs(T *s, int tid) {
    T v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = s[tid + e * NT];
    if (E * NT > E * WAVE) __syncthreads();   // the LDS stages overwrite s
    reg_bitonic<E, NT, T>(v, tid, s);
    if (E * NT > E * WAVE) __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) s[lds_pad(tid * E + e)] = v[e];
}

// The register sort for P = E * NT with E in {4, 8, 16}; false: not such a P
// (the caller sorts in LDS instead).
template <int NT, class T = uint64_t>
__device__ __forceinline__ bool block_sort_regs_p(T *s, int P) {
    if (P == 4 * NT) block_sort_regs<4, NT, T>(s, threadIdx.x);
    else if (P == 8 * NT) block_sort_regs<8, NT, T>(s, threadIdx.x);
    else if (P == 16 * NT) block_sort_regs<16, NT, T>(s, threadIdx.x);
    else return false;
    return true;
}

// Sorts s[0, P) ascending (P a power of two, 2 <= P) with the block's NT
// threads into the padded layout (s holds lds_padded(P) entries): in
// registers where P = 4, 8 or 16 per thread, else in LDS, where the stages
// whose compare distance stays inside one wave's contiguous slice of the
// array (P / waves elements) need only that wave's LDS order and only the
// few wider stages take a block barrier, followed by a move into the padded
// layout.  Ends with a block barrier.
template <int NT, class T = uint64_t>
__device__ __forceinline__ void block_sort(T *s, int P) {
    constexpr int NW = NT / WAVE;
    if (block_sort_regs_p<NT, T>(s, P)) {
        __syncthreads();
        return;
    }
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    const int chunk = P / NW;             // a wave's slice
    const bool wave_stages = chunk >= WAVE;
    bool synced = true;                   // every wave's LDS writes seen by the block
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (!wave_stages || j >= chunk) {
                if (!synced) __syncthreads();
                bitonic_stage(s, 0, P / 2, k, j, threadIdx.x, NT);
                __syncthreads();
                synced = true;
            } else {
                bitonic_stage(s, wv * chunk, chunk / 2, k, j, lane, WAVE);
                wave_sync_lds();
                synced = false;
            }
        }
    }
    if (!synced) __syncthreads();
    // into the padded layout, NT positions at a time from the top: a chunk's
    // slots lie at or above its own positions, so no unread position below
    // it is overwritten
    for (int hi = P; hi > 0; hi -= NT) {
        const int p = hi - NT + (int)threadIdx.x;
        const T v = p >= 0 ? s[p] : (T)0;
        __syncthreads();
        if (p >= 0) s[lds_pad(p)] = v;
        __syncthreads();
    }
}

// --- 2b. sort values of a merged row.  Wide: (key << 32 | weight) in 64 bits.
//          Narrow, where every coarse id shifted by lp = log2(P) bits fits in
//          32 (nc << lp < 2^32): (key << lp | position) in 32 bits, the weight
//          kept by position in a second LDS array, so that an exchange of the
//          sort is one shuffle, one 32-bit compare and one select.  Padding and the
//          contracted edge are all ones in either form (a narrow value never
//          is: its key is below nc) and read as INVALID_KEY.
struct WideRep {
    using T = uint64_t;
    __device__ T make(uint32_t key, uint32_t w, int) const {
        return key == INVALID_KEY ? ~0ull : ((uint64_t)key << 32) | w;
    }
    __device__ uint32_t key(T v) const { return (uint32_t)(v >> 32); }
    __device__ uint32_t weight(T v) const { return (uint32_t)v; }
};
// base: keys are stored less base (every key of the sort at least base and
// below base + span, with span << lp < 2^32).
struct NarrowRep {
    using T = uint32_t;
    uint32_t *wt;   // weights by position
    int lp;
    uint32_t base;
    __device__ T make(uint32_t key, uint32_t w, int pos) const {
        wt[pos] = w;
        return key == INVALID_KEY ? ~0u : ((key - base) << lp) | (uint32_t)pos;
    }
    __device__ uint32_t key(T v) const { return v == ~0u ? INVALID_KEY : (v >> lp) + base; }
    __device__ uint32_t weight(T v) const { return wt[v & ((1u << lp) - 1)]; }
};
// span << lp < 2^32 (span: the number of distinct keys possible)
__device__ __forceinline__ bool narrow_fits(int64_t span, int lp) {
    return ((uint64_t)span << lp) < ((uint64_t)1 << 32);
}

// --- 2b'. mid and big rows: one block per row, the row staged in LDS and
//          sorted (block_sort), then a leader scan.  s: lds_padded(PMAX)
//          64-bit entries of LDS. -------------------------------------------
template <int NT, class Rep>
__device__ __forceinline__ int64_t block_row_merge(const Ctx &c, const DevGraph &g,
                                                   const int32_t *cmap, const RowSrc &r, int P,
                                                   typename Rep::T *s, const Rep &rep, int64_t *sh) {
    using T = typename Rep::T;
    const int tot = (int)r.tot;
    for (int t0 = threadIdx.x; t0 < P; t0 += NT * 4) {
        T val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * NT;
            val[u] = (T)~(T)0;
            if (t < tot) {
                uint32_t k, w;
                row_entry(g, cmap, r, t, k, w);
                val[u] = rep.make(k, w, t);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t0 + u * NT < P) s[t0 + u * NT] = val[u];
    }
    __syncthreads();
    if constexpr (sizeof(T) == 8) {
        block_sort<NT>(s, P);
    } else {   // the callers take the narrow form only for P = 4, 8 or 16 per thread
        if (P == 4 * NT) block_sort_regs<4, NT, T>(s, threadIdx.x);
        else if (P == 8 * NT) block_sort_regs<8, NT, T>(s, threadIdx.x);
        else block_sort_regs<16, NT, T>(s, threadIdx.x);
        __syncthreads();
    }
    // leaders: first entry of each run of equal keys (padded layout)
    const int ipt = (P + NT - 1) / NT;
    const int t0 = threadIdx.x * ipt;
    int64_t mine = 0;
    for (int q = 0; q < ipt; ++q) {
        const int t = t0 + q;
        if (t >= P) break;
        const uint32_t k = rep.key(s[lds_pad(t)]);
        if (k != INVALID_KEY && (t == 0 || rep.key(s[lds_pad(t - 1)]) != k)) ++mine;
    }
    int64_t total;
    int64_t rank = block_excl_scan(mine, sh, &total);
    for (int q = 0; q < ipt; ++q) {
        const int t = t0 + q;
        if (t >= P) break;
        const uint32_t k = rep.key(s[lds_pad(t)]);
        if (k == INVALID_KEY || (t > 0 && rep.key(s[lds_pad(t - 1)]) == k)) continue;
        uint32_t sum = 0;
        for (int e = t; e < P; ++e) {
            const T v = s[lds_pad(e)];
            if (rep.key(v) != k) break;
            sum += rep.weight(v);
        }
        const int64_t at = staged_at(r, rank);
        c.cs.tmp_adj[at] = (int32_t)k;
        c.cs.tmp_ew[at] = sum;
        ++rank;
    }
    return total;
}
template <int NT, int PMAX>
__device__ __forceinline__ void fill_block_body(const Ctx &c, int l, unsigned bid, unsigned nb,
                                                int cls, uint64_t *s) {
    __shared__ int64_t sh[NT / WAVE + 1];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    const int32_t *cmap = L->cmap;
    const int64_t nc = c.lv[l + 1].n;
    const int64_t count = c.cs.row_cnt[cls];
    const int32_t *list = class_list(c.cs, g.n, cls);
    for (int64_t i = bid; i < count; i += nb) {
        const int32_t x = list[i];
        const RowSrc r = row_src(g, c, x);
        int P = 2;
        while (P < r.tot) P <<= 1;
        if (P > PMAX) {   // valid class lists never
            if (threadIdx.x == 0) atomicOr(&c.ctrl->flags, (uint32_t)CF_STATE);
            continue;
        }
        const int lp = __builtin_ctz(P);
        int64_t total;
        if ((P == 4 * NT || P == 8 * NT || P == 16 * NT) && narrow_fits(nc, lp)) {
            // values in the first lds_padded(P) words, weights after lds_padded(PMAX)
            uint32_t *s32 = (uint32_t *)s;
            total = block_row_merge<NT>(c, g, cmap, r, P, s32,
                                        NarrowRep{s32 + lds_padded(PMAX), lp, 0}, sh);
        } else {
            total = block_row_merge<NT>(c, g, cmap, r, P, s, WideRep{}, sh);
        }
        if (threadIdx.x == 0) c.cs.cdeg[x] = (int32_t)total;
        __syncthreads();
    }
}
template <int NT>
__device__ __forceinline__ void fill_mid_body(const Ctx &c, int l, unsigned bid, unsigned nb,
                                              int cls = 3) {
    __shared__ uint64_t s[lds_padded(MID_P)];
    fill_block_body<NT, MID_P>(c, l, bid, nb, cls, s);
}

// Rows of 4095..16382 entries: one block of BIG_THREADS per row, the whole
// row sorted in 128 KiB of LDS (one block per CU).
constexpr int BIG_P = ROW_BIG_MAX + 2;
constexpr int BIG_THREADS = 1024;
static_assert((BIG_P & (BIG_P - 1)) == 0, "big-row sort size");
__global__ void __launch_bounds__(BIG_THREADS) fill_big_k(Ctx c, int l) {
    __shared__ uint64_t s[lds_padded(BIG_P)];
    fill_block_body<BIG_THREADS, BIG_P>(c, l, blockIdx.x, gridDim.x, 4, s);
}
// --- 2a'. rows of 65..512 entries: one wave per row; the renamed entries are
//          compacted into the wave's LDS slice, bitonic-sorted in registers and
//          lane shuffles, written back in order, then a leader scan ------------------
constexpr int WR_P = ROW_WAVE_MAX;   // sort size of a wave row (power of two)
constexpr int WR_LP = 9;             // log2(WR_P): the narrow form's position bits
static_assert((1 << WR_LP) == WR_P, "wave row position bits");
template <class Rep>
__device__ __forceinline__ int32_t wave_row_merge(const Ctx &c, const DevGraph &g,
                                                  const int32_t *cmap, const RowSrc &r,
                                                  typename Rep::T *s, const Rep &rep) {
    using T = typename Rep::T;
    const int lane = lane_id();
    // the renamed entries without the contracted edge (at most the row's
    // bound, <= WR_P of them), packed to the front of the slice
    const int tot = (int)r.tot;
    constexpr int U = (WR_P + 2 + WAVE - 1) / WAVE;   // entries per lane (bound + 2 at most)
    uint32_t kk[U], ww[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = u * WAVE + lane;
        kk[u] = INVALID_KEY;
        ww[u] = 0;
        if (t < tot) row_entry(g, cmap, r, t, kk[u], ww[u]);
    }
    int q = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool keep = kk[u] != INVALID_KEY;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int pos = q + (int)__popcll(m & lanemask_lt());
            s[pos] = rep.make(kk[u], ww[u], pos);
        }
        q += (int)__popcll(m);
    }
    int P = WAVE;
    while (P < q) P <<= 1;
    for (int t = q + lane; t < P; t += WAVE) s[t] = (T)~(T)0;   // padding sorts last
    wave_sync_lds();
    // in registers and lane shuffles (P / WAVE values per lane)
    if (P == WAVE) block_sort_regs<1, WAVE, T>(s, lane);
    else if (P == 2 * WAVE) block_sort_regs<2, WAVE, T>(s, lane);
    else if (P == 4 * WAVE) block_sort_regs<4, WAVE, T>(s, lane);
    else block_sort_regs<8, WAVE, T>(s, lane);
    wave_sync_lds();
    // leaders (first entry of each run of equal keys) in order; runs summed
    // (the sorted entries are in the padded layout)
    int32_t rank = 0;
    for (int t0 = 0; t0 < P; t0 += WAVE) {
        const int t = t0 + lane;
        const uint32_t k = rep.key(s[lds_pad(t)]);
        const bool lead = k != INVALID_KEY && (t == 0 || rep.key(s[lds_pad(t - 1)]) != k);
        const uint64_t m = __ballot(lead);
        if (lead) {
            uint32_t sum = 0;
            for (int e = t; e < P; ++e) {
                const T v = s[lds_pad(e)];
                if (rep.key(v) != k) break;
                sum += rep.weight(v);
            }
            const int64_t at = staged_at(r, rank + (int32_t)__popcll(m & lanemask_lt()));
            c.cs.tmp_adj[at] = (int32_t)k;
            c.cs.tmp_ew[at] = sum;
        }
        rank += (int32_t)__popcll(m);
    }
    return rank;
}
template <int NT>
__device__ __forceinline__ void fill_wave_body(const Ctx &c, int l, unsigned bid, unsigned nb,
                                               uint64_t *lds) {
    static_assert((WR_P & (WR_P - 1)) == 0 && WR_P % WAVE == 0, "wave sort size");
    static_assert(lds_padded(WR_P) + WR_P <= 2 * lds_padded(WR_P), "narrow weights fit the slice");
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    const int32_t *cmap = L->cmap;
    const bool narrow = narrow_fits(c.lv[l + 1].n, WR_LP);
    const int64_t count = c.cs.row_cnt[1];
    const int32_t *list = class_list(c.cs, g.n, 1);
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    uint64_t *s = lds + (int64_t)wv * lds_padded(WR_P);
    uint32_t *s32 = (uint32_t *)s;
    const int64_t gw = (int64_t)bid * (NT / WAVE) + wv, gs = (int64_t)nb * (NT / WAVE);
    for (int64_t i = gw; i < count; i += gs) {   // wave-uniform
        const int32_t x = list[i];
        const RowSrc r = row_src(g, c, x);
        const int32_t rank =
            narrow ? wave_row_merge(c, g, cmap, r, s32, NarrowRep{s32 + lds_padded(WR_P), WR_LP, 0})
                   : wave_row_merge(c, g, cmap, r, s, WideRep{});
        if (lane == 0) c.cs.cdeg[x] = rank;
        wave_sync_lds();   // the slice is rewritten by the next row
    }
}

// Both mid classes in one class-partitioned grid: blocks [0, wave_blocks)
// merge the rows of 65..512 entries one wave each, the others the rows of
// 513..4094 entries one block each (one LDS array serves either).
__global__ void __launch_bounds__(BLOCK) fill_mid_k(Ctx c, int l, unsigned wave_blocks) {
    static_assert((BLOCK / WAVE) * lds_padded(WR_P) <= lds_padded(MID_P),
                  "the wave rows' slices fit the block rows' array");
    __shared__ uint64_t s[lds_padded(MID_P)];
    if (blockIdx.x < wave_blocks)
        fill_wave_body<BLOCK>(c, l, blockIdx.x, wave_blocks, s);
    else
        fill_block_body<BLOCK, MID_P>(c, l, blockIdx.x - wave_blocks, gridDim.x - wave_blocks, 3, s);
}

// --- 2c. large rows: dense accumulator per slot --------------------------------------
// Slot `bid` of the hub accumulators (bid < hub_slots): a dense sum per
// coarse id, a bitmap of the ids present (one bit per id) and a summary
// bitmap (one bit per nonzero bitmap word).  The read-back walks the summary
// in chunks of summary words, gathers the chunk's nonzero bitmap words
// into LDS, and hands out the chunk's ids by rank (a thread finds the word
// holding its rank by a binary search over the words' prefix counts), so the
// work follows the ids present rather than the id range and is spread evenly
// over the block.  Every array is left zero for the next row.
constexpr int LG_IDS = 4;                   // ids per thread in flight (read-back)
constexpr int LG_ACC = 8;                   // entries per thread in flight (accumulation)
// LG_SUM summary words per chunk (LG_WORDS = 32 * LG_SUM nonzero bitmap words at most).
template <int NT, int LG_SUM>
__device__ __forceinline__ void fill_large_body(const Ctx &c, int l, unsigned bid, unsigned nb,
                                                bool skip_bucketed = false) {
    constexpr int LG_WORDS = LG_SUM * 32;
    static_assert(NT >= LG_SUM && LG_WORDS % NT == 0, "chunk layout");
    constexpr int WPT = LG_WORDS / NT;       // bitmap words per thread of a chunk
    __shared__ int32_t s_word[LG_WORDS];     // the chunk's nonzero bitmap words: index
    __shared__ uint32_t s_bits[LG_WORDS];    //   and value
    __shared__ int32_t s_pre[LG_WORDS];      //   and the ids in the words before it
    __shared__ int64_t sh[NT / WAVE + 1];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    if (!c.cs.hub_acc) return;
    const int32_t *cmap = L->cmap;
    uint32_t *acc = c.cs.hub_acc + (int64_t)bid * g.n;
    uint32_t *bits = c.cs.hub_bits + (int64_t)bid * c.cs.hub_words;
    uint32_t *sbits = bits + c.cs.hub_w1;
    const int64_t nc = c.lv[l + 1].n;
    const int64_t nwords = (nc + 31) / 32, nsum = (nwords + 31) / 32;
    const int64_t count = c.cs.row_cnt[2];
    for (int64_t i = bid; i < count; i += nb) {
        const int32_t x = c.cs.rows[2 * (int64_t)g.n + i];
        const RowSrc r = row_src(g, c, x);
        if (skip_bucketed && c.huge && huge_row(nc, r.tot)) continue;   // the key buckets merge it
        // LG_ACC entries per thread in flight: their loads, renames and
        // atomics are issued before any result is waited for
        for (int64_t t0 = threadIdx.x; t0 < r.tot; t0 += (int64_t)NT * LG_ACC) {
            uint32_t k[LG_ACC], w[LG_ACC], old[LG_ACC];
#pragma unroll
            for (int u = 0; u < LG_ACC; ++u) {
                const int64_t t = t0 + (int64_t)u * NT;
                k[u] = INVALID_KEY;
                w[u] = 0;
                if (t < r.tot) row_entry(g, cmap, r, t, k[u], w[u]);
            }
#pragma unroll
            for (int u = 0; u < LG_ACC; ++u) {
                old[u] = 1;
                if (k[u] == INVALID_KEY) continue;
                atomicAdd(&acc[k[u]], w[u]);
                old[u] = atomicOr(&bits[k[u] >> 5], 1u << (k[u] & 31));
            }
#pragma unroll
            for (int u = 0; u < LG_ACC; ++u)
                if (old[u] == 0) atomicOr(&sbits[k[u] >> 10], 1u << ((k[u] >> 5) & 31));
        }
        __threadfence();
        __syncthreads();
        int64_t pos = 0;   // ids written so far (block-uniform)
        for (int64_t s0 = 0; s0 < nsum; s0 += LG_SUM) {
            // 1. the chunk's nonzero bitmap words in ascending order
            uint32_t sw = 0;
            if (threadIdx.x < LG_SUM && s0 + threadIdx.x < nsum) {
                uint32_t *p = &sbits[s0 + threadIdx.x];
                sw = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (sw) *p = 0u;
            }
            int64_t nw_tot;
            const int64_t at = block_excl_scan((int64_t)__popc(sw), sh, &nw_tot);
            if (nw_tot == 0) continue;   // block-uniform; nothing was written to LDS
            {
                int32_t q = (int32_t)at;
                uint32_t m = sw;
                while (m) {
                    const int b = __ffs(m) - 1;
                    m &= m - 1;
                    s_word[q++] = (int32_t)((s0 + threadIdx.x) * 32 + b);
                }
            }
            __syncthreads();
            // 2. the words themselves (WPT consecutive list entries per thread)
            const int nw = (int)nw_tot;
            uint32_t wv[WPT];
#pragma unroll
            for (int j = 0; j < WPT; ++j) {
                const int q = threadIdx.x * WPT + j;
                wv[j] = q < nw ? __hip_atomic_load(&bits[s_word[q]], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                               : 0u;
            }
            int64_t mine = 0;
#pragma unroll
            for (int j = 0; j < WPT; ++j) mine += __popc(wv[j]);
            int64_t ids_tot;
            int64_t run = block_excl_scan(mine, sh, &ids_tot);
#pragma unroll
            for (int j = 0; j < WPT; ++j) {
                const int q = threadIdx.x * WPT + j;
                if (q < nw) {
                    s_pre[q] = (int32_t)run;
                    s_bits[q] = wv[j];
                    bits[s_word[q]] = 0u;
                }
                run += __popc(wv[j]);
            }
            __syncthreads();
            // 3. ids by rank: the word holding rank k, then the bit within it
            const int32_t kt = (int32_t)ids_tot;
            for (int32_t k0 = 0; k0 < kt; k0 += NT * LG_IDS) {
                uint32_t key[LG_IDS], val[LG_IDS];
                bool ok[LG_IDS];
#pragma unroll
                for (int u = 0; u < LG_IDS; ++u) {
                    const int32_t k = k0 + u * NT + (int32_t)threadIdx.x;
                    ok[u] = k < kt;
                    key[u] = 0;
                    if (!ok[u]) continue;
                    int lo = 0, hi = nw - 1;   // the last word with s_pre <= k
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= k) lo = mid; else hi = mid - 1;
                    }
                    uint32_t wb = s_bits[lo];
                    for (int z = k - s_pre[lo]; z > 0; --z) wb &= wb - 1;
                    key[u] = (uint32_t)s_word[lo] * 32u + (uint32_t)(__ffs(wb) - 1);
                }
#pragma unroll
                for (int u = 0; u < LG_IDS; ++u)
                    val[u] = ok[u] ? __hip_atomic_load(&acc[key[u]], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)
                                   : 0u;
#pragma unroll
                for (int u = 0; u < LG_IDS; ++u) {
                    if (!ok[u]) continue;
                    const int64_t st = staged_at(r, pos + k0 + u * NT + threadIdx.x);
                    c.cs.tmp_adj[st] = (int32_t)key[u];
                    c.cs.tmp_ew[st] = val[u];
                    acc[key[u]] = 0u;
                }
            }
            pos += kt;
            __syncthreads();   // the chunk's LDS lists are read before the next chunk writes them
        }
        if (threadIdx.x == 0) c.cs.cdeg[x] = (int32_t)pos;
        __threadfence();
        __syncthreads();
    }
}
constexpr int LARGE_THREADS = 1024;   // one workgroup per hub slot (one per CU)
__global__ void __launch_bounds__(LARGE_THREADS) fill_large_k(Ctx c, int l) {
    fill_large_body<LARGE_THREADS, 256>(c, l, blockIdx.x, gridDim.x, true);
}

// --- 2d. large rows by key buckets, in four launches ------------------------------
// prep (a block per row): a histogram of the row's keys over HG_BINS buckets
//   of 2^shb consecutive keys (a key occurs at most four times in a row: from
//   u and w, each through a node and its partner, so a bucket holds at most
//   2^(shb+2) <= 8192 entries), its exclusive scan, the groups (the buckets
//   whose first entry falls in one window of `win` positions; win >= 256
//   keeps at most HG_WINS groups, and a group has fewer than win + 8192 <=
//   16384 entries), the entries scattered into bucket order in the row's
//   staging slots, and one descriptor per group (in the small list when it
//   has at most WR_P entries);
// merge_small (a wave per group) and merge_big (a block per group): the group
//   sorted and merged into hg_adj / hg_ew from its own first position on;
// pack (a block per row): the groups' merged counts scanned, and every merged
//   entry copied to its place in the row's staging slots.
// Equal keys share a bucket, so runs never cross groups; the merge output is
// in a separate array, so the copy needs no ordering between its threads.
constexpr int HUGE_THREADS = 1024;
constexpr int HG_U = 8;      // entries per thread in flight
constexpr int HG_KEEP = 16;  // entries per thread kept between the two passes
__global__ void __launch_bounds__(HUGE_THREADS) fill_huge_prep_k(Ctx c, int l) {
    constexpr int NT = HUGE_THREADS;
    static_assert(HG_BINS % NT == 0, "buckets per thread");
    __shared__ int32_t hist[HG_BINS];
    __shared__ int32_t fs[HG_WINS + 1];
    __shared__ int64_t sh[NT / WAVE + 1];
    __shared__ int32_t s_base, s_cnt[2];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    const int64_t nc = c.lv[l + 1].n;
    if (nc > HUGE_NC_MAX) return;   // the dense accumulators take every large row
    const int32_t *cmap = L->cmap;
    int shb = 0;
    while ((((nc > 0 ? nc : 1) - 1) >> shb) >= HG_BINS) ++shb;   // keys < nc -> buckets < HG_BINS
    const int64_t count = c.cs.row_cnt[2];
    const int32_t *list = class_list(c.cs, g.n, 2);
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int32_t x = list[i];
        const RowSrc r = row_src(g, c, x);
        if (!huge_row(nc, r.tot)) continue;   // block-uniform
        for (int b = threadIdx.x; b < HG_BINS; b += NT) hist[b] = 0;
        __syncthreads();
        // histogram; a row of at most NT * HG_KEEP entries keeps its renamed
        // entries in registers for the scatter below (one gather, not two)
        const bool keep = r.tot <= (int64_t)NT * HG_KEEP;   // block-uniform
        uint32_t kk[HG_KEEP], kw[HG_KEEP];
        if (keep) {
#pragma unroll
            for (int u = 0; u < HG_KEEP; ++u) {
                const int64_t t = threadIdx.x + (int64_t)u * NT;
                kk[u] = INVALID_KEY;
                kw[u] = 0;
                if (t < r.tot) row_entry(g, cmap, r, t, kk[u], kw[u]);
            }
#pragma unroll
            for (int u = 0; u < HG_KEEP; ++u)
                if (kk[u] != INVALID_KEY) atomicAdd(&hist[kk[u] >> shb], 1);
        } else {
            for (int64_t t0 = threadIdx.x; t0 < r.tot; t0 += (int64_t)NT * HG_U) {
                uint32_t k[HG_U], w[HG_U];
#pragma unroll
                for (int u = 0; u < HG_U; ++u) {
                    const int64_t t = t0 + (int64_t)u * NT;
                    k[u] = INVALID_KEY;
                    if (t < r.tot) row_entry(g, cmap, r, t, k[u], w[u]);
                }
#pragma unroll
                for (int u = 0; u < HG_U; ++u)
                    if (k[u] != INVALID_KEY) atomicAdd(&hist[k[u] >> shb], 1);
            }
        }
        __syncthreads();
        // exclusive scan (HG_BINS / NT consecutive buckets per thread)
        constexpr int BPT = HG_BINS / NT;
        int32_t cnt[BPT];
        int64_t mine = 0;
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            cnt[q] = hist[threadIdx.x * BPT + q];
            mine += cnt[q];
        }
        int64_t valid;
        int64_t run = block_excl_scan(mine, sh, &valid);
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            hist[threadIdx.x * BPT + q] = (int32_t)run;
            run += cnt[q];
        }
        __syncthreads();
        // the groups' first positions
        int32_t win = HG_WIN_MIN;
        while ((int64_t)win * HG_WINS < valid) win <<= 1;
        const int32_t nwin = (int32_t)((valid + win - 1) / win);
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int b = threadIdx.x * BPT + q;
            const int32_t st = hist[b];
            const int32_t wp = b > 0 ? hist[b - 1] / win : -1;
            const int32_t wb = min(st / win, nwin - 1);
            for (int32_t j = wp + 1; j <= wb; ++j) fs[j] = st;
        }
        if (threadIdx.x == 0) {
            fs[nwin] = (int32_t)valid;
            s_base = atomicAdd(&c.cs.hg_cnt[2], nwin);   // the row's group slots
            if (i >= c.cs.hg_rows || (int64_t)s_base + nwin > c.cs.hg_cap) {   // valid state never
                atomicOr(&c.ctrl->flags, (uint32_t)CF_STATE);
                if (i < c.cs.hg_rows) c.cs.hg_row[i] = make_int2(-1, 0);
                s_base = -1;
            } else {
                c.cs.hg_row[i] = make_int2(s_base, nwin);
            }
        }
        __syncthreads();
        if (s_base < 0) continue;   // block-uniform
        // scatter into bucket order (hist as cursors)
        if (keep) {
#pragma unroll
            for (int u = 0; u < HG_KEEP; ++u) {
                if (kk[u] == INVALID_KEY) continue;
                const int32_t pos = atomicAdd(&hist[kk[u] >> shb], 1);
                const int64_t at = staged_at(r, pos);
                c.cs.tmp_adj[at] = (int32_t)kk[u];
                c.cs.tmp_ew[at] = kw[u];
            }
        }
        for (int64_t t0 = keep ? r.tot : threadIdx.x; t0 < r.tot; t0 += (int64_t)NT * HG_U) {
            uint32_t k[HG_U], w[HG_U];
#pragma unroll
            for (int u = 0; u < HG_U; ++u) {
                const int64_t t = t0 + (int64_t)u * NT;
                k[u] = INVALID_KEY;
                if (t < r.tot) row_entry(g, cmap, r, t, k[u], w[u]);
            }
#pragma unroll
            for (int u = 0; u < HG_U; ++u) {
                if (k[u] == INVALID_KEY) continue;
                const int32_t pos = atomicAdd(&hist[k[u] >> shb], 1);
                const int64_t at = staged_at(r, pos);
                c.cs.tmp_adj[at] = (int32_t)k[u];
                c.cs.tmp_ew[at] = w[u];
            }
        }
        // group descriptors: small ones (<= WR_P entries) and the others
        if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
        __syncthreads();
        constexpr int WPT = (HG_WINS + NT - 1) / NT;
        int kind[WPT], at_k[WPT];
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int j = threadIdx.x * WPT + q;
            kind[q] = -1;
            if (j < nwin) {
                const int32_t m = fs[j + 1] - fs[j];
                kind[q] = m <= 0 ? -1 : (m <= WR_P ? 0 : 1);
                if (kind[q] >= 0) at_k[q] = atomicAdd(&s_cnt[kind[q]], 1);
            }
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            const int32_t n_k = s_cnt[threadIdx.x];
            const int32_t b_k = atomicAdd(&c.cs.hg_cnt[threadIdx.x], n_k);
            if ((int64_t)b_k + n_k > c.cs.hg_cap) atomicOr(&c.ctrl->flags, (uint32_t)CF_STATE);
            s_cnt[threadIdx.x] = b_k;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int j = threadIdx.x * WPT + q;
            if (j >= nwin) continue;
            const int32_t a = fs[j], m = fs[j + 1] - a;
            c.cs.hg_slot[s_base + j] = make_int2(a, 0);
            if (kind[q] < 0) continue;
            int4 *lst = kind[q] == 0 ? c.cs.hg_small : c.cs.hg_big;
            const int64_t at = (int64_t)s_cnt[kind[q]] + at_k[q];
            if (at < c.cs.hg_cap) lst[at] = make_int4((int32_t)i, a, m, s_base + j);
        }
        __syncthreads();   // hist, fs and the counters are reset for the next row
    }
}

// The merged entries of a sorted group s[0, P) (padded layout; NT threads, a
// block or one wave) into hg_adj / hg_ew at positions a, a + 1, ... of row r;
// returns how many (every thread).  sh: NT / WAVE + 1 int64 of LDS (a block
// only).
template <int NT, class Rep>
__device__ __forceinline__ int32_t hg_emit(const Ctx &c, const typename Rep::T *s, int P,
                                           const RowSrc &r, int32_t a, int64_t *sh,
                                           const Rep &rep) {
    using T = typename Rep::T;
    const int tid = NT == WAVE ? lane_id() : (int)threadIdx.x;
    const int ipt = (P + NT - 1) / NT;
    const int t0 = tid * ipt;
    int64_t mine = 0;
    for (int q = 0; q < ipt; ++q) {
        const int t = t0 + q;
        if (t >= P) break;
        const uint32_t k = rep.key(s[lds_pad(t)]);
        if (k != INVALID_KEY && (t == 0 || rep.key(s[lds_pad(t - 1)]) != k)) ++mine;
    }
    int64_t total, rank;
    if (NT == WAVE) {
        const int64_t inc = wave_incl_scan(mine);
        total = __shfl(inc, WAVE - 1, WAVE);
        rank = inc - mine;
    } else {
        rank = block_excl_scan(mine, sh, &total);
    }
    for (int q = 0; q < ipt; ++q) {
        const int t = t0 + q;
        if (t >= P) break;
        const uint32_t k = rep.key(s[lds_pad(t)]);
        if (k == INVALID_KEY || (t > 0 && rep.key(s[lds_pad(t - 1)]) == k)) continue;
        uint32_t sum = 0;
        for (int e = t; e < P; ++e) {
            const T v = s[lds_pad(e)];
            if (rep.key(v) != k) break;
            sum += rep.weight(v);
        }
        const int64_t at = staged_at(r, a + rank);
        c.cs.hg_adj[at] = (int32_t)k;
        c.cs.hg_ew[at] = sum;
        ++rank;
    }
    return (int32_t)total;
}

// The keys of a group lie in its first and last entries' buckets (the
// entries are in bucket order): the narrow form's key base and span.
__device__ __forceinline__ void hg_key_range(const Ctx &c, const RowSrc &r, int32_t a, int32_t m,
                                             int shb, uint32_t &base, int64_t &span) {
    const uint32_t k0 = (uint32_t)c.cs.tmp_adj[staged_at(r, a)];
    const uint32_t k1 = (uint32_t)c.cs.tmp_adj[staged_at(r, a + m - 1)];
    base = (k0 >> shb) << shb;
    span = ((int64_t)(k1 >> shb) + 1 - (k0 >> shb)) << shb;
}
__device__ __forceinline__ int hg_shift(int64_t nc) {
    int shb = 0;
    while ((((nc > 0 ? nc : 1) - 1) >> shb) >= HG_BINS) ++shb;   // keys < nc -> buckets < HG_BINS
    return shb;
}

// A group's P values (m entries, the rest padding) into s, sorted (block or
// wave sort by NT), then merged; returns the merged count.
template <int NT, class Rep>
__device__ __forceinline__ int32_t hg_group(const Ctx &c, const RowSrc &r, int32_t a, int32_t m,
                                            int P, typename Rep::T *s, const Rep &rep,
                                            int64_t *sh) {
    using T = typename Rep::T;
    const int tid = NT == WAVE ? lane_id() : (int)threadIdx.x;
    for (int t0 = tid; t0 < P; t0 += NT * 4) {
        T val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * NT;
            val[u] = (T)~(T)0;
            if (t < m) {
                const int64_t at = staged_at(r, a + t);
                val[u] = rep.make((uint32_t)c.cs.tmp_adj[at], c.cs.tmp_ew[at], t);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t0 + u * NT < P) s[t0 + u * NT] = val[u];
    }
    if (NT == WAVE) {
        wave_sync_lds();
        if (P == WAVE) block_sort_regs<1, WAVE, T>(s, tid);
        else if (P == 2 * WAVE) block_sort_regs<2, WAVE, T>(s, tid);
        else if (P == 4 * WAVE) block_sort_regs<4, WAVE, T>(s, tid);
        else block_sort_regs<8, WAVE, T>(s, tid);
        wave_sync_lds();
    } else {
        __syncthreads();
        block_sort<NT, T>(s, P);
    }
    return hg_emit<NT>(c, s, P, r, a, sh, rep);
}

// Groups of at most WR_P entries: one wave each, sorted in registers.
__global__ void __launch_bounds__(BLOCK) fill_huge_small_k(Ctx c, int l) {
    __shared__ uint64_t lds[(BLOCK / WAVE) * lds_padded(WR_P)];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    const int64_t nc = c.lv[l + 1].n;
    if (nc > HUGE_NC_MAX) return;
    const int shb = hg_shift(nc);
    const int wv = threadIdx.x / WAVE, lane = lane_id();
    uint64_t *sl = lds + wv * lds_padded(WR_P);
    uint32_t *sl32 = (uint32_t *)sl;
    const int32_t *list = class_list(c.cs, g.n, 2);
    const int64_t count = min<int64_t>(c.cs.hg_cnt[0], c.cs.hg_cap);
    for (int64_t q = (int64_t)blockIdx.x * (BLOCK / WAVE) + wv; q < count;
         q += (int64_t)gridDim.x * (BLOCK / WAVE)) {   // wave-uniform
        const int4 d = c.cs.hg_small[q];
        const RowSrc r = row_src(g, c, list[d.x]);
        const int32_t a = d.y, m = d.z;
        int P = WAVE;
        while (P < m) P <<= 1;
        uint32_t base;
        int64_t span;
        hg_key_range(c, r, a, m, shb, base, span);
        const int lp = __builtin_ctz(P);
        const int32_t merged =
            narrow_fits(span, lp)
                ? hg_group<WAVE>(c, r, a, m, P, sl32, NarrowRep{sl32 + lds_padded(WR_P), lp, base},
                                 nullptr)
                : hg_group<WAVE>(c, r, a, m, P, sl, WideRep{}, nullptr);
        if (lane == 0) c.cs.hg_slot[d.w].y = merged;
        wave_sync_lds();   // the slice is reloaded for the wave's next group
    }
}

// The larger groups: one block of NT threads each, those of MIN+1..PMAX
// entries (a block of BLOCK threads sorts up to MID_P in registers with few
// barriers; the 1024-thread blocks take only the groups beyond that).
template <int NT, int PMAX, int MIN>
__device__ __forceinline__ void huge_group_body(const Ctx &c, int l, uint64_t *s, int64_t *sh) {
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    const int64_t nc = c.lv[l + 1].n;
    if (nc > HUGE_NC_MAX) return;
    const int shb = hg_shift(nc);
    uint32_t *s32 = (uint32_t *)s;
    const int32_t *list = class_list(c.cs, g.n, 2);
    const int64_t count = min<int64_t>(c.cs.hg_cnt[1], c.cs.hg_cap);
    for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {   // block-uniform
        const int4 d = c.cs.hg_big[q];
        const int32_t a = d.y, m = d.z;
        if (m <= MIN) continue;   // the other group kernel's
        int P = 2;
        while (P < m) P <<= 1;
        if (P > PMAX) {
            // the mid kernel leaves these to the big one; valid groups never
            // exceed the big kernel's sort
            if (PMAX == BIG_P && threadIdx.x == 0) atomicOr(&c.ctrl->flags, (uint32_t)CF_STATE);
            continue;
        }
        const RowSrc r = row_src(g, c, list[d.x]);
        uint32_t base;
        int64_t span;
        hg_key_range(c, r, a, m, shb, base, span);
        const int lp = __builtin_ctz(P);
        const int32_t merged =
            narrow_fits(span, lp)
                ? hg_group<NT>(c, r, a, m, P, s32, NarrowRep{s32 + lds_padded(PMAX), lp, base}, sh)
                : hg_group<NT>(c, r, a, m, P, s, WideRep{}, sh);
        if (threadIdx.x == 0) c.cs.hg_slot[d.w].y = merged;
        __syncthreads();   // s is reloaded for the block's next group
    }
}
__global__ void __launch_bounds__(BLOCK) fill_huge_mid_k(Ctx c, int l) {
    __shared__ uint64_t s[lds_padded(MID_P)];
    __shared__ int64_t sh[BLOCK / WAVE + 1];
    huge_group_body<BLOCK, MID_P, WR_P>(c, l, s, sh);
}
__global__ void __launch_bounds__(HUGE_THREADS) fill_huge_big_k(Ctx c, int l) {
    __shared__ uint64_t s[lds_padded(BIG_P)];
    __shared__ int64_t sh[HUGE_THREADS / WAVE + 1];
    huge_group_body<HUGE_THREADS, BIG_P, MID_P>(c, l, s, sh);
}

// Each large row's merged groups packed from position 0 on.
__global__ void __launch_bounds__(HUGE_THREADS) fill_huge_pack_k(Ctx c, int l) {
    constexpr int NT = HUGE_THREADS;
    constexpr int WPT = (HG_WINS + NT - 1) / NT;
    __shared__ int32_t off[HG_WINS + 1], first[HG_WINS];
    __shared__ int64_t sh[NT / WAVE + 1];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_CONTRACT, g)) return;
    const int64_t nc = c.lv[l + 1].n;
    if (nc > HUGE_NC_MAX) return;
    const int64_t count = c.cs.row_cnt[2];
    const int32_t *list = class_list(c.cs, g.n, 2);
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        const int32_t x = list[i];
        const RowSrc r = row_src(g, c, x);
        if (!huge_row(nc, r.tot)) continue;   // block-uniform
        if (i >= c.cs.hg_rows) continue;   // flagged by the prep
        const int2 ri = c.cs.hg_row[i];
        if (ri.x < 0 || ri.y > HG_WINS || (int64_t)ri.x + ri.y > c.cs.hg_cap) continue;
        const int32_t nwin = ri.y;
        int32_t gv[WPT];
        int64_t gsum = 0;
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int j = threadIdx.x * WPT + q;
            gv[q] = 0;
            if (j < nwin) {
                const int2 sl = c.cs.hg_slot[ri.x + j];
                first[j] = sl.x;
                gv[q] = sl.y;
            }
            gsum += gv[q];
        }
        int64_t total;
        int64_t o = block_excl_scan(gsum, sh, &total);
#pragma unroll
        for (int q = 0; q < WPT; ++q) {
            const int j = threadIdx.x * WPT + q;
            if (j < nwin) off[j] = (int32_t)o;
            o += gv[q];
        }
        if (threadIdx.x == 0) off[nwin] = (int32_t)total;
        __syncthreads();
        // four positions per thread, loaded before they are stored
        for (int64_t p0 = threadIdx.x; p0 < total; p0 += 4 * NT) {
            int32_t kk[4];
            uint32_t ww[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t p = p0 + (int64_t)u * NT;
                if (p >= total) continue;
                int lo = 0, hi = nwin - 1;   // the group holding output position p
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (off[mid] <= p) lo = mid;
                    else hi = mid - 1;
                }
                const int64_t src = staged_at(r, first[lo] + (p - off[lo]));
                kk[u] = c.cs.hg_adj[src];
                ww[u] = c.cs.hg_ew[src];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t p = p0 + (int64_t)u * NT;
                if (p >= total) continue;
                const int64_t dst = staged_at(r, p);
                c.cs.tmp_adj[dst] = kk[u];
                c.cs.tmp_ew[dst] = ww[u];
            }
        }
        if (threadIdx.x == 0) c.cs.cdeg[x] = (int32_t)total;
        __syncthreads();   // off and first are rewritten for the next row
    }
}

// --- 4. compaction ----------------------------------------------------------------
// Also writes Out(x) = sum of the coarse row's weights when the rating needs
// it (innerOuter): the next level's matching reads it.
template <int NT>
__device__ __forceinline__ void compact_small_body(const Ctx &c, int l, unsigned bid, unsigned nb) {
    constexpr int ROWS = NT / ROW_SMALL_G;
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_COMPACT, g)) return;
    const LevelDesc *N = c.lv + l + 1;
    uint32_t *out = c.rating == KAPPA_INNER_OUTER ? c.ms.out : nullptr;
    const int grp = threadIdx.x / ROW_SMALL_G, sub = threadIdx.x % ROW_SMALL_G;
    const int64_t count = N->n;
    const int64_t gs = (int64_t)nb * ROWS;
    const int64_t lim = (count + gs - 1) / gs * gs;   // uniform trip count (group shuffles)
    for (int64_t x = (int64_t)bid * ROWS + grp; x < lim; x += gs) {
        int32_t len = x < count ? c.cs.cdeg[x] : 0;
        bool mine = len > 0;
        RowSrc r;
        if (mine) {
            r = row_src(g, c, (int32_t)x);
            mine = row_bound(r) <= c.t.row_small_max;   // else compact_big copies it
        }
        uint32_t sum = 0;
        if (mine && len <= ROW_SMALL_G) {   // one entry per lane
            const int64_t dst = N->xadj[x];
            if (sub < len) {
                const int64_t at = staged_at(r, sub);
                const int32_t k = c.cs.tmp_adj[at];
                const uint32_t w = c.cs.tmp_ew[at];
                N->adj[dst + sub] = k;
                N->ew[dst + sub] = w;
                sum = w;
            }
        } else if (mine) {
            // a lane's entries loaded before any is stored (the stores could
            // alias the loads as far as the compiler knows)
            constexpr int U = (SM_CAP + ROW_SMALL_G - 1) / ROW_SMALL_G;
            const int64_t dst = N->xadj[x];
            int32_t kk[U];
            uint32_t ww[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = sub + u * ROW_SMALL_G;
                if (t < len) {
                    const int64_t at = staged_at(r, t);
                    kk[u] = c.cs.tmp_adj[at];
                    ww[u] = c.cs.tmp_ew[at];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = sub + u * ROW_SMALL_G;
                if (t < len) {
                    N->adj[dst + t] = kk[u];
                    N->ew[dst + t] = ww[u];
                    sum += ww[u];
                }
            }
        }
        if (out) {
            for (int o = ROW_SMALL_G / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, ROW_SMALL_G);
            if (sub == 0 && x < count && (mine || len == 0)) out[x] = sum;
        }
    }
}

// Rows of 65..512 entries (class 1): one wave each.
template <int NT>
__device__ __forceinline__ void compact_wave_body(const Ctx &c, int l, unsigned bid, unsigned nb) {
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_COMPACT, g)) return;
    const LevelDesc *N = c.lv + l + 1;
    uint32_t *out = c.rating == KAPPA_INNER_OUTER ? c.ms.out : nullptr;
    const int64_t c1 = c.cs.row_cnt[1];
    const int32_t *list = class_list(c.cs, g.n, 1);
    const int lane = lane_id();
    for (int64_t i = (int64_t)bid * (NT / WAVE) + threadIdx.x / WAVE; i < c1;
         i += (int64_t)nb * (NT / WAVE)) {   // wave-uniform
        const int32_t x = list[i];
        const RowSrc r = row_src(g, c, x);
        const int64_t dst = N->xadj[x];
        const int32_t len = c.cs.cdeg[x];
        uint32_t sum = 0;
        // a lane's entries loaded before any is stored
        constexpr int U = ROW_WAVE_MAX / WAVE;
        int32_t kk[U];
        uint32_t ww[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = lane + u * WAVE;
            if (t < len) {
                const int64_t at = staged_at(r, t);
                kk[u] = c.cs.tmp_adj[at];
                ww[u] = c.cs.tmp_ew[at];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = lane + u * WAVE;
            if (t < len) {
                N->adj[dst + t] = kk[u];
                N->ew[dst + t] = ww[u];
                sum += ww[u];
            }
        }
        if (out) {
            sum = wave_sum(sum);
            if (lane == 0) out[x] = sum;
        }
    }
}

// Rows of the classes above (from `first_cls`): one block each.
template <int NT>
__device__ __forceinline__ void compact_big_body(const Ctx &c, int l, unsigned bid, unsigned nb,
                                                 int first_cls = 1) {
    __shared__ uint32_t sh[NT / WAVE + 1];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_COMPACT, g)) return;
    const LevelDesc *N = c.lv + l + 1;
    uint32_t *out = c.rating == KAPPA_INNER_OUTER ? c.ms.out : nullptr;
    const int64_t c1 = first_cls <= 1 ? c.cs.row_cnt[1] : 0, c2 = c.cs.row_cnt[2],
                  c3 = c.cs.row_cnt[3], c4 = c.cs.row_cnt[4];
    for (int64_t i = bid; i < c1 + c2 + c3 + c4; i += nb) {
        const int32_t x = i < c1 ? class_list(c.cs, g.n, 1)[i]
                        : i < c1 + c2 ? class_list(c.cs, g.n, 2)[i - c1]
                        : i < c1 + c2 + c3 ? class_list(c.cs, g.n, 3)[i - c1 - c2]
                                           : class_list(c.cs, g.n, 4)[i - c1 - c2 - c3];
        RowSrc r = row_src(g, c, x);
        int64_t dst = N->xadj[x];
        int32_t len = c.cs.cdeg[x];
        uint32_t sum = 0;
        // four entries per thread loaded before they are stored
        for (int t0 = threadIdx.x; t0 < len; t0 += 4 * NT) {
            int32_t kk[4];
            uint32_t ww[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * NT;
                if (t < len) {
                    const int64_t at = staged_at(r, t);
                    kk[u] = c.cs.tmp_adj[at];
                    ww[u] = c.cs.tmp_ew[at];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * NT;
                if (t < len) {
                    N->adj[dst + t] = kk[u];
                    N->ew[dst + t] = ww[u];
                    sum += ww[u];
                }
            }
        }
        if (out) {
            sum = block_sum(sum, sh);
            if (threadIdx.x == 0) out[x] = sum;
        }
    }
}
// Every row kind in one launch: blocks [0, small_blocks) copy the small rows,
// the next wave_blocks the rows of 65..512 entries a wave each, the rest the
// longer rows a block each.
__global__ void __launch_bounds__(BLOCK) compact_k(Ctx c, int l, unsigned small_blocks,
                                                   unsigned wave_blocks) {
    if (blockIdx.x < small_blocks)
        compact_small_body<BLOCK>(c, l, blockIdx.x, small_blocks);
    else if (blockIdx.x < small_blocks + wave_blocks)
        compact_wave_body<BLOCK>(c, l, blockIdx.x - small_blocks, wave_blocks);
    else
        compact_big_body<BLOCK>(c, l, blockIdx.x - small_blocks - wave_blocks,
                                gridDim.x - small_blocks - wave_blocks, 2);
}

// ===========================================================================
// Tail: once a level is small, that level and every later one run in a single
// workgroup, in one launch.  A deep level is a few thousand nodes; as separate
// grid launches it pays for some twenty launches (each waiting for the one
// before), while here its phases are separated by workgroup barriers and its
// arrays stay in the L2 of one XCD from one level to the next.  The phases
// and their results are those of the grid kernels (same functions, one block).
// ===========================================================================
// One level's matching and contraction, as separate (not inlined) functions
// so that each phase gets the registers of the whole thread.
// Matching state shared by the two halves of a tail level's matching.
struct TailMatchLds {
    int32_t cnt[2][4];   // list sizes by round parity ([.][3] unused)
};

template <int R>
__device__ __noinline__ void tail_round1(const Ctx &c, int l, TailMatchLds &t) {
    __shared__ Cand shc[TAIL_THREADS / WAVE];
    __shared__ int64_t sh[5 * (TAIL_THREADS / WAVE) + 1];
    __shared__ int32_t sbase[3];
    LevelDesc *L = c.lv + l;
    DevGraph g;
    load_level(L, PH_MATCH, g);
    if (threadIdx.x < 4) t.cnt[0][threadIdx.x] = t.cnt[1][threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        L->matched = 0;
        L->rounds = 0;
    }
    __syncthreads();
    const uint64_t seed = level_seed(c, l);
    init_phase(c, g, L, sh, sbase, 0, 1, t.cnt[0], false);
    __syncthreads();
    const RoundIn ri = round_inputs<true>(c, g, 1, t.cnt[0]);
    pick_bin0<R, true>(c, g, seed, ri, 0, 1);
    pick_bin1<R, true>(c, g, seed, ri, 0, 1);
    __syncthreads();
    pick_bin2<R, true, TAIL_THREADS>(c, g, seed, ri, 0, 1, shc);
    __syncthreads();
    mate_phase<R, true>(c, g, L, 1, ri, t.cnt[1], 0, 1, sh, sbase);
    __syncthreads();
}

template <int R>
__device__ __noinline__ void tail_rounds(const Ctx &c, int l, TailMatchLds &t) {
    __shared__ Cand shc[TAIL_THREADS / WAVE];
    __shared__ int64_t sh[5 * (TAIL_THREADS / WAVE) + 1];
    __shared__ int32_t sbase[3];
    __shared__ int64_t s_acc[2];
    LevelDesc *L = c.lv + l;
    DevGraph g;
    load_level(L, PH_MATCH, g);
    const bool capped =
        wg_rounds<R, TAIL_THREADS>(c, g, L, level_seed(c, l), 1, t.cnt, shc, sh, sbase);
    close_matching<TAIL_THREADS>(c, L, capped, 0, s_acc);
}

__device__ __noinline__ void tail_merge(const Ctx &c, int l) {
    // no LDS for the big-row sort next to the other phases: those rows take
    // the large rows' accumulators
    fill_small_body<TAIL_THREADS, false>(c, l, 0, 1);
    __syncthreads();
    fill_mid_body<TAIL_THREADS>(c, l, 0, 1, 1);   // the wave class by the block sort here
    __syncthreads();
    fill_mid_body<TAIL_THREADS>(c, l, 0, 1);
    __syncthreads();
    fill_large_body<TAIL_THREADS, 128>(c, l, 0, 1);
    __syncthreads();
}

__device__ __noinline__ void tail_offsets(const Ctx &c, int l) {
    __shared__ int64_t sh[ONE_SCAN_THREADS / WAVE + 1];
    __shared__ int go;
    scan_one_block(DegF{c, l}, CoarseOffW{c, l}, c.cs.totals + 2, sh, &go);
    __syncthreads();
}

__device__ __noinline__ void tail_compact(const Ctx &c, int l) {
    compact_small_body<TAIL_THREADS>(c, l, 0, 1);
    __syncthreads();
    compact_big_body<TAIL_THREADS>(c, l, 0, 1);
    __syncthreads();
}

template <int R>
__global__ void __launch_bounds__(TAIL_THREADS) tail_k(Ctx c, int l0) {
    __shared__ int go;
    __shared__ TailMatchLds t;
    for (int l = l0; l < MAX_LEVELS; ++l) {
        if (threadIdx.x == 0) {
            const LevelDesc *L = c.lv + l;
            // every later level is no larger, so the tail keeps them all
            const bool fits = L->n <= TAIL_MAX_N && L->nnz <= TAIL_MAX_NNZ;
            go = fits && level_gate(c, l, true, true);
        }
        __syncthreads();
        if (!go) return;
        tail_round1<R>(c, l, t);
        tail_rounds<R>(c, l, t);
        ids_one_block(c, l);
        tail_merge(c, l);
        tail_offsets(c, l);
        tail_compact(c, l);
        LevelDesc *L = c.lv + l;
        if (threadIdx.x == 0 && L->phase == PH_COMPACT) L->phase = PH_DONE;
        __syncthreads();
    }
}

// ===========================================================================
// Batched form: per-graph stop rules (one workgroup; graphs are few next to
// nodes).  A graph's coarsest level and stop reason are recorded when it
// stops; it is frozen from then on.
// ===========================================================================
constexpr int BATCH_THREADS = 1024;

__global__ void __launch_bounds__(BATCH_THREADS) batch_begin_k(Ctx c, int l) {
    __shared__ int any, stopped, cut;
    Control *ctrl = c.ctrl;
    LevelDesc *L = c.lv + l;
    if (ctrl->done || ctrl->nlevels != l + 1 || L->phase != PH_IDLE) return;   // same for all
    if (threadIdx.x == 0) {
        any = 0;
        stopped = 0;
    }
    __syncthreads();
    const int32_t *noff = L->noff;
    const int32_t maxl = ctrl->max_levels;
    bool mine = false, st = false;
    for (int g = threadIdx.x; g < c.b.count; g += blockDim.x) {
        if (!c.b.active[g]) continue;
        const int32_t ng = noff[g + 1] - noff[g];
        const int32_t lim = c.b.lmax ? c.b.lmax[g] : maxl;
        int32_t stop = KAPPA_STOP_NONE;
        if (ng <= c.b.stop_n[g]) stop = KAPPA_STOP_SIZE;
        else if (l >= lim) stop = KAPPA_STOP_MAXLEVEL;
        if (stop != KAPPA_STOP_NONE) {
            c.b.active[g] = 0;
            c.b.coarsest[g] = l;
            c.b.reason[g] = stop;
            st = true;
        } else {
            mine = true;
            if (c.b.gbase) c.b.gseed[g] = mix64(c.b.gbase[g] + (uint64_t)l);
        }
    }
    if (mine) any = 1;
    if (st) stopped = 1;
    __syncthreads();
    // a served step ends here if a graph has stopped in it or the host asks
    // for a boundary (one read of each flag, shared by the block)
    if (threadIdx.x == 0) {
        cut = 0;
        if (c.b.stop_seen && l > 0 && any)
            cut = stopped || *c.b.stop_seen ||
                  (c.b.interrupt &&
                   __hip_atomic_load(c.b.interrupt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
    }
    __syncthreads();
    if (cut) {
        for (int g = threadIdx.x; g < c.b.count; g += blockDim.x) {
            if (!c.b.active[g]) continue;
            c.b.active[g] = 0;
            c.b.coarsest[g] = l;
            c.b.reason[g] = KAPPA_STOP_NONE;   // goes on in the next step
        }
    }
    if (threadIdx.x == 0 && (!any || cut)) {   // every graph has stopped: so does the union
        L->stop = KAPPA_STOP_SIZE;
        L->phase = PH_STOPPED;
        ctrl->done = 1;
    }
}

__global__ void __launch_bounds__(BATCH_THREADS) batch_end_k(Ctx c, int l) {
    const LevelDesc *L = c.lv + l, *N = c.lv + l + 1;
    if (L->phase != PH_COMPACT) return;   // the level did not contract
    const int32_t n = L->n, nc = N->n;
    const int32_t *noff = L->noff;
    int32_t *noffN = N->noff;
    for (int g = threadIdx.x; g <= c.b.count; g += blockDim.x)
        noffN[g] = noff[g] < n ? c.b.excl[noff[g]] : nc;
    __syncthreads();
    for (int g = threadIdx.x; g < c.b.count; g += blockDim.x) {
        if (!c.b.active[g]) continue;
        const int64_t ng = noff[g + 1] - noff[g], ngc = noffN[g + 1] - noffN[g];
        if (ngc == ng) {   // no pair: the level just built is a copy, dropped
            c.b.active[g] = 0;
            c.b.coarsest[g] = l;
            c.b.reason[g] = KAPPA_STOP_EMPTY;
            if (c.b.stop_seen) *c.b.stop_seen = 1;
        } else if (c.b.stall_num > 0 &&
                   (uint64_t)(ng - ngc) * c.b.stall_den < (uint64_t)c.b.stall_num * (uint64_t)ng) {
            c.b.active[g] = 0;
            c.b.coarsest[g] = l + 1;
            c.b.reason[g] = KAPPA_STOP_STALL;
            if (c.b.stop_seen) *c.b.stop_seen = 1;
        }
    }
}

// gid[v] = the graph of node v: the last g with noff[g] <= v (empty graphs
// are skipped).  Per block-sized tile of nodes, one binary search over the
// count + 1 ascending offsets finds the graph of the tile's first node; each
// thread walks on from there (a tile spans few graphs).
__device__ __forceinline__ int32_t graph_of(const int32_t *noff, int32_t count, int64_t v) {
    int32_t lo = 0, hi = count - 1;   // noff[lo] <= v < noff[hi + 1]
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (noff[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__global__ void __launch_bounds__(BLOCK) batch_gid_k(const int32_t *noff, int32_t count, int32_t n,
                                                     int32_t *gid) {
    __shared__ int32_t g0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
         base += (int64_t)gridDim.x * blockDim.x) {   // block-uniform
        if (threadIdx.x == 0) g0 = graph_of(noff, count, base);
        __syncthreads();
        const int64_t v = base + threadIdx.x;
        if (v < n) {
            int32_t g = g0;
            while (g + 1 < count && noff[g + 1] <= v) ++g;
            gid[v] = g;
        }
        __syncthreads();   // g0 is rewritten for the next tile
    }
}

// Rows ascend, so a row stays inside its graph iff its first and last entries do.
__global__ void batch_check_k(DevGraph g, uint32_t *flags) {
    bool bad = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = g.xadj[v], e = g.xadj[v + 1];
        if (b == e) continue;
        const int32_t q = g.gid[v];
        if (g.adj[b] < g.noff[q] || g.adj[e - 1] >= g.noff[q + 1]) bad = true;
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(flags, 1u);
}

// One graph's level out of a batch level: node range [a, b) of the union,
// entries from ea; ids made local (cmap relative to the graph's first node
// on the next level, cbase; cmap null on the coarsest level).
__global__ void batch_extract_k(DevGraph u, const int32_t *cmap, const int32_t *mate, int32_t a,
                                int32_t b, int64_t ea, int32_t cbase, int64_t *xadj, int32_t *adj,
                                uint32_t *ew, uint32_t *vw, int32_t *cmap_out, int32_t *mate_out) {
    const int32_t n = b - a;
    const int64_t nnz = u.xadj[b] - ea;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
        xadj[i] = u.xadj[a + i] - ea;
        if (i == n) continue;
        vw[i] = u.vw[a + i];
        if (cmap) cmap_out[i] = cmap[a + i] - cbase;
        if (mate) {
            const int32_t m = mate[a + i];
            mate_out[i] = m >= 0 ? m - a : -1;
        }
    }
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += stride) {
        adj[j] = u.adj[ea + j] - a;
        ew[j] = u.ew[ea + j];
    }
}

// Served steps: level j of every graph of a step's union, with ids made
// local, in one pass (and each graph's largest degree there, in dmax, which
// starts at zero).  Graph g's arrays keep their place in the union
// (nodes from noff1[g], entries from the union's offsets); its row offsets
// need one slot more per graph, so they start at noff1[g] + g.  cmap of the
// union's level j - 1 is made local as well (-1 for nodes of graphs that
// stopped).
__global__ void __launch_bounds__(BLOCK) serve_extract_k(DevGraph u1, const int32_t *noff1,
                                                         int32_t count, int64_t *xadj,
                                                         int32_t *adj, uint32_t *ew,
                                                         uint32_t *vw, int32_t *dmax) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // nodes: a block-uniform loop, so that whole waves take part in the
    // degree maximum (one atomic per wave whose nodes share a graph, the
    // usual case: a graph's nodes are consecutive)
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < u1.n; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool live = i < u1.n;
        int32_t g = -1, d = 0;
        if (live) {
            g = u1.gid[i];
            const int32_t a = noff1[g];
            const int64_t e0 = u1.xadj[a];
            const int64_t x = u1.xadj[i];
            xadj[i + g] = x - e0;
            vw[i] = u1.vw[i];
            d = (int32_t)(u1.xadj[i + 1] - x);
        }
        const int32_t g0 = __shfl(g, 0, WAVE);
        if (__all(!live || g == g0)) {
            const int32_t m = wave_max(d);
            if (lane_id() == 0 && g0 >= 0 && m > 0) atomicMax(&dmax[g0], m);
        } else if (live && d > 0) {
            atomicMax(&dmax[g], d);
        }
    }
    for (int64_t g = t0; g < count; g += stride) {   // each graph's closing offset
        const int32_t a = noff1[g], b = noff1[g + 1];
        xadj[(int64_t)b + g] = u1.xadj[b] - u1.xadj[a];
    }
    for (int64_t j = t0; j < u1.nnz; j += stride) {
        const int32_t w = u1.adj[j];
        adj[j] = w - noff1[u1.gid[w]];
        ew[j] = u1.ew[j];
    }
}

__global__ void __launch_bounds__(BLOCK) serve_cmap_k(const int32_t *cmap0, const int32_t *gid0,
                                                      int32_t n0, const int32_t *noff1,
                                                      int32_t *cmap) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = cmap0[i];
        cmap[i] = x >= 0 ? x - noff1[gid0[i]] : -1;
    }
}

// The first entry of every graph on a level: e[g] = xadj[noff[g]], g <= count.
__global__ void __launch_bounds__(BLOCK) serve_eoff_k(const int64_t *xadj, const int32_t *noff,
                                                      int32_t count, int64_t *e) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= count;
         g += (int64_t)gridDim.x * blockDim.x)
        e[g] = xadj[noff[g]];
}

void launch_serve_extract(const DevGraph &u1, const int32_t *noff1, int32_t count,
                          const int32_t *cmap0, const int32_t *gid0, int32_t n0, int64_t *xadj,
                          int32_t *adj, uint32_t *ew, uint32_t *vw, int32_t *cmap, int64_t *eoff1,
                          int32_t *dmax, hipStream_t s) {
    KAPPA_PROF("serve_extract", s);
    const int64_t items = std::max<int64_t>(std::max<int64_t>(u1.n, u1.nnz), count + 1);
    if (u1.n > 0 || count > 0)
        hipLaunchKernelGGL(serve_extract_k, dim3(grid_for(items, BLOCK * 4, 4096)), dim3(BLOCK), 0, s,
                           u1, noff1, count, xadj, adj, ew, vw, dmax);
    if (n0 > 0)
        hipLaunchKernelGGL(serve_cmap_k, dim3(grid_for(n0, BLOCK * 4, 4096)), dim3(BLOCK), 0, s,
                           cmap0, gid0, n0, noff1, cmap);
    hipLaunchKernelGGL(serve_eoff_k, dim3(grid_for(count + 1, BLOCK, 64)), dim3(BLOCK), 0, s,
                       u1.xadj, noff1, count, eoff1);
}

// Union of separate graphs (kappa_coarsen_graphs): graph g's nodes and
// entries move to offsets noff[g] and eoff[g], its ids and row offsets are
// shifted by those.  The graph of an item is found by binary search over
// the offsets (count + 1 ascending values).
__device__ __forceinline__ int32_t owner_of(const int64_t *off, int32_t count, int64_t i) {
    int32_t lo = 0, hi = count - 1;   // largest g with off[g] <= i
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(BLOCK) union_nodes_k(const UnionSrc *src, int32_t count,
                                                       const int64_t *noff, const int64_t *eoff,
                                                       int64_t *xadj, uint32_t *vw) {
    const int64_t n = noff[count];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
        if (v == n) {
            xadj[n] = eoff[count];
            continue;
        }
        const int32_t g = owner_of(noff, count, v);
        const int64_t i = v - noff[g];
        xadj[v] = src[g].xadj[i] + eoff[g];
        vw[v] = src[g].vw[i];
    }
}

__global__ void __launch_bounds__(BLOCK) union_entries_k(const UnionSrc *src, int32_t count,
                                                         const int64_t *noff, const int64_t *eoff,
                                                         int32_t *adj, uint32_t *ew) {
    const int64_t nnz = eoff[count];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += stride) {
        const int32_t g = owner_of(eoff, count, j);
        const int64_t i = j - eoff[g];
        adj[j] = src[g].adj[i] + (int32_t)noff[g];
        ew[j] = src[g].ew[i];
    }
}

void launch_union_build(const UnionSrc *src, int32_t count, const int64_t *noff,
                        const int64_t *eoff, int64_t n, int64_t nnz, int64_t *xadj, int32_t *adj,
                        uint32_t *ew, uint32_t *vw, hipStream_t s) {
    {
        KAPPA_PROF("union_nodes", s);
        hipLaunchKernelGGL(union_nodes_k, dim3(grid_for(n + 1, BLOCK * 4, 8192)), dim3(BLOCK), 0, s,
                           src, count, noff, eoff, xadj, vw);
    }
    if (nnz > 0) {
        KAPPA_PROF("union_entries", s);
        hipLaunchKernelGGL(union_entries_k, dim3(grid_for(nnz, BLOCK * 4, 8192)), dim3(BLOCK), 0, s,
                           src, count, noff, eoff, adj, ew);
    }
}

// ===========================================================================
// Host side
// ===========================================================================

// Launched only when the long rows of the level are scanned in chunks.
template <bool FIRST>
static void launch_hub_reduce(const Ctx &c, int l, int r, hipStream_t s) {
    if (!c.ms.hub.rec) return;
    KAPPA_PROF("hub_reduce", s);
    hipLaunchKernelGGL(hub_reduce_k<FIRST>, dim3(256), dim3(BLOCK), 0, s, c, l, r);
}

// Grid round r >= 2 (e: estimate of the pending entries).  With long rows in
// chunks: preparation (the rows that rescan), pick over those, reduction of
// the chunked rows, mutual check; otherwise pick over the pending lists and
// the mutual check.
template <int R>
static void launch_later_round(const Ctx &c, int l, int r, const PickGrid &pg, int64_t e,
                               hipStream_t s) {
    const unsigned pick_blocks = pg.b0 + pg.b1 + pg.b2;
    const unsigned list_blocks = grid_for(e, BLOCK, 2048);
    if (c.ms.hub.rec) {
        {
            KAPPA_PROF("prep", s);
            hipLaunchKernelGGL(prep_k, dim3(grid_for(e, BLOCK * MK, 2048)), dim3(BLOCK), 0, s, c,
                               l, r);
        }
        {
            KAPPA_PROF("pick", s);
            hipLaunchKernelGGL((pick_k<R, false, 0, true>), dim3(pick_blocks), dim3(BLOCK), 0, s,
                               c, l, r, pg);
        }
        launch_hub_reduce<false>(c, l, r, s);
    } else {
        KAPPA_PROF("pick", s);
        hipLaunchKernelGGL((pick_k<R, false>), dim3(pick_blocks), dim3(BLOCK), 0, s, c, l, r, pg);
    }
    KAPPA_PROF("mate", s);
    hipLaunchKernelGGL((mate_k<R, false>), dim3(list_blocks), dim3(BLOCK), 0, s, c, l, r);
}

// ---------------------------------------------------------------------------
// Persistent matching rounds (opt-in, kappa_persistent_enable): rounds 2, 3,
// ... of a level in one cooperative launch (every block resident), the pick
// and mate phases of a round separated by grid barriers, until the pending
// set is empty or small enough for the finisher (the same hand-over tests as
// the round kernels) or r_cap rounds have run.  Levels whose long rows are
// scanned in chunks (power-law graphs) keep the round kernels.
// ---------------------------------------------------------------------------
bool g_persistent_on = false;
constexpr int COOP_SPIN_LIMIT = 1 << 24;   // polls before a barrier wait gives up

// Grid barrier: bar[0] the generation, bar[1] the groups arrived, bar[2 + g]
// the blocks of group g arrived (groups of ARRIVE_GROUP blocks).  The last
// arrival resets the counters and advances the generation.  A wait is
// bounded: after COOP_SPIN_LIMIT polls the block flags CF_STATE and returns
// false (the call then fails), so no wave spins forever.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, uint32_t *flags) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned gen0 = __hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();   // this block's writes before its arrival
        const unsigned nb = gridDim.x, grp = blockIdx.x / ARRIVE_GROUP;
        const unsigned ngrp = (nb + ARRIVE_GROUP - 1) / ARRIVE_GROUP;
        const unsigned gsz = min((unsigned)ARRIVE_GROUP, nb - grp * ARRIVE_GROUP);
        bool last = false;
        if (atomicAdd(&bar[2 + grp], 1u) == gsz - 1) {
            atomicExch(&bar[2 + grp], 0u);
            if (atomicAdd(&bar[1], 1u) == ngrp - 1) {
                atomicExch(&bar[1], 0u);
                last = true;
            }
        }
        if (last) {
            __threadfence();
            atomicAdd(&bar[0], 1u);
        } else {
            int spins = 0;
            while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen0) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > COOP_SPIN_LIMIT) {
                    atomicOr(flags, (uint32_t)CF_STATE);
                    ok = 0;
                    break;
                }
            }
        }
        __threadfence();   // the other blocks' writes before this block goes on
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

template <int R>
__global__ void __launch_bounds__(BLOCK) rounds_coop_k(Ctx c, int l, int r_first, int r_cap,
                                                       PickGrid pg) {
    __shared__ Cand shc[BLOCK / WAVE];
    __shared__ int64_t sh[5 * (BLOCK / WAVE) + 1];
    __shared__ int32_t sbase[3];
    DevGraph g;
    LevelDesc *L = c.lv + l;
    if (!load_level(L, PH_MATCH, g)) return;   // the same for every block
    MatchState *st = c.ms.state;
    const uint64_t seed = level_seed(c, l);
    for (int r = r_first; r <= r_cap; ++r) {
        // every block reads the same state after a barrier: uniform exits
        if (__hip_atomic_load(&st->handoff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != -1) return;
        const RoundIn ri = round_inputs<false>(c, g, r, st->cnt[(r - 1) & 3]);
        const int64_t total = (int64_t)ri.cn[0] + ri.cn[1] + ri.cn[2];
        if (total == 0 || total <= c.t.tail_max) {
            if (blockIdx.x == 0 && threadIdx.x == 0)
                atomicCAS(&st->handoff, -1, total == 0 ? -2 : r - 1);
            return;
        }
        unsigned bid = blockIdx.x;
        if (bid < pg.b0) {
            pick_bin0<R, false>(c, g, seed, ri, bid, pg.b0);
        } else if ((bid -= pg.b0) < pg.b1) {
            pick_bin1<R, false>(c, g, seed, ri, bid, pg.b1);
        } else {
            bid -= pg.b1;
            pick_bin2<R, false, BLOCK>(c, g, seed, ri, bid, pg.b2, shc);
        }
        if (!grid_barrier(c.ms.coop_bar, &c.ctrl->flags)) return;
        if (blockIdx.x == 0 && threadIdx.x < 4) {   // as mate_k
            st->cnt[(r + 2) & 3][threadIdx.x] = 0;
            st->scnt[(r + 2) & 3][threadIdx.x] = 0;
        }
        mate_phase<R, false>(c, g, L, r, ri, st->cnt[r & 3], blockIdx.x, gridDim.x, sh, sbase);
        if (!grid_barrier(c.ms.coop_bar, &c.ctrl->flags)) return;
    }
}

// Blocks of a cooperative launch of rounds_coop_k<R> on this device (every
// block resident), cached per rating.
template <int R>
static unsigned coop_blocks() {
    static unsigned cached[64] = {};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return 0;
    if (!cached[dev]) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rounds_coop_k<R>, BLOCK, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = (unsigned)std::min<int64_t>((int64_t)per_cu * cus, ARRIVE_MAX_BLOCKS);
    }
    return cached[dev];
}

template <int R>
static void match_impl(const Ctx &c, int l, int32_t n_hint, int rounds, hipStream_t s) {
    // per-round kernels; round r's grid follows a geometric estimate of the
    // pending count (any grid is correct: all loops stride)
    // power-law graphs keep most of their pending nodes for many rounds (hubs
    // wait on each other), so their grids do not shrink with the rounds
    const double decay = c.big_blocks > 64 ? 1.0 : 0.7;
    const unsigned coop = g_persistent_on && !c.ms.hub.rec ? coop_blocks<R>() : 0;
    double est = n_hint;
    for (int r = 1; r <= rounds; ++r, est *= decay) {
        if (r == 2 && coop >= 16) {
            // the later rounds in one persistent launch (if it cannot be
            // launched, the round kernels go on)
            const unsigned nb = std::min<unsigned>(coop, grid_for((int64_t)est + 1, BLOCK / SMALL_G,
                                                                  4096));
            PickGrid cg;
            cg.b2 = std::max(1u, std::min(64u, nb / 16));
            cg.b1 = std::max(1u, std::min(256u, nb / 4));
            cg.b0 = nb > cg.b1 + cg.b2 + 1 ? nb - cg.b1 - cg.b2 : 1;
            const unsigned grid = cg.b0 + cg.b1 + cg.b2;
            const int r_cap = std::max(rounds, STAT_ROUNDS - 2);
            if (grid <= coop) {
                hipError_t e;
                {
                    KAPPA_PROF("rounds_persistent", s);
                    Ctx cc = c;
                    int ll = l, r0 = 2, rc = r_cap;
                    void *args[] = {&cc, &ll, &r0, &rc, &cg};
                    e = hipLaunchCooperativeKernel((const void *)rounds_coop_k<R>, dim3(grid),
                                                   dim3(BLOCK), args, 0, s);
                }
                if (e == hipSuccess) {
                    KAPPA_PROF("match_finish", s);
                    hipLaunchKernelGGL(finish_k<R>, dim3(1), dim3(FINISH_THREADS), 0, s, c, l, r_cap);
                    return;
                }
                (void)hipGetLastError();   // not launched: no state changed
            }
        }
        int64_t e = (int64_t)est + 1;
        PickGrid pg;
        pg.b0 = grid_for(e, BLOCK / SMALL_G, 2048);
        pg.b1 = c.big_blocks > 64 ? 2u * c.big_blocks : grid_for(e, BLOCK / WAVE * 8, 128);
        pg.b2 = c.big_blocks > 64 ? (unsigned)c.big_blocks : grid_for(e, 4096, 64);
        const unsigned pick_blocks = pg.b0 + pg.b1 + pg.b2;
        const unsigned mate_blocks = grid_for(e, BLOCK, 2048);
        if (r == 1) {
            {
                KAPPA_PROF("pick_first", s);
                hipLaunchKernelGGL((pick_k<R, true>), dim3(pick_blocks), dim3(BLOCK), 0, s, c, l, r,
                                   pg);
            }
            launch_hub_reduce<true>(c, l, r, s);
            KAPPA_PROF("mate_first", s);
            hipLaunchKernelGGL((mate_k<R, true>), dim3(mate_blocks), dim3(BLOCK), 0, s, c, l, r);
        } else {
            launch_later_round<R>(c, l, r, pg, e, s);
        }
    }
    KAPPA_PROF("match_finish", s);
    hipLaunchKernelGGL(finish_k<R>, dim3(1), dim3(FINISH_THREADS), 0, s, c, l, rounds);
}

// Two-phase matcher: the block phase, a few gap rounds as grid launches (the
// gap graph is small: edges between blocks above both block edges; the
// finisher completes any remainder), then the merge.
template <int R>
static void two_phase_impl(const Ctx &c, int l, int32_t n_hint, hipStream_t s) {
    const int rounds = n_hint >= (1 << 17) ? 3 : (n_hint >= (1 << 14) ? 2 : 1);
    {
        KAPPA_PROF("block_match", s);
        const int64_t blocks = ((int64_t)n_hint + (1 << c.block_bits) - 1) >> c.block_bits;
        hipLaunchKernelGGL(block_match_k<R>, dim3(grid_for(blocks, 1, 4096)), dim3(BM_THREADS), 0,
                           s, c, l);
    }
    // the gap rounds start from the lists the block phase wrote (round 1 is
    // an ordinary later round); a quarter of the nodes is a generous start
    double est = n_hint / 4.0;
    for (int r = 1; r <= rounds; ++r, est *= 0.7) {
        int64_t e = (int64_t)est + 1;
        PickGrid pg;
        pg.b0 = grid_for(e, BLOCK / SMALL_G, 2048);
        pg.b1 = c.big_blocks > 64 ? 2u * c.big_blocks : grid_for(e, BLOCK / WAVE * 8, 128);
        pg.b2 = c.big_blocks > 64 ? (unsigned)c.big_blocks : grid_for(e, 4096, 64);
        {
            KAPPA_PROF("gap_pick", s);
            hipLaunchKernelGGL((pick_k<R, false, 1>), dim3(pg.b0 + pg.b1 + pg.b2), dim3(BLOCK), 0, s,
                               c, l, r, pg);
        }
        KAPPA_PROF("gap_mate", s);
        hipLaunchKernelGGL((mate_k<R, false>), dim3(grid_for(e, BLOCK, 2048)), dim3(BLOCK), 0, s, c,
                           l, r);
    }
    {
        KAPPA_PROF("gap_finish", s);
        hipLaunchKernelGGL((finish_k<R, 1>), dim3(1), dim3(FINISH_THREADS), 0, s, c, l, rounds);
    }
    {
        KAPPA_PROF("merge", s);
        hipLaunchKernelGGL(merge_k, dim3(grid_for(n_hint, BLOCK, 2048)), dim3(BLOCK), 0, s, c, l);
    }
    KAPPA_PROF("merge_close", s);
    hipLaunchKernelGGL(merge_close_k, dim3(1), dim3(WAVE), 0, s, c, l);
}

// More grid rounds for a level the finisher handed back (CF_EXTEND): rounds
// r_from+1 .. r_from+count, the finisher, then the level's contraction (and,
// batched, its end).
template <int R>
static void extend_impl(const Ctx &c, int l, int32_t n_hint, int r_from, int count, hipStream_t s) {
    const double decay = c.big_blocks > 64 ? 1.0 : 0.7;
    double est = n_hint * std::pow(decay, r_from);
    for (int r = r_from + 1; r <= r_from + count; ++r, est *= decay) {
        int64_t e = (int64_t)est + 1;
        PickGrid pg;
        pg.b0 = grid_for(e, BLOCK / SMALL_G, 2048);
        pg.b1 = c.big_blocks > 64 ? 2u * c.big_blocks : grid_for(e, BLOCK / WAVE * 8, 128);
        pg.b2 = c.big_blocks > 64 ? (unsigned)c.big_blocks : grid_for(e, 4096, 64);
        launch_later_round<R>(c, l, r, pg, e, s);
    }
    KAPPA_PROF("match_finish", s);
    hipLaunchKernelGGL(finish_k<R>, dim3(1), dim3(FINISH_THREADS), 0, s, c, l, r_from + count);
}

void launch_level_extend(const Ctx &c, int l, int32_t n_hint, int32_t n_cap, int r_from,
                         int count, bool contract, hipStream_t s) {
    switch (c.rating) {
    case KAPPA_INNER_OUTER: extend_impl<KAPPA_INNER_OUTER>(c, l, n_hint, r_from, count, s); break;
    case KAPPA_WEIGHT: extend_impl<KAPPA_WEIGHT>(c, l, n_hint, r_from, count, s); break;
    case KAPPA_EXPANSION: extend_impl<KAPPA_EXPANSION>(c, l, n_hint, r_from, count, s); break;
    case KAPPA_EXPANSION_STAR: extend_impl<KAPPA_EXPANSION_STAR>(c, l, n_hint, r_from, count, s); break;
    default: extend_impl<KAPPA_EXPANSION_STAR2>(c, l, n_hint, r_from, count, s); break;
    }
    if (!contract) return;
    launch_level_contract(c, l, n_hint, n_cap, s);
    if (c.b.count) launch_batch_end(c, l, s);
}

void launch_level_match(const Ctx &c, int l, int32_t n_hint, int64_t nnz_cap, int rounds,
                        bool stop_rules, bool out_kernels, hipStream_t s) {
    if (rounds < 1) rounds = 1;
    const bool two = c.block_bits >= 0;
    {
        KAPPA_PROF("match_init", s);
        hipLaunchKernelGGL(match_init_k, dim3(two ? 1 : grid_for(n_hint, BLOCK, 2048)), dim3(BLOCK),
                           0, s, c, l, stop_rules ? 1 : 0, two ? 0 : 1);
    }
    if (c.rating == KAPPA_INNER_OUTER && out_kernels) launch_level_out(c, l, nnz_cap, n_hint, s);
    if (two) {
        switch (c.rating) {
        case KAPPA_INNER_OUTER: two_phase_impl<KAPPA_INNER_OUTER>(c, l, n_hint, s); break;
        case KAPPA_WEIGHT: two_phase_impl<KAPPA_WEIGHT>(c, l, n_hint, s); break;
        case KAPPA_EXPANSION: two_phase_impl<KAPPA_EXPANSION>(c, l, n_hint, s); break;
        case KAPPA_EXPANSION_STAR: two_phase_impl<KAPPA_EXPANSION_STAR>(c, l, n_hint, s); break;
        default: two_phase_impl<KAPPA_EXPANSION_STAR2>(c, l, n_hint, s); break;
        }
        return;
    }
    switch (c.rating) {
    case KAPPA_INNER_OUTER: match_impl<KAPPA_INNER_OUTER>(c, l, n_hint, rounds, s); break;
    case KAPPA_WEIGHT: match_impl<KAPPA_WEIGHT>(c, l, n_hint, rounds, s); break;
    case KAPPA_EXPANSION: match_impl<KAPPA_EXPANSION>(c, l, n_hint, rounds, s); break;
    case KAPPA_EXPANSION_STAR: match_impl<KAPPA_EXPANSION_STAR>(c, l, n_hint, rounds, s); break;
    default: match_impl<KAPPA_EXPANSION_STAR2>(c, l, n_hint, rounds, s); break;
    }
}

void launch_level_contract(const Ctx &c, int l, int32_t n_hint, int32_t n_cap, hipStream_t s) {
    launch_scan((int64_t)n_hint, RepF{c, l}, RepW{c, l}, c.cs.partials, c.cs.arrive,
                c.cs.totals + 0, s);
    {
        KAPPA_PROF("fill_small", s);
        if (c.big_rows)
            hipLaunchKernelGGL(fill_small_k<true>, dim3(grid_for(n_hint, SM_ROWS * 2, 4096)),
                               dim3(BLOCK), 0, s, c, l);
        else
            hipLaunchKernelGGL(fill_small_k<false>, dim3(grid_for(n_hint, SM_ROWS * 2, 4096)),
                               dim3(BLOCK), 0, s, c, l);
    }
    {
        KAPPA_PROF("fill_mid", s);
        const unsigned wb = grid_for(n_hint, 64, 2048), mb = grid_for(n_hint, 256, 1024);
        hipLaunchKernelGGL(fill_mid_k, dim3(wb + mb), dim3(BLOCK), 0, s, c, l, wb);
    }
    if (c.big_rows) {
        KAPPA_PROF("fill_big", s);
        hipLaunchKernelGGL(fill_big_k, dim3(grid_for(n_hint, 4096, 256)), dim3(BIG_THREADS), 0, s,
                           c, l);
    }
    if (c.huge) {
        const unsigned rows = grid_for(n_hint, 4096, 512);
        {
            KAPPA_PROF("fill_huge_prep", s);
            hipLaunchKernelGGL(fill_huge_prep_k, dim3(rows), dim3(HUGE_THREADS), 0, s, c, l);
        }
        {
            KAPPA_PROF("fill_huge_small", s);
            hipLaunchKernelGGL(fill_huge_small_k, dim3(grid_for(n_hint, 256, 2048)), dim3(BLOCK), 0,
                               s, c, l);
        }
        {
            KAPPA_PROF("fill_huge_mid", s);
            hipLaunchKernelGGL(fill_huge_mid_k, dim3(grid_for(n_hint, 2048, 1024)), dim3(BLOCK), 0,
                               s, c, l);
        }
        {
            KAPPA_PROF("fill_huge_big", s);
            hipLaunchKernelGGL(fill_huge_big_k, dim3(grid_for(n_hint, 16384, 256)),
                               dim3(HUGE_THREADS), 0, s, c, l);
        }
        KAPPA_PROF("fill_huge_pack", s);
        hipLaunchKernelGGL(fill_huge_pack_k, dim3(rows), dim3(HUGE_THREADS), 0, s, c, l);
    }
    if (c.cs.hub_acc) {
        KAPPA_PROF("fill_large", s);
        hipLaunchKernelGGL(fill_large_k, dim3(c.cs.hub_slots), dim3(LARGE_THREADS), 0, s, c, l);
    }
    launch_scan((int64_t)n_hint + 1, DegF{c, l}, CoarseOffW{c, l}, c.cs.partials, c.cs.arrive,
                c.cs.totals + 2, s);
    {
        KAPPA_PROF("compact", s);
        const unsigned sb = grid_for(n_hint, SM_ROWS * 2, 4096), wb = grid_for(n_hint, 256, 1024),
                       bb = grid_for(n_hint, 1024, 512);
        hipLaunchKernelGGL(compact_k, dim3(sb + wb + bb), dim3(BLOCK), 0, s, c, l, sb, wb);
    }
    (void)n_cap;
}

void launch_tail(const Ctx &c, int l, hipStream_t s) {
    KAPPA_PROF("tail", s);
    switch (c.rating) {
    case KAPPA_INNER_OUTER: hipLaunchKernelGGL(tail_k<KAPPA_INNER_OUTER>, dim3(1), dim3(TAIL_THREADS), 0, s, c, l); break;
    case KAPPA_WEIGHT: hipLaunchKernelGGL(tail_k<KAPPA_WEIGHT>, dim3(1), dim3(TAIL_THREADS), 0, s, c, l); break;
    case KAPPA_EXPANSION: hipLaunchKernelGGL(tail_k<KAPPA_EXPANSION>, dim3(1), dim3(TAIL_THREADS), 0, s, c, l); break;
    case KAPPA_EXPANSION_STAR: hipLaunchKernelGGL(tail_k<KAPPA_EXPANSION_STAR>, dim3(1), dim3(TAIL_THREADS), 0, s, c, l); break;
    default: hipLaunchKernelGGL(tail_k<KAPPA_EXPANSION_STAR2>, dim3(1), dim3(TAIL_THREADS), 0, s, c, l); break;
    }
}

void launch_level(const Ctx &c, int l, int32_t n_hint, int64_t nnz_cap, int32_t n_cap,
                  int rounds, hipStream_t s) {
    if (c.b.count) launch_batch_begin(c, l, s);
    // Out(v) of levels above 0 is written by the previous level's compaction
    launch_level_match(c, l, n_hint, nnz_cap, rounds, true, l == 0, s);
    launch_level_contract(c, l, n_hint, n_cap, s);
    if (c.b.count) launch_batch_end(c, l, s);
}

void launch_batch_begin(const Ctx &c, int l, hipStream_t s) {
    KAPPA_PROF("batch_begin", s);
    hipLaunchKernelGGL(batch_begin_k, dim3(1), dim3(BATCH_THREADS), 0, s, c, l);
}

void launch_batch_end(const Ctx &c, int l, hipStream_t s) {
    KAPPA_PROF("batch_end", s);
    hipLaunchKernelGGL(batch_end_k, dim3(1), dim3(BATCH_THREADS), 0, s, c, l);
}

void launch_batch_gid(const int32_t *noff, int32_t count, int32_t n, int32_t *gid, hipStream_t s) {
    if (count <= 0 || n <= 0) return;
    KAPPA_PROF("batch_gid", s);
    hipLaunchKernelGGL(batch_gid_k, dim3(grid_for(n, BLOCK * 4, 4096)), dim3(BLOCK), 0, s, noff,
                       count, n, gid);
}

void launch_batch_extract(const DevGraph &u, const int32_t *cmap, const int32_t *mate, int32_t a,
                          int32_t b, int64_t ea, int64_t nnz, int32_t cbase, int64_t *xadj,
                          int32_t *adj, uint32_t *ew, uint32_t *vw, int32_t *cmap_out,
                          int32_t *mate_out, hipStream_t s) {
    KAPPA_PROF("batch_extract", s);
    hipLaunchKernelGGL(batch_extract_k, dim3(grid_for(std::max<int64_t>(nnz, b - a + 1), BLOCK, 4096)),
                       dim3(BLOCK), 0, s, u, cmap, mate, a, b, ea, cbase, xadj, adj, ew, vw,
                       cmap_out, mate_out);
}

void launch_batch_check(const DevGraph &g, uint32_t *flags, hipStream_t s) {
    if (g.n <= 0) return;
    KAPPA_PROF("batch_check", s);
    hipLaunchKernelGGL(batch_check_k, dim3(grid_for(g.n, BLOCK, 4096)), dim3(BLOCK), 0, s, g,
                       flags);
}

}  // namespace kappa
