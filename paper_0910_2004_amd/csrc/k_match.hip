// k_match.hip -- parallel locally-heaviest-edge matching (Section 3.3).
//
// Rounds as in the paper's parallel scheme: every free node that still has a
// free neighbour points at its best edge to a free neighbour (the strict order
// of kappa.h); edges that are best at both ends are matched; repeat until no
// free node has a free neighbour.  Under a strict total order this yields
// exactly the Greedy matching of Section 3.2.
//
// GPU layout of a round:
//   pick kernel  -- node-centric argmax over the row, nodes binned by degree:
//                   bin 0 (deg <= 16) 8 lanes per node, bin 1 (deg <= 1024)
//                   one wave per node, bin 2 one block per node.  A pending
//                   node whose previous choice is still free keeps it (free
//                   sets only shrink, so it is still the maximum).
//   mate kernel  -- mutual check best[best[v]] == v, matched pairs written,
//                   survivors appended (wave-aggregated) to the next round's
//                   lists, per-round statistics.
// Once at most TAIL_MAX nodes remain, one 1024-thread workgroup runs all
// remaining rounds with workgroup barriers instead of kernel launches.
// Round control is device-resident (MatchState), so the host launches a batch
// of rounds without reading counts back; kernels of rounds that are no longer
// needed return at once.
#include "kappa_internal.h"

namespace kappa {

__device__ __forceinline__ int bin_of(int64_t deg) {
    return deg <= BIN_SMALL_MAX ? 0 : (deg <= BIN_MID_MAX ? 1 : 2);
}

__device__ __forceinline__ int32_t *list_ptr(int32_t *lists, int32_t n, int par, int bin) {
    return lists + ((int64_t)(par * 3 + bin)) * n;
}

// Best candidate of v over entries sub, sub+G, ... of its row (per-lane part).
template <int R, int G>
__device__ __forceinline__ Cand scan_row(const DevGraph &g, int32_t v, int sub,
                                         const int32_t *mate, const uint32_t *out,
                                         uint64_t seed, bool first) {
    Cand best = cand_none();
    int64_t b = g.xadj[v], e = g.xadj[v + 1];
    uint32_t cv = g.vw[v];
    uint32_t ov = (R == KAPPA_INNER_OUTER) ? out[v] : 0u;
    for (int64_t j = b + sub; j < e; j += G) {
        int32_t u = g.adj[j];
        if (!first && mate[u] >= 0) continue;
        Cand c;
        rate<R>(g.ew[j], g.vw[u], cv, (R == KAPPA_INNER_OUTER) ? out[u] : 0u, ov, c.num, c.den);
        c.h = mix64(seed ^ edge_id(v, u));
        c.u = u;
        if (cand_better(c, best, v)) best = c;
    }
    return best;
}

template <int G>
__device__ __forceinline__ Cand group_reduce(Cand c, int32_t v) {
    for (int off = G / 2; off > 0; off >>= 1) {
        Cand o = cand_shfl_xor(c, off, G);
        if (cand_better(o, c, v)) c = o;
    }
    return c;
}

// Whole-block argmax (all threads call; contains barriers).
__device__ __forceinline__ Cand block_reduce_cand(Cand c, int32_t v, Cand *sh) {
    c = group_reduce<WAVE>(c, v);
    int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    if (lane_id() == 0) sh[w] = c;
    __syncthreads();
    Cand r = sh[0];
    for (int i = 1; i < nw; ++i)
        if (cand_better(sh[i], r, v)) r = sh[i];
    __syncthreads();
    return r;
}

// A pending node keeps its choice while that neighbour is still free.
__device__ __forceinline__ bool needs_rescan(int32_t v, const int32_t *best, const int32_t *mate,
                                             bool first) {
    if (first) return true;
    int32_t b = best[v];
    return !(b >= 0 && mate[b] < 0);
}

// ---------------------------------------------------------------------------
// Level start
// ---------------------------------------------------------------------------
__global__ void match_state_reset_k(MatchState *st) {
    int t = threadIdx.x;
    if (t < 16) st->cnt[t >> 2][t & 3] = 0;
    if (t == 0) {
        st->handoff = -1;
        st->rounds = 0;
        st->matched = 0;
    }
    for (int i = t; i < MAX_ROUND_STATS; i += blockDim.x) {
        st->stat[i][0] = 0;
        st->stat[i][1] = 0;
    }
}

// mate = best = -1; nodes of bins 1 and 2 go to the round-1 lists (parity 0).
__global__ void __launch_bounds__(BLOCK) match_init_k(DevGraph g, int32_t *mate, int32_t *best,
                                                      int32_t *lists, MatchState *st) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // wave-uniform loop: wb is the first node of this wave's batch
    int64_t wb0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1));
    for (int64_t wb = wb0; wb < g.n; wb += stride) {
        int64_t v = wb + lane_id();
        bool live = v < g.n;
        int64_t deg = 0;
        if (live) {
            mate[v] = -1;
            best[v] = -1;
            deg = g.xadj[v + 1] - g.xadj[v];
        }
        int bn = live ? bin_of(deg) : 0;
        wave_append(live && bn == 1, (int32_t)v, list_ptr(lists, g.n, 0, 1), &st->cnt[0][1]);
        wave_append(live && bn == 2, (int32_t)v, list_ptr(lists, g.n, 0, 2), &st->cnt[0][2]);
    }
}

void launch_max_degree(const DevGraph &g, int32_t *out, hipStream_t s);

// ---------------------------------------------------------------------------
// Pick kernel of round r
// ---------------------------------------------------------------------------
struct PickGrid {
    unsigned b0, b1, b2;  // blocks per bin
};

template <int R>
__global__ void __launch_bounds__(BLOCK) pick_k(DevGraph g, int r, uint64_t seed, PickGrid pg,
                                                const int32_t *mate, int32_t *best,
                                                int32_t *lists, const uint32_t *out,
                                                MatchState *st) {
    __shared__ Cand sh[BLOCK / WAVE];
    if (st->handoff != -1) return;
    const bool first = r == 1;
    int32_t c[3];
    const int32_t *L[3];
    if (first) {
        c[0] = g.n; c[1] = st->cnt[0][1]; c[2] = st->cnt[0][2];
        L[0] = nullptr; L[1] = list_ptr(lists, g.n, 0, 1); L[2] = list_ptr(lists, g.n, 0, 2);
    } else {
        int slot = (r - 1) & 3, par = (r - 1) & 1;
        c[0] = st->cnt[slot][0]; c[1] = st->cnt[slot][1]; c[2] = st->cnt[slot][2];
        int64_t total = (int64_t)c[0] + c[1] + c[2];
        if (total == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&st->handoff, -1, -2);
            return;
        }
        if (total <= TAIL_MAX) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&st->handoff, -1, r - 1);
            return;
        }
        L[0] = list_ptr(lists, g.n, par, 0);
        L[1] = list_ptr(lists, g.n, par, 1);
        L[2] = list_ptr(lists, g.n, par, 2);
    }
    unsigned bid = blockIdx.x;
    if (bid < pg.b0) {
        // bin 0: 8 lanes per node, 32 nodes per block-iteration
        const int G = SMALL_G;
        int sub = threadIdx.x & (G - 1);
        int64_t gi = (int64_t)bid * (BLOCK / G) + threadIdx.x / G;
        int64_t gs = (int64_t)pg.b0 * (BLOCK / G);
        int64_t lim = ((int64_t)c[0] + gs - 1) / gs * gs;   // uniform trip count
        for (int64_t i = gi; i < lim; i += gs) {
            bool live = i < c[0];
            int32_t v = -1;
            bool act = false;
            if (live) {
                v = first ? (int32_t)i : L[0][i];
                if (first) {
                    int64_t d = g.xadj[v + 1] - g.xadj[v];
                    act = d >= 1 && d <= BIN_SMALL_MAX;
                } else {
                    act = needs_rescan(v, best, mate, false);
                }
            }
            Cand cd = act ? scan_row<R, G>(g, v, sub, mate, out, seed, first) : cand_none();
            cd = group_reduce<G>(cd, v);
            if (act && sub == 0) best[v] = cd.u;
        }
        return;
    }
    bid -= pg.b0;
    if (bid < pg.b1) {
        // bin 1: one wave per node
        int64_t gi = (int64_t)bid * (BLOCK / WAVE) + threadIdx.x / WAVE;
        int64_t gs = (int64_t)pg.b1 * (BLOCK / WAVE);
        for (int64_t i = gi; i < c[1]; i += gs) {
            int32_t v = L[1][i];
            if (!needs_rescan(v, best, mate, first)) continue;   // wave-uniform
            Cand cd = scan_row<R, WAVE>(g, v, lane_id(), mate, out, seed, first);
            cd = group_reduce<WAVE>(cd, v);
            if (lane_id() == 0) best[v] = cd.u;
        }
        return;
    }
    bid -= pg.b1;
    // bin 2: one block per node
    for (int64_t i = bid; i < c[2]; i += pg.b2) {
        int32_t v = L[2][i];
        if (!needs_rescan(v, best, mate, first)) continue;       // block-uniform
        Cand cd = scan_row<R, BLOCK>(g, v, threadIdx.x, mate, out, seed, first);
        cd = block_reduce_cand(cd, v, sh);
        if (threadIdx.x == 0) best[v] = cd.u;
    }
}

// ---------------------------------------------------------------------------
// Mate kernel of round r: mutual check, survivors to the next lists.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) mate_k(DevGraph g, int r, int32_t *mate,
                                                const int32_t *best, int32_t *lists,
                                                MatchState *st) {
    __shared__ int64_t sh[BLOCK / WAVE + 1];
    if (st->handoff != -1) return;
    const bool first = r == 1;
    int32_t c[3];
    const int32_t *L[3] = {nullptr, nullptr, nullptr};
    int64_t total;
    if (first) {
        total = g.n;
        c[0] = g.n; c[1] = 0; c[2] = 0;
    } else {
        int slot = (r - 1) & 3, par = (r - 1) & 1;
        c[0] = st->cnt[slot][0]; c[1] = st->cnt[slot][1]; c[2] = st->cnt[slot][2];
        total = (int64_t)c[0] + c[1] + c[2];
        L[0] = list_ptr(lists, g.n, par, 0);
        L[1] = list_ptr(lists, g.n, par, 1);
        L[2] = list_ptr(lists, g.n, par, 2);
    }
    int opar = r & 1, oslot = r & 3;
    if (blockIdx.x == 0 && threadIdx.x < 3) st->cnt[(r + 2) & 3][threadIdx.x] = 0;
    int32_t *O0 = list_ptr(lists, g.n, opar, 0);
    int32_t *O1 = list_ptr(lists, g.n, opar, 1);
    int32_t *O2 = list_ptr(lists, g.n, opar, 2);
    int64_t point = 0, degs = 0, pairs = 0;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t wb0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1));
    for (int64_t wb = wb0; wb < total; wb += stride) {
        int64_t i = wb + lane_id();
        bool keep = false;
        int bn = 0;
        int32_t v = -1;
        if (i < total) {
            if (first) v = (int32_t)i;
            else if (i < c[0]) v = L[0][i];
            else if (i < (int64_t)c[0] + c[1]) v = L[1][i - c[0]];
            else v = L[2][i - c[0] - c[1]];
            int32_t b = best[v];
            if (b >= 0) {
                int64_t d = g.xadj[v + 1] - g.xadj[v];
                ++point;
                degs += d;
                if (best[b] == v) {
                    mate[v] = b;
                    if (v < b) ++pairs;
                } else {
                    keep = true;
                    bn = bin_of(d);
                }
            }
        }
        wave_append(keep && bn == 0, v, O0, &st->cnt[oslot][0]);
        wave_append(keep && bn == 1, v, O1, &st->cnt[oslot][1]);
        wave_append(keep && bn == 2, v, O2, &st->cnt[oslot][2]);
    }
    point = block_sum(point, sh);
    degs = block_sum(degs, sh);
    pairs = block_sum(pairs, sh);
    if (threadIdx.x == 0 && point > 0) {
        int ri = r - 1 < MAX_ROUND_STATS ? r - 1 : MAX_ROUND_STATS - 1;
        atomicAdd((unsigned long long *)&st->stat[ri][0], (unsigned long long)point);
        atomicAdd((unsigned long long *)&st->stat[ri][1], (unsigned long long)degs);
        if (pairs) atomicAdd((unsigned long long *)&st->matched, (unsigned long long)pairs);
        atomicMax(&st->rounds, r);
    }
}

// ---------------------------------------------------------------------------
// Finisher: one workgroup runs the remaining rounds.
// ---------------------------------------------------------------------------
template <int R>
__global__ void __launch_bounds__(FINISH_THREADS) finish_k(DevGraph g, uint64_t seed, int r_last,
                                                           int32_t *mate, int32_t *best,
                                                           int32_t *lists, const uint32_t *out,
                                                           MatchState *st) {
    __shared__ Cand shc[FINISH_THREADS / WAVE];
    __shared__ int32_t s_cnt[2][3];
    __shared__ int64_t s_acc[3];   // pointing, degsum, pairs of the current round
    __shared__ int32_t s_r0;
    if (threadIdx.x == 0) {
        int h = st->handoff;
        if (h == -1) {
            // every round up to r_last ran: take over if few nodes are left
            int slot = r_last & 3;
            int64_t total = (int64_t)st->cnt[slot][0] + st->cnt[slot][1] + st->cnt[slot][2];
            if (total <= TAIL_MAX) h = r_last;
        }
        s_r0 = h;
    }
    __syncthreads();
    int r0 = s_r0;
    if (r0 < 0) return;   // more multi-block rounds needed, or already done
    if (threadIdx.x < 3) {
        s_cnt[r0 & 1][threadIdx.x] = st->cnt[r0 & 3][threadIdx.x];
        s_cnt[(r0 + 1) & 1][threadIdx.x] = 0;
    }
    __syncthreads();
    int64_t pairs_total = 0;
    // Every round that has a pointing node matches at least one pair, so at
    // most n/2 + 1 rounds remain; the cap only guards against a broken state.
    const int64_t r_cap = (int64_t)r0 + 2 + g.n;
    bool capped = true;
    for (int r = r0 + 1; r <= r_cap; ++r) {
        int ip = (r - 1) & 1, op = r & 1;
        int32_t c0 = s_cnt[ip][0], c1 = s_cnt[ip][1], c2 = s_cnt[ip][2];
        if ((int64_t)c0 + c1 + c2 == 0) { capped = false; break; }
        const int32_t *L0 = list_ptr(lists, g.n, ip, 0);
        const int32_t *L1 = list_ptr(lists, g.n, ip, 1);
        const int32_t *L2 = list_ptr(lists, g.n, ip, 2);
        // --- pick ---
        {
            const int G = SMALL_G;
            int sub = threadIdx.x & (G - 1);
            int gi = threadIdx.x / G, gs = FINISH_THREADS / G;
            int lim = (c0 + gs - 1) / gs * gs;
            for (int i = gi; i < lim; i += gs) {
                int32_t v = i < c0 ? L0[i] : -1;
                bool act = v >= 0 && needs_rescan(v, best, mate, false);
                Cand cd = act ? scan_row<R, G>(g, v, sub, mate, out, seed, false) : cand_none();
                cd = group_reduce<G>(cd, v);
                if (act && sub == 0) best[v] = cd.u;
            }
            int wi = threadIdx.x / WAVE, ws = FINISH_THREADS / WAVE;
            for (int i = wi; i < c1; i += ws) {
                int32_t v = L1[i];
                if (!needs_rescan(v, best, mate, false)) continue;
                Cand cd = scan_row<R, WAVE>(g, v, lane_id(), mate, out, seed, false);
                cd = group_reduce<WAVE>(cd, v);
                if (lane_id() == 0) best[v] = cd.u;
            }
        }
        __syncthreads();
        for (int i = 0; i < c2; ++i) {
            int32_t v = L2[i];
            if (!needs_rescan(v, best, mate, false)) continue;   // block-uniform
            Cand cd = scan_row<R, FINISH_THREADS>(g, v, threadIdx.x, mate, out, seed, false);
            cd = block_reduce_cand(cd, v, shc);
            if (threadIdx.x == 0) best[v] = cd.u;
        }
        if (threadIdx.x < 3) { s_acc[threadIdx.x] = 0; s_cnt[op][threadIdx.x] = 0; }
        __syncthreads();
        // --- mate ---
        int32_t total = c0 + c1 + c2;
        int64_t point = 0, degs = 0, pairs = 0;
        int lim = (total + FINISH_THREADS - 1) / FINISH_THREADS * FINISH_THREADS;
        for (int i = threadIdx.x; i < lim; i += FINISH_THREADS) {
            bool keep = false;
            int bn = 0;
            int32_t v = -1;
            if (i < total) {
                v = i < c0 ? L0[i] : (i < c0 + c1 ? L1[i - c0] : L2[i - c0 - c1]);
                int32_t b = best[v];
                if (b >= 0) {
                    int64_t d = g.xadj[v + 1] - g.xadj[v];
                    ++point;
                    degs += d;
                    if (best[b] == v) {
                        mate[v] = b;
                        if (v < b) ++pairs;
                    } else {
                        keep = true;
                        bn = bin_of(d);
                    }
                }
            }
            wave_append(keep && bn == 0, v, list_ptr(lists, g.n, op, 0), &s_cnt[op][0]);
            wave_append(keep && bn == 1, v, list_ptr(lists, g.n, op, 1), &s_cnt[op][1]);
            wave_append(keep && bn == 2, v, list_ptr(lists, g.n, op, 2), &s_cnt[op][2]);
        }
        point = wave_sum(point);
        degs = wave_sum(degs);
        pairs = wave_sum(pairs);
        if (lane_id() == 0) {
            if (point) atomicAdd((unsigned long long *)&s_acc[0], (unsigned long long)point);
            if (degs) atomicAdd((unsigned long long *)&s_acc[1], (unsigned long long)degs);
            if (pairs) atomicAdd((unsigned long long *)&s_acc[2], (unsigned long long)pairs);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_acc[0] > 0) {
                int ri = r - 1 < MAX_ROUND_STATS ? r - 1 : MAX_ROUND_STATS - 1;
                st->stat[ri][0] += s_acc[0];
                st->stat[ri][1] += s_acc[1];
                st->rounds = r;
            }
            pairs_total += s_acc[2];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->matched += pairs_total;
        st->handoff = capped ? -3 : -2;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) max_degree_k(DevGraph g, int32_t *out) {
    int32_t m = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = g.xadj[v + 1] - g.xadj[v];
        m = d > m ? (int32_t)d : m;
    }
    m = wave_max(m);
    if (lane_id() == 0 && m) atomicMax(out, m);
}

void launch_max_degree(const DevGraph &g, int32_t *out, hipStream_t s) {
    if (g.n <= 0) return;
    KAPPA_PROF("max_degree", s);
    hipLaunchKernelGGL(max_degree_k, dim3(grid_for(g.n, BLOCK, 2048)), dim3(BLOCK), 0, s, g, out);
}

void launch_match_begin(const DevGraph &g, int rating, int32_t *mate, MatchScratch &ms,
                        hipStream_t s) {
    if (rating == KAPPA_INNER_OUTER) launch_out(g, ms.tile_row, ms.out, s);
    {
        KAPPA_PROF("match_reset", s);
        hipLaunchKernelGGL(match_state_reset_k, dim3(1), dim3(BLOCK), 0, s, ms.state);
    }
    if (g.n <= 0) return;
    KAPPA_PROF("match_init", s);
    hipLaunchKernelGGL(match_init_k, dim3(grid_for(g.n, BLOCK, 2048)), dim3(BLOCK), 0, s, g, mate,
                       ms.best, ms.lists, ms.state);
}

template <int R>
static void rounds_impl(const DevGraph &g, uint64_t seed, int32_t maxdeg, int32_t *mate,
                        MatchScratch &ms, int r_first, int count, hipStream_t s) {
    PickGrid pg;
    pg.b0 = grid_for(g.n, BLOCK / SMALL_G, 2048);
    pg.b1 = maxdeg > BIN_SMALL_MAX ? grid_for(g.n, BLOCK / WAVE, 512) : 0;
    pg.b2 = maxdeg > BIN_MID_MAX ? grid_for(g.n, 1, 256) : 0;
    unsigned pick_blocks = pg.b0 + pg.b1 + pg.b2;
    unsigned mate_blocks = grid_for(g.n, BLOCK, 2048);
    for (int r = r_first; r < r_first + count; ++r) {
        {
            KAPPA_PROF(r == 1 ? "pick_first" : "pick", s);
            hipLaunchKernelGGL(pick_k<R>, dim3(pick_blocks), dim3(BLOCK), 0, s, g, r, seed, pg,
                               mate, ms.best, ms.lists, ms.out, ms.state);
        }
        {
            KAPPA_PROF(r == 1 ? "mate_first" : "mate", s);
            hipLaunchKernelGGL(mate_k, dim3(mate_blocks), dim3(BLOCK), 0, s, g, r, mate, ms.best,
                               ms.lists, ms.state);
        }
    }
    KAPPA_PROF("match_finish", s);
    hipLaunchKernelGGL(finish_k<R>, dim3(1), dim3(FINISH_THREADS), 0, s, g, seed,
                       r_first + count - 1, mate, ms.best, ms.lists, ms.out, ms.state);
}

void launch_match_rounds(const DevGraph &g, int rating, uint64_t seed, int32_t maxdeg,
                         int32_t *mate, MatchScratch &ms, int r_first, int count, hipStream_t s) {
    if (g.n <= 0) return;
    switch (rating) {
    case KAPPA_INNER_OUTER: rounds_impl<KAPPA_INNER_OUTER>(g, seed, maxdeg, mate, ms, r_first, count, s); break;
    case KAPPA_WEIGHT: rounds_impl<KAPPA_WEIGHT>(g, seed, maxdeg, mate, ms, r_first, count, s); break;
    case KAPPA_EXPANSION: rounds_impl<KAPPA_EXPANSION>(g, seed, maxdeg, mate, ms, r_first, count, s); break;
    case KAPPA_EXPANSION_STAR: rounds_impl<KAPPA_EXPANSION_STAR>(g, seed, maxdeg, mate, ms, r_first, count, s); break;
    default: rounds_impl<KAPPA_EXPANSION_STAR2>(g, seed, maxdeg, mate, ms, r_first, count, s); break;
    }
}

}  // namespace kappa
