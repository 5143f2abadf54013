// kappa_internal.h -- device helpers and launch-wrapper declarations shared by
// the library's translation units.  gfx950 only (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kappa.h"

namespace kappa {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;          // threads per block of the sweep kernels
constexpr int SCAN_ITEMS = 8;       // items per thread in the scan tiles
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;

// Degree classes of the node-centric kernels.
constexpr int BIN_SMALL_MAX = 16;   // deg <= 16: SMALL_G lanes per node
constexpr int BIN_MID_MAX = 1024;   // deg <= 1024: one wave per node; above: one block
constexpr int SMALL_G = 4;

// Matching rounds: a single workgroup finishes once at most TAIL_MAX nodes
// still point somewhere.
constexpr int TAIL_MAX = 128;
// The finisher takes a level whose launched grid rounds ran out only while at
// most FINISH_MAX nodes (and FINISH_MAX_BIG of degree above BIN_MID_MAX) are
// pending; otherwise it hands the level back for more grid rounds.
constexpr int FINISH_MAX = 4096;
constexpr int FINISH_MAX_BIG = 64;
constexpr int EXTEND_ROUNDS = 8;   // doubled on every further hand-back of a level, up to 64
constexpr int BM_BITS_MAX = 11;     // two-phase matcher: blocks of at most 2^11 nodes
constexpr int BM_THREADS = 512;     //   matched by one workgroup each
constexpr int FINISH_THREADS = 1024;
// Levels of at most TAIL_MAX_N nodes and TAIL_MAX_NNZ entries (and every
// level after them) run in one workgroup of TAIL_THREADS threads.
constexpr int TAIL_THREADS = 1024;
constexpr int32_t TAIL_MAX_N = 16384;
constexpr int64_t TAIL_MAX_NNZ = 131072;
constexpr int STAT_ROUNDS = 64;     // per-round statistics kept per level (last slot aggregates)
constexpr int MAX_LEVELS = 256;

// Row classes of the contraction (bound = deg(u) + deg(v) - 2 for a pair).
constexpr int ROW_SMALL_MAX = 64;   // 16 lanes per row, rank sort in LDS
constexpr int ROW_SMALL_G = 16;
constexpr int ROW_WAVE_MAX = 512;   // one wave per row, bitonic sort of <= 512 in LDS
constexpr int ROW_MID_MAX = 4094;   // one block per row, bitonic sort of <= 4096 in LDS
constexpr int ROW_BIG_MAX = 16382;  // one 1024-thread block per row, sort of <= 16384 in LDS
// Rows above ROW_BIG_MAX (large rows) are merged by key buckets when the
// next level has at most HUGE_NC_MAX nodes and the row at most HUGE_ROW_MAX
// entries; the others by dense hub accumulators, which only graphs of more
// than HUGE_NC_MAX nodes allocate.  Rows of ROW_MID_MAX+1..ROW_BIG_MAX
// entries take the key buckets too where those apply; the big-row block
// sort only otherwise.
constexpr int HG_BINS = 4096;                       // key buckets of a row
constexpr int HG_WINS = 2048;                       // groups per row at most
constexpr int HG_WIN_MIN = 256;                     // positions per group window (at least)
constexpr int64_t HUGE_NC_MAX = (int64_t)HG_BINS << 11;   // buckets of at most 2^11 keys
constexpr int64_t HUGE_ROW_MAX = (int64_t)HG_WINS * 8192;
constexpr int HUB_SLOTS = 32;       // rows above ROW_MID_MAX: dense accumulators (at least)
constexpr int HUB_SLOTS_MAX = 256;  //   and at most, within HUB_BUDGET bytes of accumulators
constexpr int64_t HUB_BUDGET = (int64_t)4 << 30;

// The tunable thresholds (kappa_tuning), copied into every launch context.
// Compile-time sizes bound them: bin_small_max <= BIN_SMALL_MAX and
// row_small_max <= ROW_SMALL_MAX (register and LDS arrays).
struct Tune {
    int32_t bin_small_max = BIN_SMALL_MAX;
    int32_t tail_max = TAIL_MAX;
    int32_t finish_max = FINISH_MAX;
    int32_t finish_max_big = FINISH_MAX_BIG;
    int32_t row_small_max = ROW_SMALL_MAX;
    int32_t scan_one_block_max = 16384;
    int32_t rounds_base = 3, rounds_n0 = 2048, rounds_growth = 8, rounds_cap = 8;
};
Tune tuning_now();   // the library's current table (host)

// Device-scope atomics on one address from many blocks serialise where the
// XCDs meet (about 10 ns each), so kernel-wide accumulators are split over
// NSHARD slots picked by block index and summed by their consumer, and
// "last block" detection counts arrivals in groups of ARRIVE_GROUP blocks.
constexpr int NSHARD = 64;
constexpr int ARRIVE_GROUP = 32;
constexpr int ARRIVE_MAX_BLOCKS = 4096;   // grids that use arrival counters stay below
constexpr int ARRIVE_WORDS = 1 + ARRIVE_MAX_BLOCKS / ARRIVE_GROUP;

struct DevGraph {
    int32_t n;
    int64_t nnz;
    const int64_t *xadj;
    const int32_t *adj;
    const uint32_t *ew;
    const uint32_t *vw;
    // batched form (a disjoint union of graphs; null for a single graph):
    // graph of each node, first node of each graph at this level
    const int32_t *gid = nullptr;
    const int32_t *noff = nullptr;
};

// First node of v's graph: tie hashes use graph-local ids, so a graph's
// hierarchy is the same alone and inside a batch.
__device__ __forceinline__ int32_t local_base(const DevGraph &g, int32_t v) {
    return g.gid ? g.noff[g.gid[v]] : 0;
}

// ---------------------------------------------------------------------------
// SplitMix64 output function (Steele, Lea, Flood 2014), the tie-break hash.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t edge_id(int32_t a, int32_t b) {
    uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((uint64_t)lo << 32) | hi;
}

// The same with ids relative to `base` (the first node of the edge's graph).
__host__ __device__ inline uint64_t edge_id_local(int32_t a, int32_t b, int32_t base) {
    return edge_id(a - base, b - base);
}

// ---------------------------------------------------------------------------
// Ratings (Section 3.1) as exact rationals.  Out() is only read by innerOuter.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void rate(uint32_t w, uint32_t cu, uint32_t cv, uint32_t ou,
                                     uint32_t ov, uint64_t &num, uint64_t &den) {
    if (R == KAPPA_WEIGHT) { num = w; den = 1; }
    else if (R == KAPPA_EXPANSION) { num = w; den = (uint64_t)cu + cv; }
    else if (R == KAPPA_EXPANSION_STAR) { num = w; den = (uint64_t)cu * cv; }
    else if (R == KAPPA_INNER_OUTER) { num = w; den = (uint64_t)ou + ov - 2ull * w; }
    else { num = (uint64_t)w * w; den = (uint64_t)cu * cv; }
}

// A candidate edge {v, u} seen from v.  u < 0 means "none".
struct Cand {
    uint64_t num, den, h;
    int32_t u;
};

__device__ __forceinline__ Cand cand_none() {
    Cand c;
    c.num = 0; c.den = 1; c.h = 0; c.u = -1;
    return c;
}

// a above b in the strict order (both incident to v).  Rational part by
// 128-bit cross products num_a*den_b vs num_b*den_a, then hash, then the
// smaller edge id.
__device__ __forceinline__ bool cand_better(const Cand &a, const Cand &b, int32_t v) {
    if (a.u < 0) return false;
    if (b.u < 0) return true;
    if (((a.num | a.den | b.num | b.den) >> 32) == 0) {
        // all four below 2^32: the cross products fit 64 bits
        const uint64_t l = a.num * b.den, r = b.num * a.den;
        if (l != r) return l > r;
    } else {
        uint64_t l_lo = a.num * b.den, l_hi = __umul64hi(a.num, b.den);
        uint64_t r_lo = b.num * a.den, r_hi = __umul64hi(b.num, a.den);
        if (l_hi != r_hi) return l_hi > r_hi;
        if (l_lo != r_lo) return l_lo > r_lo;
    }
    if (a.h != b.h) return a.h > b.h;
    return edge_id(v, a.u) < edge_id(v, b.u);
}

__device__ __forceinline__ Cand cand_shfl_xor(const Cand &c, int mask, int width) {
    Cand o;
    o.num = __shfl_xor(c.num, mask, width);
    o.den = __shfl_xor(c.den, mask, width);
    o.h = __shfl_xor(c.h, mask, width);
    o.u = __shfl_xor(c.u, mask, width);
    return o;
}

// ---------------------------------------------------------------------------
// Wave / block primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : ((~0ull) >> (64 - l));
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, WAVE);
        v = o > v ? o : v;
    }
    return v;
}

// Inclusive scan over the wave.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    int l = lane_id();
    for (int off = 1; off < WAVE; off <<= 1) {
        T o = __shfl_up(v, off, WAVE);
        if (l >= off) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024).
// `sh` must hold blockDim.x / WAVE + 1 entries.  Returns the exclusive prefix;
// *total receives the block sum.  Contains __syncthreads.
template <class T>
__device__ T block_excl_scan(T v, T *sh, T *total) {
    int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    T inc = wave_incl_scan(v);
    if (lane_id() == WAVE - 1) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < nw; ++i) { T t = sh[i]; sh[i] = run; run += t; }
        sh[nw] = run;
    }
    __syncthreads();
    T res = sh[w] + inc - v;
    *total = sh[nw];
    __syncthreads();
    return res;
}

// Appends val to list where pred holds, one atomic per wave.  All 64 lanes
// must call it (wave-uniform control flow).  Order inside the list is not
// deterministic; no consumer depends on it.
__device__ __forceinline__ void wave_append(bool pred, int32_t val, int32_t *list,
                                            int32_t *counter) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (int)__popcll(mask));
    base = __shfl(base, leader, WAVE);
    if (pred) list[base + __popcll(mask & lanemask_lt())] = val;
}

__device__ __forceinline__ int shard_of_block() { return (int)(blockIdx.x & (NSHARD - 1)); }

// Called by thread 0 of every block of a grid (<= ARRIVE_MAX_BLOCKS blocks)
// after its global writes; returns true in exactly one block, the last to
// arrive, which then sees every other block's writes.  `cnt` holds
// ARRIVE_WORDS zeroed words and is zero again when the grid ends.
// Arrivals only release: an agent-scope release waits for the block's
// writes (ordered before by a block barrier) and writes the XCD's L2 back to
// memory before the counter moves, so once every arrival has counted, every
// block's data is in memory.  The one acquire (it invalidates the XCD's L2,
// which would evict every other block's gathered lines) is taken by the last
// block alone, before it reads the others' data.
__device__ __forceinline__ bool arrive_last(unsigned *cnt) {
    const unsigned nb = gridDim.x, g = blockIdx.x / ARRIVE_GROUP;
    const unsigned ng = (nb + ARRIVE_GROUP - 1) / ARRIVE_GROUP;
    const unsigned gsize = g + 1 < ng ? ARRIVE_GROUP : nb - g * ARRIVE_GROUP;
    unsigned old = __hip_atomic_fetch_add(&cnt[1 + g], 1u, __ATOMIC_RELEASE,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if (old != gsize - 1) return false;
    __hip_atomic_store(&cnt[1 + g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = __hip_atomic_fetch_add(&cnt[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (old != ng - 1) return false;
    __hip_atomic_store(&cnt[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Block sums of K per-thread values, valid in thread 0 (two barriers).
// sh: K * (blockDim.x / WAVE) entries.
template <int K>
__device__ __forceinline__ void block_sum_n(int64_t (&v)[K], int64_t *sh) {
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = wave_sum(v[q]);
    const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    __syncthreads();   // sh may still be read by a previous use
    if (lane_id() == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) sh[q * nw + w] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            v[q] = 0;
            for (int i = 0; i < nw; ++i) v[q] += sh[q * nw + i];
        }
    }
}

// Block sums of three per-thread values, valid in thread 0 (two barriers).
// sh: 3 * (blockDim.x / WAVE) entries.
__device__ __forceinline__ void block_sum3(int64_t &a, int64_t &b, int64_t &c, int64_t *sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    __syncthreads();   // sh may still be read by a previous use
    if (lane_id() == 0) {
        sh[w] = a;
        sh[nw + w] = b;
        sh[2 * nw + w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = c = 0;
        for (int i = 0; i < nw; ++i) {
            a += sh[i];
            b += sh[nw + i];
            c += sh[2 * nw + i];
        }
    }
}

template <class T>
__device__ T block_sum(T v, T *sh) {
    T t;
    block_excl_scan(v, sh, &t);
    return t;
}

// Block-aggregated append into one of up to three lists (bin < 0: none).
// One global atomic per list per call.  Every thread of the block must call
// it (block-uniform control flow).  `sh` needs 3 * (blockDim.x / WAVE) + 3
// int32 of shared memory.  Order inside a list is not deterministic; no
// consumer depends on it.
__device__ __forceinline__ void block_append3(int bin, int32_t val, int32_t *const lists[3],
                                              int32_t *const counters[3], int32_t *sh) {
    const int nw = blockDim.x / WAVE, w = threadIdx.x / WAVE;
    uint64_t m[3];
    for (int b = 0; b < 3; ++b) {
        m[b] = __ballot(bin == b);
        if (lane_id() == 0) sh[b * nw + w] = (int32_t)__popcll(m[b]);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int b = threadIdx.x, run = 0;
        for (int i = 0; i < nw; ++i) { int t = sh[b * nw + i]; sh[b * nw + i] = run; run += t; }
        sh[3 * nw + b] = run ? atomicAdd(counters[b], run) : 0;
    }
    __syncthreads();
    if (bin >= 0) {
        uint64_t mb = bin == 0 ? m[0] : (bin == 1 ? m[1] : m[2]);
        int pos = sh[3 * nw + bin] + sh[bin * nw + w] + (int)__popcll(mb & lanemask_lt());
        lists[bin][pos] = val;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Generic exclusive scan with a device-side length, two kernels.
// F: size() -> int64 (< 0: skip the whole scan), operator()(i) -> int64
// value, post(total) run by one thread once the total is known (before the
// apply kernel starts).  W: bind() -> B, called after post(), holding the
// output pointers; B::prefetch(i, value) -> B::Pre loads what the store
// needs; B::operator()(i, prefix, value, pre) stores.  A thread prefetches
// all of its items before it stores any, so their loads overlap.
//   reduce: tile sums; the last block to finish scans the tile sums in place,
//           writes the total and runs post()
//   apply:  rescan of each tile from its tile prefix
// Grids are hints (at most ARRIVE_MAX_BLOCKS); loops stride over the live
// tile count.  `ws` holds the tile sums (scan_tiles(cap) + 1 int64); `arr`
// the arrival counters (ARRIVE_WORDS, zero between uses).
// ---------------------------------------------------------------------------
template <class F>
__global__ void __launch_bounds__(BLOCK) scan_reduce_k(F f, int64_t *ws, unsigned *arr,
                                                       int64_t *total) {
    __shared__ int64_t sh[BLOCK / WAVE + 1];
    __shared__ int last;
    const int64_t n = f.size();
    if (n < 0) return;
    int64_t *partials = ws;
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        int64_t base = t * SCAN_TILE, s = 0;
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            int64_t idx = base + (int64_t)i * BLOCK + threadIdx.x;
            if (idx < n) s += f(idx);
        }
        s = block_sum(s, sh);
        if (threadIdx.x == 0) partials[t] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) last = arrive_last(arr);
    __syncthreads();
    if (!last) return;
    // exclusive scan of the tile sums, in chunks of blockDim.x
    int64_t run = 0;
    for (int64_t b0 = 0; b0 < tiles; b0 += blockDim.x) {
        int64_t i = b0 + threadIdx.x;
        int64_t v = i < tiles ? __hip_atomic_load(&partials[i], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) : 0;
        int64_t tot;
        int64_t pre = block_excl_scan(v, sh, &tot);
        if (i < tiles) partials[i] = run + pre;
        run += tot;
    }
    if (threadIdx.x == 0) {
        if (total) *total = run;
        f.post(run);
    }
}

template <class F, class W>
__global__ void __launch_bounds__(BLOCK) scan_apply_k(F f, W w, const int64_t *ws) {
    __shared__ int64_t sh[BLOCK / WAVE + 1];
    const int64_t n = f.size();
    if (n <= 0) return;
    const int64_t *partials = ws;
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    const auto wb = w.bind();
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        // each thread owns SCAN_ITEMS consecutive items
        int64_t first = t * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
        int64_t vals[SCAN_ITEMS];
        int64_t s = 0;
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            int64_t idx = first + i;
            vals[i] = idx < n ? f(idx) : 0;
            s += vals[i];
        }
        typename W::Pre pf[SCAN_ITEMS];
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; ++i)
            if (first + i < n) pf[i] = wb.prefetch(first + i, vals[i]);
        int64_t tot;
        int64_t pre = block_excl_scan(s, sh, &tot) + partials[t];
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            int64_t idx = first + i;
            if (idx < n) wb(idx, pre, vals[i], pf[i]);
            pre += vals[i];
        }
    }
}

// The same scan in one workgroup, for short inputs (no second launch, no
// arrival counter): items held in registers when n <= ONE_SCAN_CHUNK, else
// a reduction pass, post(), then chunked scan-and-apply passes.  post()
// runs (thread 0) before any apply, as in the two-kernel form, and the apply
// runs only if size() is still positive afterwards (as the apply kernel of
// the two-kernel form checks): a post() whose arena allocation failed leaves
// null output pointers and ends the level.
constexpr int ONE_SCAN_THREADS = 1024, ONE_SCAN_ITEMS = 16;
constexpr int64_t ONE_SCAN_CHUNK = (int64_t)ONE_SCAN_THREADS * ONE_SCAN_ITEMS;

// The body, for one workgroup of ONE_SCAN_THREADS threads; sh: LDS of
// ONE_SCAN_THREADS / WAVE + 1 int64, go: one int of LDS.  Every thread returns
// at the same point.
template <class F, class W>
__device__ __forceinline__ void scan_one_block(F f, W w, int64_t *total, int64_t *sh, int *go_p) {
    int &go = *go_p;
    const int64_t n = f.size();
    if (n < 0) return;
    const int64_t first = (int64_t)threadIdx.x * ONE_SCAN_ITEMS;
    if (n <= ONE_SCAN_CHUNK) {
        int64_t vals[ONE_SCAN_ITEMS];
        int64_t s = 0;
#pragma unroll
        for (int i = 0; i < ONE_SCAN_ITEMS; ++i) {
            vals[i] = first + i < n ? f(first + i) : 0;
            s += vals[i];
        }
        int64_t tot;
        int64_t pre = block_excl_scan(s, sh, &tot);
        if (threadIdx.x == 0) {
            if (total) *total = tot;
            f.post(tot);
            go = f.size() > 0;   // post() may end the level (allocation failed, stop rule)
        }
        __syncthreads();
        if (!go) return;
        const auto wb = w.bind();
        typename W::Pre pf[ONE_SCAN_ITEMS];
#pragma unroll
        for (int i = 0; i < ONE_SCAN_ITEMS; ++i)
            if (first + i < n) pf[i] = wb.prefetch(first + i, vals[i]);
#pragma unroll
        for (int i = 0; i < ONE_SCAN_ITEMS; ++i) {
            if (first + i < n) wb(first + i, pre, vals[i], pf[i]);
            pre += vals[i];
        }
        return;
    }
    int64_t s = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += f(i);
    int64_t tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) {
        if (total) *total = tot;
        f.post(tot);
        go = f.size() > 0;
    }
    __syncthreads();
    if (!go) return;
    const auto wb = w.bind();
    int64_t run = 0;
    for (int64_t base = 0; base < n; base += ONE_SCAN_CHUNK) {
        int64_t vals[ONE_SCAN_ITEMS];
        typename W::Pre pf[ONE_SCAN_ITEMS];
        int64_t t = 0;
#pragma unroll
        for (int i = 0; i < ONE_SCAN_ITEMS; ++i) {
            const int64_t idx = base + first + i;
            vals[i] = idx < n ? f(idx) : 0;
            t += vals[i];
        }
#pragma unroll
        for (int i = 0; i < ONE_SCAN_ITEMS; ++i)
            if (base + first + i < n) pf[i] = wb.prefetch(base + first + i, vals[i]);
        int64_t ctot;
        int64_t pre = block_excl_scan(t, sh, &ctot) + run;
#pragma unroll
        for (int i = 0; i < ONE_SCAN_ITEMS; ++i) {
            const int64_t idx = base + first + i;
            if (idx < n) wb(idx, pre, vals[i], pf[i]);
            pre += vals[i];
        }
        run += ctot;
    }
}

template <class F, class W>
__global__ void __launch_bounds__(ONE_SCAN_THREADS) scan_one_block_k(F f, W w, int64_t *total) {
    __shared__ int64_t sh[ONE_SCAN_THREADS / WAVE + 1];
    __shared__ int go;
    scan_one_block(f, w, total, sh, &go);
}

inline int64_t scan_tiles(int64_t n_max) { return (n_max + SCAN_TILE - 1) / SCAN_TILE; }

inline unsigned grid_for(int64_t items, int per_block, unsigned cap = 65535u * 4) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Profiling (events around launches), implemented in api.hip
// ---------------------------------------------------------------------------
struct ProfScope {
    int id;
    size_t rec;   // this launch's record (launches from several threads interleave)
    hipStream_t s;
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
};
#define KAPPA_PROF(name, stream) ::kappa::ProfScope _kappa_prof_scope(name, stream)

// n_hint: host-side estimate of the live size (grid sizing only); ws: the
// scan workspace described above.
template <class F, class W>
inline void launch_scan(int64_t n_hint, F f, W w, int64_t *ws, unsigned *arr, int64_t *total,
                        hipStream_t s) {
    if (n_hint <= tuning_now().scan_one_block_max) {   // any n is correct; short ones are fast
        KAPPA_PROF("scan_one_block", s);
        hipLaunchKernelGGL((scan_one_block_k<F, W>), dim3(1), dim3(ONE_SCAN_THREADS), 0, s, f, w,
                           total);
        return;
    }
    unsigned tiles = grid_for(n_hint, SCAN_TILE, 2048);
    {
        KAPPA_PROF("scan_reduce", s);
        hipLaunchKernelGGL(scan_reduce_k<F>, dim3(tiles), dim3(BLOCK), 0, s, f, ws, arr, total);
    }
    KAPPA_PROF("scan_apply", s);
    hipLaunchKernelGGL((scan_apply_k<F, W>), dim3(tiles), dim3(BLOCK), 0, s, f, w, ws);
}

// ---------------------------------------------------------------------------
// Device-resident multilevel state
// ---------------------------------------------------------------------------
enum LevelPhase : int32_t {
    PH_IDLE = 0,      // built, not started
    PH_MATCH = 1,     // matching in progress
    PH_CONTRACT = 2,  // matching done, contraction in progress
    PH_COMPACT = 3,   // next level allocated, rows being copied
    PH_DONE = 4,      // finished inside the tail kernel (later launches for it are no-ops)
    PH_MERGE = 5,     // two-phase matcher: gap rounds done, the matchings are merged next
    PH_STOPPED = -1   // a stop rule fired on this level
};

struct LevelDesc {
    int32_t n, maxdeg;
    int64_t nnz;
    int64_t *xadj;
    int32_t *adj;
    uint32_t *ew;
    uint32_t *vw;
    int32_t *cmap;    // to the next level
    int32_t *mate;
    int32_t *gid;     // batched form: graph of each node (null for a single graph)
    int32_t *noff;    // batched form: first node of each graph, count + 1 entries
    int64_t matched;
    int32_t rounds, stop, phase;
    int32_t grid_rounds;   // rounds run by the multi-block kernels (the rest: the finisher)
    // per round: nodes with a free neighbour, their degree sum; the rows
    // rescanned in the round and their degree sum (the same two where every
    // such node rescans)
    int64_t stat[STAT_ROUNDS][4];
};

enum ControlFlags : uint32_t {
    CF_ARENA = 1u,      // arena too small
    CF_HUBS = 2u,       // a coarse row needs the hub accumulators, which are not allocated
    CF_ROUNDS = 4u,     // round cap hit (cannot happen on valid state)
    CF_STATE = 8u,      // a list held a node id out of range (cannot happen on valid state)
    CF_EXTEND = 16u,    // level ext_level needs grid rounds after ext_round (the host resumes it)
};

struct Control {
    int32_t done;       // no further level starts
    int32_t nlevels;    // levels built (level nlevels-1 is the coarsest so far)
    uint32_t flags;
    int32_t ext_level;  // CF_EXTEND: the level whose matching continues on the host's
    int32_t ext_round;  //   next launch, and the last round it ran
    uint64_t cursor, cap;   // arena bytes used / available
    char *base;
    int32_t stop_n, max_levels;
    uint32_t stall_num, stall_den;
    int32_t last_n;     // node count of the newest level built (host grid sizing)
};

// Matching scratch (sized for level 0; reused by every level).
struct MatchState {
    int32_t cnt[4][4];      // [round & 3][bin]: sizes of the pending lists written by a round
                            // ([0][3]: chunk records of round 1's bin-2 list)
    int32_t scnt[4][4];     // [round & 3][bin]: rows round r rescans ([.][3]: chunk records)
    int32_t handoff;        // -1: rounds continue; r >= 0: the finisher resumes after round r; -2: done
    int32_t pad[3];
    int32_t sround[NSHARD];               // per shard: last round in which some node pointed
    // per round and shard: pointing nodes, their degree sum, pairs, rows
    // rescanned, their degree sum
    int64_t sstat[STAT_ROUNDS][5][NSHARD];
    int64_t spairs[NSHARD];                 // two-phase merge: pairs per shard (zero between uses)
};

// Two-phase matcher: the rating key (num, den, h) of the edge the block
// phase matched at a node (read only where that node has a block partner).
struct LocKey {
    uint64_t num, den, h;
};
// Rows above BIN_MID_MAX entries are scanned in chunks of HUB_CHUNK entries,
// one block per chunk, so that a round's latency does not grow with the
// longest row; the chunks' partial maxima are reduced per row by a separate
// launch before the mutual check.
constexpr int HUB_CHUNK = 2048;
// Chunk records of a level's bin-2 lists, per list parity: at most one per
// HUB_CHUNK entries of a row plus one per row, and every bin-2 row has more
// than BIN_MID_MAX entries, so nnz / 512 + 64 records always suffice.
inline int64_t hub_chunk_cap(int64_t nnz) { return nnz / 512 + 64; }
struct HubChunks {
    int2 *rec;       // 2 * cap: per parity, {position in the bin-2 list, chunk index}
    int32_t *first;  // 2 * n: per parity and bin-2 list position, the row's first record
                     // (-1: the row keeps its choice this round)
    Cand *part;      // cap: the chunks' maxima of the current round
    int64_t cap;
    int2 *scan;      // 2 * n: per bin 0 / 1, {node, list position} of the rows a round
                     // rescans (written by the round's preparation)
    int32_t *kfirst; // n: per node of a chunked row, its first record of round 1, where
                     // part keeps the row's chunk maxima for the rest of the level
};
struct MatchScratch {
    int32_t *best;          // n: current choice of every node (-1: none)
    int32_t *lv, *lb, *ld;  // 6n each: pending lists [parity][bin] (node, choice, degree)
    int2 *nrec;             // n: {rating attribute c(v) or Out(v), mate} per node
    uint32_t *out;          // n (innerOuter)
    int32_t *tile_row;      // tile rows of the level (innerOuter)
    MatchState *state;
    int32_t *loc;           // two-phase: n, the block phase's partner (-1: none)
    LocKey *lkey;           // two-phase: n, the key of that edge
    HubChunks hub;          // rec == nullptr: long rows are scanned by one block each
    unsigned *coop_bar;     // 2 + ARRIVE_WORDS: the persistent rounds' grid barrier (zero)
};

// Contraction scratch (sized for level 0).
struct ContractScratch {
    int32_t *rep_of;      // n   coarse -> representative fine node
    int32_t *partner;     // n   coarse -> partner of the representative (-1)
    int32_t *cdeg;        // n   coarse degrees
    int32_t *rows;        // 4n  row-class lists: [0, n) class 3, [n, 2n) class 1,
                          //     [2n, 3n) class 2, [3n, 4n) class 4
    int32_t *row_cnt;     // 8   row-class counts (classes 1 to 4)
    int32_t *tmp_adj;     // nnz
    uint32_t *tmp_ew;     // nnz
    int64_t *partials;    // scan workspace: tile sums
    unsigned *arrive;     // ARRIVE_WORDS arrival counters of the scans (zero between uses)
    int64_t *totals;      // [0] n', [1] unused, [2] nnz', [3] unused
    uint32_t *hub_acc;    // hub_slots * n, zero between uses (may be null)
    uint32_t *hub_bits;   // hub_slots * hub_words, zero between uses: per slot the id
                          // bitmap (hub_w1 words), then its summary (a bit per word)
    int64_t hub_words, hub_w1;
    int32_t hub_slots;    // rows merged at once in the hub accumulators
    // large rows by key buckets (null unless Ctx::huge): the groups merged
    // where they lie in hg_adj / hg_ew (the staging positions' twins), group
    // lists by size, per group slot its first position and merged count, per
    // large row its first slot and group count; hg_cnt: small groups, large
    // groups, slots (zero between levels)
    int32_t *hg_adj;      // nnz
    uint32_t *hg_ew;      // nnz
    int4 *hg_small;       // hg_cap: row list index, first position, size, slot
    int4 *hg_big;         // hg_cap
    int2 *hg_slot;        // hg_cap
    int2 *hg_row;         // hg_rows
    int32_t *hg_cnt;      // 4
    int64_t hg_cap, hg_rows;
};

// Batched form: per-graph stop rules on a disjoint union of `count` graphs.
// A graph that stops is frozen: its nodes neither match nor carry over to
// the next level.
struct BatchCtx {
    int32_t count = 0;              // 0: a single graph
    uint32_t stall_num = 0, stall_den = 1;
    const int32_t *stop_n = nullptr;   // [count]
    uint8_t *active = nullptr;         // [count] 1 while the graph coarsens
    int32_t *coarsest = nullptr;       // [count] level of the graph's coarsest graph
    int32_t *reason = nullptr;         // [count] kappa_stop of the graph
    int32_t *excl = nullptr;           // [n] exclusive prefix of the coarse-id scan
    // Served steps (all null otherwise).  A graph of the union is somewhere
    // down its own hierarchy: gbase[g] is the seed plus its depth, and every
    // level start writes gseed[g] = mix64(gbase[g] + level); lmax[g] is how
    // many levels it may still build.  The step ends at the first level
    // boundary after a graph stopped (stop_seen, or a stop at that boundary)
    // or the host raised *interrupt (host memory): graphs still coarsening
    // get reason KAPPA_STOP_NONE there.
    const uint64_t *gbase = nullptr;   // [count]
    uint64_t *gseed = nullptr;         // [count]
    const int32_t *lmax = nullptr;     // [count]
    const uint32_t *interrupt = nullptr;
    uint32_t *stop_seen = nullptr;
};

struct Ctx {
    Tune t = tuning_now();
    Control *ctrl;
    LevelDesc *lv;
    int32_t rating;
    int32_t seed_direct;   // 1: level seeds are `seed` itself; 0: mix64(seed + level)
    uint64_t seed;
    MatchScratch ms;
    ContractScratch cs;
    BatchCtx b;
    int32_t block_bits = -1;   // >= 0: two-phase matcher with blocks of 2^block_bits ids
    int32_t big_blocks = 64;   // blocks per round launch for rows above BIN_MID_MAX entries
    int32_t big_rows = 1;      // 1: rows of 4095..16382 entries get the big-row sort launch
                               // where the key buckets do not apply (and the small-row
                               // merge buffers its list appends); 0: they join the large rows
    int32_t huge = 0;          // 1: large rows get the key-bucket merge launches
    int32_t rescan_stats = 0;  // 1: record the rescan statistics (while the profiler is on)
};

// K bump allocations in the arena with one read and one write of the cursor
// (one thread).  false (and every pointer null) on overflow.
template <int K>
__device__ __forceinline__ bool arena_alloc_k(Control *c, const uint64_t (&bytes)[K],
                                              void *(&out)[K]) {
    uint64_t cur = c->cursor;
    const uint64_t cap = c->cap;
    char *const base = c->base;
    uint64_t off[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        cur = (cur + 255u) & ~(uint64_t)255u;
        off[i] = cur;
        cur += bytes[i] ? bytes[i] : 1;
    }
    if (cur > cap) {
        c->flags |= CF_ARENA;
#pragma unroll
        for (int i = 0; i < K; ++i) out[i] = nullptr;
        return false;
    }
    c->cursor = cur;
#pragma unroll
    for (int i = 0; i < K; ++i) out[i] = base + off[i];
    return true;
}

// ---------------------------------------------------------------------------
// Launch wrappers (host functions) per translation unit
// ---------------------------------------------------------------------------
// k_graph.hip
// Up to ZERO_MAX ranges of 4-byte words zeroed by one launch.
constexpr int ZERO_MAX = 8;
struct ZeroRanges {
    uint32_t *p[ZERO_MAX];
    int64_t words[ZERO_MAX];
    int32_t count = 0;
    void add(void *ptr, int64_t n) {   // n 4-byte words; ignored if empty
        if (!ptr || n <= 0) return;
        p[count] = (uint32_t *)ptr;
        words[count] = n;
        ++count;
    }
};
void launch_zero(const ZeroRanges &z, hipStream_t s);
// ctrl and lv[0] = l0 written, lv[1 .. nlv-1] zeroed, in one launch.
void launch_init_levels(Control *dctrl, LevelDesc *lv, int32_t nlv, const Control &ctrl,
                        const LevelDesc &l0, hipStream_t s);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
// Entry tiles: tile_row[t] = row holding CSR entry t * 2048.  Needs
// tile_rows_needed(nnz) int32 entries.  Valid until the graph changes.
int64_t tile_rows_needed(int64_t nnz);
void launch_tile_rows(const DevGraph &g, int32_t *tile_row, hipStream_t s);
// flags: bit0 offsets, bit1 structure, bit2 range.  sums[4][NSHARD] (zeroed
// by the caller), summed over shards: [0] = sum w(E), [1] = sum c(V),
// [2] / [3] = entries above / below the diagonal (must be equal);
// maxdeg[NSHARD] (zeroed): max row length per shard.  Computes its own tile
// rows into tile_row.
// offsets_only: the offsets pass alone (row offsets, c(V), maximum degree).
// With a sort_ws of val_sort_ws_bytes bytes (graphs of at least
// VAL_SORT_MIN_NNZ entries) symmetry is checked by sorting, else by binary
// searches.  The caller passes sort_ws only for graphs with rows above
// VAL_SORT_MIN_DEG entries (the offsets pass's maximum degree): there each
// search probe of a long row fetches a line of its own, while the searches
// of short, cache-resident rows cost less than the sort.  entries_only: the
// offsets pass has run already.
constexpr int64_t VAL_SORT_MIN_NNZ = (int64_t)1 << 22;
constexpr int32_t VAL_SORT_MIN_DEG = 1024;
size_t val_sort_ws_bytes(int64_t n, int64_t nnz);
void launch_validate(const DevGraph &g, int32_t *tile_row, uint32_t *flags, uint64_t *sums,
                     int32_t *maxdeg, hipStream_t s, bool offsets_only = false,
                     char *sort_ws = nullptr, bool entries_only = false);
void launch_out(const DevGraph &g, const int32_t *tile_row, uint32_t *out, hipStream_t s);
void launch_rate(const DevGraph &g, const int32_t *tile_row, int rating, const uint32_t *out,
                 uint64_t *num, uint64_t *den, hipStream_t s);
// flags |= 1 if mate is not a matching of g (entry out of range, not
// symmetric, or a matched pair that is not an edge).
void launch_check_matching(const DevGraph &g, const int32_t *mate, uint32_t *flags,
                           hipStream_t s);
void launch_initial_partition(int32_t n, int32_t k, uint64_t seed, int32_t *part,
                              hipStream_t s);
void launch_project(const int32_t *cmap, int32_t n_fine, int32_t n_coarse,
                    const int32_t *part_coarse, int32_t *part_fine, uint32_t *flag,
                    hipStream_t s);
// One level of the way back up: the level's partition (mode: UP_GIVEN reads
// part, UP_PROJECT writes part[v] = part_c[cmap[v]], UP_INITIAL writes the
// stand-in part[v] = mix64(part_seed + v) mod k), then cut and balance into
// res (device).  block_w_out (device [k], may be null) receives the block
// weights.  The accumulators in `a` are zero on entry and left zero
// (launch_up_clear zeroes them once).  tile_row: tile_rows_needed(g.nnz).
enum UpMode { UP_GIVEN = 0, UP_PROJECT = 1, UP_INITIAL = 2 };
constexpr int BW_SHARDS = 8;
struct UpAcc {
    uint64_t *bw;      // BW_SHARDS * k
    uint64_t *acc;     // 3 * NSHARD
    unsigned *arrive;  // ARRIVE_WORDS
    uint32_t *flag;    // 1: bit 0 map entry, bit 1 block id out of range
};
void launch_up_level(const DevGraph &g, int mode, const int32_t *cmap, int32_t n_coarse,
                     const int32_t *part_c, uint64_t part_seed, int32_t *part, int32_t k,
                     uint32_t eps_num, uint32_t eps_den, int32_t *tile_row, const UpAcc &a,
                     uint64_t *block_w_out, kappa_cut_result *res, hipStream_t s);
void launch_up_clear(const UpAcc &a, int32_t k, hipStream_t s);
// Level-resident variants of Out(v) (innerOuter): read level l's graph from the
// descriptor; run only while level l is matching.
void launch_level_out(const Ctx &c, int l, int64_t nnz_cap, int32_t n_hint, hipStream_t s);

// k_level.hip: one level of the multilevel loop, driven by device state.
// n_hint: host estimate of the level's size (grid sizing only).  rounds:
// multi-block matching rounds before the one-workgroup finisher.
// Tries the one-workgroup tail from level l (a no-op unless level l is
// small, not started, and the loop still runs).
void launch_tail(const Ctx &c, int l, hipStream_t s);
void launch_level(const Ctx &c, int l, int32_t n_hint, int64_t nnz_cap, int32_t n_cap,
                  int rounds, hipStream_t s);
// Batched form, per level: per-graph size and level-count rules before the
// level (ends the loop when no graph is left), and per-graph empty-matching
// and stall rules once the coarse ids are known.
void launch_batch_begin(const Ctx &c, int l, hipStream_t s);
void launch_batch_end(const Ctx &c, int l, hipStream_t s);
// Graph id of every node from the graphs' first nodes (noff, count + 1).
void launch_batch_gid(const int32_t *noff, int32_t count, int32_t n, int32_t *gid, hipStream_t s);
// flags |= 1 if some row of g has an entry outside its graph's node range.
void launch_batch_check(const DevGraph &g, uint32_t *flags, hipStream_t s);
// One graph of a union to build (device arrays).
struct UnionSrc {
    const int64_t *xadj;
    const int32_t *adj;
    const uint32_t *ew, *vw;
};
// The block-diagonal union of `count` graphs (src, noff, eoff in device
// memory; noff / eoff: count + 1 node and entry offsets) into xadj[n + 1],
// adj[nnz], ew[nnz], vw[n].
void launch_union_build(const UnionSrc *src, int32_t count, const int64_t *noff,
                        const int64_t *eoff, int64_t n, int64_t nnz, int64_t *xadj, int32_t *adj,
                        uint32_t *ew, uint32_t *vw, hipStream_t s);
// Served steps (a union advanced by one level): every graph's next level with
// local ids (graph g's nodes at noff1[g], its row offsets at noff1[g] + g,
// its entries where the union has them), level 0's map made local, and each
// graph's first entry on the next level (eoff1, count + 1 values).
void launch_serve_extract(const DevGraph &u1, const int32_t *noff1, int32_t count,
                          const int32_t *cmap0, const int32_t *gid0, int32_t n0, int64_t *xadj,
                          int32_t *adj, uint32_t *ew, uint32_t *vw, int32_t *cmap, int64_t *eoff1,
                          int32_t *dmax, hipStream_t s);
// Copies nodes [a, b) of union level u (entries from ea, nnz of them) with
// ids made local; cmap/mate (may be null) shifted as well.
void launch_batch_extract(const DevGraph &u, const int32_t *cmap, const int32_t *mate, int32_t a,
                          int32_t b, int64_t ea, int64_t nnz, int32_t cbase, int64_t *xadj,
                          int32_t *adj, uint32_t *ew, uint32_t *vw, int32_t *cmap_out,
                          int32_t *mate_out, hipStream_t s);

// Matching only (first kernel: the level gate, which moves an idle level to
// PH_MATCH unless a stop rule fires; stop_rules = false checks none), e.g.
// for kappa_match.  out_kernels: compute Out(v) (innerOuter) from the graph;
// otherwise it must already be in the scratch (written by the previous
// level's compaction).  Needs st->cnt zero on entry.
extern bool g_persistent_on;   // matching rounds of a level in one cooperative launch
void launch_level_match(const Ctx &c, int l, int32_t n_hint, int64_t nnz_cap, int rounds,
                        bool stop_rules, bool out_kernels, hipStream_t s);
// k_sort.hip: stable LSD radix sort of n < 2^31 (key, 32-bit value) pairs by
// key bits [begin_bit, end_bit), 8 bits per pass (KT uint32_t or uint64_t;
// kin != kout, vin != vout; the input is not modified); ws holds
// radix_sort_ws_bytes(n, sizeof(KT)) bytes.  Stream-ordered.
size_t radix_sort_ws_bytes(int64_t n, size_t key_bytes);
template <class KT>
kappa_status radix_sort_pairs(const KT *kin, KT *kout, const uint32_t *vin, uint32_t *vout,
                              int64_t n, int begin_bit, int end_bit, char *ws, hipStream_t s);
// Exclusive sum of n int64 (out may not alias in); ws: exclusive_sum_ws_bytes(n).
size_t exclusive_sum_ws_bytes(int64_t n);
kappa_status exclusive_sum_i64(const int64_t *in, int64_t *out, int64_t n, char *ws, hipStream_t s);
// Recursive coordinate bisection order of n points (xy interleaved, device)
// and the relabelling of a graph by an order (k_relabel.hip).  ws == nullptr
// asks for the workspace size only (*need).  Both synchronise the stream.
kappa_status rcb_order_impl(const double *xy, int32_t n, int32_t leaf, int32_t *order,
                            hipStream_t s, char *ws, size_t ws_bytes, size_t *need);
kappa_status relabel_impl(const DevGraph &g, const int32_t *order, int64_t *nx, int32_t *nadj,
                          uint32_t *new_ew, uint32_t *nvw, hipStream_t s, char *ws,
                          size_t ws_bytes, size_t *need, uint32_t *hflag);
// The rest of a level the finisher handed back (CF_EXTEND after round
// r_from): `count` more grid rounds, the finisher and, if `contract`, the
// contraction.
void launch_level_extend(const Ctx &c, int l, int32_t n_hint, int32_t n_cap, int r_from,
                         int count, bool contract, hipStream_t s);
// Contraction only (level phase PH_CONTRACT, mate set), e.g. for kappa_contract.
void launch_level_contract(const Ctx &c, int l, int32_t n_hint, int32_t n_cap, hipStream_t s);


// ---- pairwise refinement (k_refine.hip) -----------------------------------
constexpr int REFINE_K_MAX = 256;                  // blocks
constexpr int REFINE_QW = REFINE_K_MAX / 64;       // bitmap words per row of Q
constexpr int REFINE_COLOURS = 512;                // greedy colouring needs at most 2k - 3
constexpr int REFINE_CW = REFINE_COLOURS / 64;

struct RefineCtl {
    unsigned long long total;     // c(V)
    unsigned long long max_node;  // max_v c(v)
    uint32_t flags;               // 1: a block id outside [0, k); 2: block counts disagree with part
    int32_t ncol, npairs, pad;
    unsigned long long stats[8];  // [1] searches, [2] moves, [3] kept, [4] adoptions, [5] bytes,
                                  // [6] / [7] clock ticks in initialisation / moves
};

struct RefineLaunch {
    const int64_t *xadj;
    const int32_t *adj;
    const uint32_t *ew;
    const uint32_t *vw;
    int32_t *part;
    int32_t n, k;
    uint32_t eps_num, eps_den;
    uint64_t seed;
    uint32_t alpha_num, alpha_den;
    int32_t depth, max_local;
    int32_t *cpairs, *col_off, *poff, *fill;
    int64_t *bw;
    int32_t *bc;
    int32_t *region, *dist;
    int64_t *gain;
    uint8_t *status;
    int32_t *qlist, *mlog, *slot;
    int32_t qcap;   // queue entries per search kept on chip (-1: the kernel's maximum)
    RefineCtl *ctl;
};

void launch_refine_weights(const int32_t *part, const uint32_t *vw, int32_t n, int32_t k,
                           int64_t *bw, int32_t *bc, RefineCtl *ctl, hipStream_t s);
// Q of the current partition and its greedy colouring (qbits must be zero).
void launch_refine_colouring(const int64_t *xadj, const int32_t *adj, const int32_t *part,
                             int32_t n, int32_t k, unsigned long long *qbits, int32_t *tmp_pair,
                             int32_t *tmp_col, int32_t *cpairs, int32_t *col_off, int32_t *fill,
                             RefineCtl *ctl, hipStream_t s);
// the local searches of colour c (npairs pairs) of global iteration gi
void launch_refine_colour(const RefineLaunch &R, int32_t gi, int32_t c, int32_t npairs,
                          hipStream_t s);

}  // namespace kappa
