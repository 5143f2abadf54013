// k_graph.hip -- CSR sweeps: validation, Out(v), ratings, initial partition,
// projection, cut/balance.
//
// The per-entry sweeps (validation, Out, ratings, cut) are load balanced by
// entries, not rows: tile t owns entries [t*ETILE, (t+1)*ETILE).  A small
// pre-pass records the row holding each tile's first entry; a block stages the
// row offsets of its tile in LDS and finds each entry's row by binary search
// there.  Reads of adj/ew are fully coalesced and a node of any degree costs
// the same per entry (power-law hubs spread over many tiles).
#include "kappa_internal.h"

namespace kappa {

constexpr int ETILE_ITEMS = 8;
constexpr int ETILE = BLOCK * ETILE_ITEMS;   // 2048 entries per tile
constexpr int ETILE_ROWS = 2048;             // row offsets staged in LDS

// ---------------------------------------------------------------------------
__global__ void fill_u32_k(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_u64_k(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// Zero up to ZERO_MAX ranges of 4-byte words in one launch.
__global__ void zero_ranges_k(ZeroRanges z) {
    for (int r = 0; r < z.count; ++r) {
        uint32_t *p = z.p[r];
        const int64_t n = z.words[r];
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            p[i] = 0u;
    }
}
void launch_zero(const ZeroRanges &z, hipStream_t s) {
    int64_t most = 0;
    for (int r = 0; r < z.count; ++r) most = z.words[r] > most ? z.words[r] : most;
    if (most <= 0) return;
    KAPPA_PROF("fill", s);
    hipLaunchKernelGGL(zero_ranges_k, dim3(grid_for(most, BLOCK, 4096)), dim3(BLOCK), 0, s, z);
}

// The control block and the level descriptors of a call: ctrl, lv[0] = l0,
// lv[1 .. nlv-1] zero (idle), in one launch.
__global__ void init_levels_k(Control *dctrl, LevelDesc *lv, int32_t nlv, Control ctrl,
                              LevelDesc l0) {
    constexpr int W = (int)(sizeof(LevelDesc) / 4);
    static_assert(sizeof(LevelDesc) % 4 == 0, "descriptor words");
    uint32_t *p = (uint32_t *)(lv + 1);
    const int64_t words = (int64_t)(nlv - 1) * W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
    if (blockIdx.x == 0) {
        const uint32_t *src = (const uint32_t *)&l0;
        uint32_t *dst = (uint32_t *)lv;
        for (int i = threadIdx.x; i < W; i += blockDim.x) dst[i] = src[i];
        if (threadIdx.x == 0) *dctrl = ctrl;
    }
}
void launch_init_levels(Control *dctrl, LevelDesc *lv, int32_t nlv, const Control &ctrl,
                        const LevelDesc &l0, hipStream_t s) {
    KAPPA_PROF("init_levels", s);
    const int64_t words = (int64_t)(nlv - 1) * (int64_t)(sizeof(LevelDesc) / 4);
    hipLaunchKernelGGL(init_levels_k, dim3(grid_for(words, BLOCK, 64)), dim3(BLOCK), 0, s, dctrl,
                       lv, nlv, ctrl, l0);
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    KAPPA_PROF("fill", s);
    hipLaunchKernelGGL(fill_u32_k, dim3(grid_for(n, BLOCK, 4096)), dim3(BLOCK), 0, s, p, n, v);
}
void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return;
    KAPPA_PROF("fill", s);
    hipLaunchKernelGGL(fill_u64_k, dim3(grid_for(n, BLOCK, 4096)), dim3(BLOCK), 0, s, p, n, v);
}

// ---------------------------------------------------------------------------
// Entry tiles
// ---------------------------------------------------------------------------
__host__ __device__ inline int64_t etiles(int64_t nnz) { return (nnz + ETILE - 1) / ETILE; }
int64_t tile_rows_needed(int64_t nnz) { return etiles(nnz) + 1; }

// tile_row[t] = row holding entry t*ETILE (largest v with xadj[v] <= t*ETILE).
__device__ __forceinline__ void tile_rows_body(const DevGraph &g, int32_t *tile_row) {
    const int64_t ntiles = etiles(g.nnz);
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = g.xadj[v], e = g.xadj[v + 1];
        if (b < 0 || e > g.nnz || e <= b) continue;   // also safe on broken offsets
        for (int64_t t = (b + ETILE - 1) / ETILE; t * ETILE < e && t < ntiles; ++t)
            tile_row[t] = (int32_t)v;
    }
}

__global__ void tile_rows_k(DevGraph g, int32_t *tile_row) { tile_rows_body(g, tile_row); }

void launch_tile_rows(const DevGraph &g, int32_t *tile_row, hipStream_t s) {
    if (etiles(g.nnz) == 0) return;
    KAPPA_PROF("tile_rows", s);
    hipLaunchKernelGGL(tile_rows_k, dim3(grid_for(g.n, BLOCK, 4096)), dim3(BLOCK), 0, s, g,
                       tile_row);
}

struct TileCtx {
    int64_t j0, j1;
    int32_t r0, r1;
    bool lds;
};

// Sets up tile t: LDS offsets of rows r0..r1 (+1) when they fit.  Block-wide.
__device__ __forceinline__ TileCtx tile_begin(const DevGraph &g, const int32_t *tile_row,
                                              int64_t t_idx, int64_t *s_off) {
    TileCtx t;
    t.j0 = t_idx * ETILE;
    t.j1 = t.j0 + ETILE < g.nnz ? t.j0 + ETILE : g.nnz;
    t.r0 = tile_row[t_idx];
    t.r1 = t_idx + 1 < etiles(g.nnz) ? tile_row[t_idx + 1] : g.n - 1;
    int32_t nr = t.r1 - t.r0 + 1;
    t.lds = nr <= ETILE_ROWS;
    __syncthreads();   // s_off may still be read for the previous tile
    if (t.lds)
        for (int i = threadIdx.x; i <= nr; i += blockDim.x) s_off[i] = g.xadj[t.r0 + i];
    __syncthreads();
    return t;
}

// Row of entry j inside the tile.
__device__ __forceinline__ int32_t tile_row_of(const DevGraph &g, const TileCtx &t,
                                               const int64_t *s_off, int64_t j) {
    int32_t lo, hi;
    if (t.lds) {
        lo = 0; hi = t.r1 - t.r0;
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= j) lo = mid; else hi = mid - 1;
        }
        return t.r0 + lo;
    }
    lo = t.r0; hi = t.r1;
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo + 1) >> 1);
        if (g.xadj[mid] <= j) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t tile_row_start(const DevGraph &g, const TileCtx &t,
                                                  const int64_t *s_off, int32_t v) {
    return t.lds ? s_off[v - t.r0] : g.xadj[v];
}

// ---------------------------------------------------------------------------
// Validation (Section 2 graph model).  flags: 1 = offsets, 2 = structure,
// 4 = weight range.  Also the maximum degree.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) validate_offsets_k(DevGraph g, uint32_t *flags,
                                                            uint64_t *sums, int32_t *maxdeg) {
    __shared__ uint64_t sh[BLOCK / WAVE + 1];
    __shared__ int32_t shm[BLOCK / WAVE];
    bool bad = false;
    uint64_t csum = 0;
    int32_t md = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (g.xadj[0] != 0 || g.xadj[g.n] != g.nnz)) bad = true;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = g.xadj[v + 1] - g.xadj[v];
        if (d < 0) bad = true;
        else if (d > md) md = d > 0x7fffffff ? 0x7fffffff : (int32_t)d;
        csum += g.vw[v];
    }
    csum = block_sum(csum, sh);
    md = wave_max(md);
    if (lane_id() == 0) shm[threadIdx.x / WAVE] = md;
    bool wbad = __ballot(bad) != 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int sd = shard_of_block();
        for (int i = 1; i < BLOCK / WAVE; ++i) md = shm[i] > md ? shm[i] : md;
        if (csum) atomicAdd((unsigned long long *)&sums[1 * NSHARD + sd], (unsigned long long)csum);
        if (md) atomicMax(&maxdeg[sd], md);
    }
    if (wbad && lane_id() == 0) atomicOr(flags, 1u);
}

// SEARCH: the reverse-entry check by binary searches (a thread's searches
// in lockstep, so their loads overlap); otherwise the sorted check below
// does it and this pass keeps the local checks and the counts.
template <bool SEARCH>
__global__ void __launch_bounds__(BLOCK) validate_entries_k(DevGraph g, const int32_t *tile_row,
                                                            uint32_t *flags, uint64_t *sums) {
    __shared__ int64_t s_off[ETILE_ROWS + 1];
    __shared__ uint64_t sh[BLOCK / WAVE + 1];
    if (flags[0] & 1u) return;   // offsets broken: rows cannot be read safely
    const int64_t ntiles = etiles(g.nnz);
    uint32_t bad = 0;
    uint64_t wsum = 0, above = 0, below = 0;
    for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        TileCtx t = tile_begin(g, tile_row, tt, s_off);
        int32_t vv[ETILE_ITEMS], uu[ETILE_ITEMS];
        uint32_t ww[ETILE_ITEMS];
        int64_t lo[ETILE_ITEMS], len[ETILE_ITEMS];
        for (int i = 0; i < ETILE_ITEMS; ++i) {
            int64_t j = t.j0 + (int64_t)i * BLOCK + threadIdx.x;
            uu[i] = -1;
            vv[i] = 0;
            ww[i] = 0;
            len[i] = 0;
            lo[i] = 0;
            if (j >= t.j1) continue;
            int32_t v = tile_row_of(g, t, s_off, j);
            int32_t u = g.adj[j];
            uint32_t w = g.ew[j];
            vv[i] = v;
            ww[i] = w;
            if (u < 0 || u >= g.n || u == v) { bad |= 2; continue; }
            if (j > tile_row_start(g, t, s_off, v) && g.adj[j - 1] >= u) bad |= 2;
            if (w == 0) bad |= 4;
            // Only entries above the diagonal look up their reverse: with no
            // duplicates in a row, that map is injective into the entries
            // below the diagonal, so equal counts above and below (checked on
            // the host) make it a bijection.
            if (u > v) { wsum += w; uu[i] = u; ++above; }
            else ++below;
        }
        if (!SEARCH) continue;
        for (int i = 0; i < ETILE_ITEMS; ++i)
            if (uu[i] >= 0) { lo[i] = g.xadj[uu[i]]; len[i] = g.xadj[uu[i] + 1] - lo[i]; }
        // lower_bound of v in row u, all searches advanced together
        bool any = true;
        while (any) {
            any = false;
            for (int i = 0; i < ETILE_ITEMS; ++i) {
                if (len[i] <= 0) continue;
                int64_t half = len[i] >> 1;
                if (g.adj[lo[i] + half] < vv[i]) { lo[i] += half + 1; len[i] -= half + 1; }
                else len[i] = half;
                any = any || len[i] > 0;
            }
        }
        for (int i = 0; i < ETILE_ITEMS; ++i) {
            if (uu[i] < 0) continue;
            int64_t end = g.xadj[uu[i] + 1];
            if (lo[i] >= end || g.adj[lo[i]] != vv[i] || g.ew[lo[i]] != ww[i]) bad |= 2;
        }
    }
    wsum = block_sum(wsum, sh);
    above = block_sum(above, sh);
    below = block_sum(below, sh);
    if (threadIdx.x == 0) {
        const int sd = shard_of_block();
        if (wsum) atomicAdd((unsigned long long *)&sums[0 * NSHARD + sd], (unsigned long long)wsum);
        if (above) atomicAdd((unsigned long long *)&sums[2 * NSHARD + sd], (unsigned long long)above);
        if (below) atomicAdd((unsigned long long *)&sums[3 * NSHARD + sd], (unsigned long long)below);
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) bad |= __shfl_xor(bad, off, WAVE);
    if (bad && lane_id() == 0) atomicOr(flags, bad);
}

// Sorted reverse-entry check (large graphs): the entries below the diagonal,
// in CSR order, are sorted by (row, neighbour); the entries above it,
// written as keys (neighbour << shift | row) and sorted, must equal them one
// for one, weights included.  With no duplicates in a row and as many
// entries above as below (both checked by the entry pass), that is the
// symmetry test.  Random searches into other rows (one cache line per step)
// become sequential passes and a radix sort.
// low[v]: entries of row v below the diagonal (a binary search for v in row v).
__global__ void __launch_bounds__(BLOCK) val_low_k(DevGraph g, const uint32_t *flags, int64_t *low) {
    if (flags[0] & 1u) return;   // offsets broken
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = g.xadj[v], len = g.xadj[v + 1] - lo;
        const int64_t b = lo;
        while (len > 0) {
            const int64_t half = len >> 1;
            if (g.adj[lo + half] < v) { lo += half + 1; len -= half + 1; }
            else len = half;
        }
        low[v] = lo - b;
    }
}
// The entries above the diagonal as sorted-check keys; row v's occupy
// positions from xadj[v] - lowstart[v] (the entries above the diagonal of
// the rows before v) on.
__global__ void __launch_bounds__(BLOCK) val_upper_k(DevGraph g, const int32_t *tile_row,
                                                     uint32_t *flags, const int64_t *low,
                                                     const int64_t *lowstart, int shift,
                                                     int64_t cap, uint64_t *key, uint32_t *val) {
    __shared__ int64_t s_off[ETILE_ROWS + 1];
    if (flags[0] & 1u) return;
    const int64_t ntiles = etiles(g.nnz);
    uint32_t bad = 0;
    for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        TileCtx t = tile_begin(g, tile_row, tt, s_off);
        for (int i = 0; i < ETILE_ITEMS; ++i) {
            const int64_t j = t.j0 + (int64_t)i * BLOCK + threadIdx.x;
            if (j >= t.j1) continue;
            const int32_t v = tile_row_of(g, t, s_off, j);
            const int32_t u = g.adj[j];
            if (u <= v || u >= g.n) continue;   // below the diagonal, or flagged by the entry pass
            const int64_t rs = tile_row_start(g, t, s_off, v);
            const int64_t k = j - rs - low[v];
            const int64_t pos = rs - lowstart[v] + k;
            if (k < 0 || pos < 0 || pos >= cap) { bad |= 2; continue; }   // unsorted or unbalanced
            key[pos] = ((uint64_t)(uint32_t)u << shift) | (uint32_t)v;
            val[pos] = g.ew[j];
        }
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) bad |= __shfl_xor(bad, off, WAVE);
    if (bad && lane_id() == 0) atomicOr(flags, bad);
}
// Every entry below the diagonal against the sorted keys: the p-th such entry
// of row u is number lowstart[u] + p.
__global__ void __launch_bounds__(BLOCK) val_match_k(DevGraph g, const int32_t *tile_row,
                                                     uint32_t *flags, const int64_t *low,
                                                     const int64_t *lowstart, int shift,
                                                     int64_t cap, const uint64_t *key,
                                                     const uint32_t *val) {
    __shared__ int64_t s_off[ETILE_ROWS + 1];
    if (flags[0] & 1u) return;
    const int64_t ntiles = etiles(g.nnz);
    uint32_t bad = 0;
    for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        TileCtx t = tile_begin(g, tile_row, tt, s_off);
        for (int i = 0; i < ETILE_ITEMS; ++i) {
            const int64_t j = t.j0 + (int64_t)i * BLOCK + threadIdx.x;
            if (j >= t.j1) continue;
            const int32_t u = tile_row_of(g, t, s_off, j);
            const int32_t v = g.adj[j];
            const int64_t p = j - tile_row_start(g, t, s_off, u);
            if (p >= low[u]) continue;   // not below the diagonal
            const int64_t idx = lowstart[u] + p;
            if (v < 0 || idx >= cap || key[idx] != (((uint64_t)(uint32_t)u << shift) | (uint32_t)v) ||
                val[idx] != g.ew[j])
                bad |= 2;
        }
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) bad |= __shfl_xor(bad, off, WAVE);
    if (bad && lane_id() == 0) atomicOr(flags, bad);
}

size_t val_sort_ws_bytes(int64_t n, int64_t nnz) {
    if (nnz < VAL_SORT_MIN_NNZ || nnz / 2 >= ((int64_t)1 << 31)) return 0;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t cap = nnz / 2 > 0 ? nnz / 2 : 1;
    return 2 * al(8 * ((size_t)n + 1)) + al(exclusive_sum_ws_bytes(n)) + 2 * al(8 * (size_t)cap) +
           2 * al(4 * (size_t)cap) + al(radix_sort_ws_bytes(cap, 8));
}

void launch_validate(const DevGraph &g, int32_t *tile_row, uint32_t *flags, uint64_t *sums,
                     int32_t *maxdeg, hipStream_t s, bool offsets_only, char *sort_ws,
                     bool entries_only) {
    int64_t nt = etiles(g.nnz);
    if (!entries_only) {
        KAPPA_PROF("validate_offsets", s);
        hipLaunchKernelGGL(validate_offsets_k, dim3(grid_for((int64_t)g.n + 1, BLOCK * 4, 1024)),
                           dim3(BLOCK), 0, s, g, flags, sums, maxdeg);
    }
    if (nt == 0 || offsets_only) return;
    launch_tile_rows(g, tile_row, s);
    const bool sorted = sort_ws && val_sort_ws_bytes(g.n, g.nnz) > 0;
    {
        KAPPA_PROF("validate_entries", s);
        if (sorted)
            hipLaunchKernelGGL(validate_entries_k<false>, dim3(grid_for(nt, 1, 8192)), dim3(BLOCK), 0,
                               s, g, tile_row, flags, sums);
        else
            hipLaunchKernelGGL(validate_entries_k<true>, dim3(grid_for(nt, 1, 8192)), dim3(BLOCK), 0,
                               s, g, tile_row, flags, sums);
    }
    if (!sorted) return;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t cap = g.nnz / 2;
    char *p = sort_ws;
    int64_t *low = (int64_t *)p;
    p += al(8 * ((size_t)g.n + 1));
    int64_t *lowstart = (int64_t *)p;
    p += al(8 * ((size_t)g.n + 1));
    char *sum_ws = p;
    p += al(exclusive_sum_ws_bytes(g.n));
    uint64_t *key = (uint64_t *)p;
    p += al(8 * (size_t)cap);
    uint64_t *kout = (uint64_t *)p;
    p += al(8 * (size_t)cap);
    uint32_t *val = (uint32_t *)p;
    p += al(4 * (size_t)cap);
    uint32_t *vout = (uint32_t *)p;
    p += al(4 * (size_t)cap);
    char *rs_ws = p;
    int shift = 1;
    while (shift < 31 && ((int64_t)1 << shift) < (int64_t)g.n) ++shift;
    {
        KAPPA_PROF("validate_sorted", s);
        hipLaunchKernelGGL(val_low_k, dim3(grid_for(g.n, BLOCK, 4096)), dim3(BLOCK), 0, s, g, flags,
                           low);
        exclusive_sum_i64(low, lowstart, g.n, sum_ws, s);
        hipLaunchKernelGGL(val_upper_k, dim3(grid_for(nt, 1, 8192)), dim3(BLOCK), 0, s, g, tile_row,
                           flags, low, lowstart, shift, cap, key, val);
        // the keys are written row by row, so those of one neighbour already
        // ascend by row: a stable sort by the neighbour bits alone orders them
        radix_sort_pairs<uint64_t>(key, kout, val, vout, cap, shift, 2 * shift, rs_ws, s);
        hipLaunchKernelGGL(val_match_k, dim3(grid_for(nt, 1, 8192)), dim3(BLOCK), 0, s, g, tile_row,
                           flags, low, lowstart, shift, cap, kout, vout);
    }
}

// ---------------------------------------------------------------------------
// Out(v) = sum of w over the edges at v (Section 3.1, innerOuter).  Row sums
// are gathered in LDS per tile, then added to out[] (zeroed first).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void out_body(const DevGraph &g, const int32_t *tile_row,
                                         uint32_t *out, int64_t *s_off, uint32_t *s_sum) {
    const int64_t ntiles = etiles(g.nnz);
    for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        TileCtx t = tile_begin(g, tile_row, tt, s_off);
        int32_t nr = t.r1 - t.r0 + 1;
        if (t.lds)
            for (int i = threadIdx.x; i < nr; i += blockDim.x) s_sum[i] = 0;
        __syncthreads();
        for (int i = 0; i < ETILE_ITEMS; ++i) {
            int64_t j = t.j0 + (int64_t)i * BLOCK + threadIdx.x;
            if (j >= t.j1) break;
            int32_t v = tile_row_of(g, t, s_off, j);
            if (t.lds) atomicAdd(&s_sum[v - t.r0], g.ew[j]);
            else atomicAdd(&out[v], g.ew[j]);
        }
        __syncthreads();
        if (t.lds)
            for (int i = threadIdx.x; i < nr; i += blockDim.x)
                if (s_sum[i]) atomicAdd(&out[t.r0 + i], s_sum[i]);
    }
}

__global__ void __launch_bounds__(BLOCK) out_k(DevGraph g, const int32_t *tile_row, uint32_t *out) {
    __shared__ int64_t s_off[ETILE_ROWS + 1];
    __shared__ uint32_t s_sum[ETILE_ROWS];
    out_body(g, tile_row, out, s_off, s_sum);
}

void launch_out(const DevGraph &g, const int32_t *tile_row, uint32_t *out, hipStream_t s) {
    launch_fill_u32(out, g.n, 0, s);
    int64_t nt = etiles(g.nnz);
    if (nt == 0) return;
    KAPPA_PROF("out", s);
    hipLaunchKernelGGL(out_k, dim3(grid_for(nt, 1, 8192)), dim3(BLOCK), 0, s, g, tile_row, out);
}

// Level-resident Out(v): level l's graph from its descriptor, only while it
// is matching.
__device__ __forceinline__ bool level_graph(const LevelDesc *L, int32_t want, DevGraph &g) {
    if (L->phase != want) return false;
    g.n = L->n; g.nnz = L->nnz; g.xadj = L->xadj; g.adj = L->adj; g.ew = L->ew; g.vw = L->vw;
    return true;
}

__global__ void lv_out_zero_k(const LevelDesc *L, uint32_t *out) {
    DevGraph g;
    if (!level_graph(L, PH_MATCH, g)) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = 0;
}
__global__ void lv_tile_rows_k(const LevelDesc *L, int32_t *tile_row) {
    DevGraph g;
    if (!level_graph(L, PH_MATCH, g)) return;
    tile_rows_body(g, tile_row);
}
__global__ void __launch_bounds__(BLOCK) lv_out_k(const LevelDesc *L, const int32_t *tile_row,
                                                  uint32_t *out) {
    __shared__ int64_t s_off[ETILE_ROWS + 1];
    __shared__ uint32_t s_sum[ETILE_ROWS];
    DevGraph g;
    if (!level_graph(L, PH_MATCH, g)) return;
    out_body(g, tile_row, out, s_off, s_sum);
}

void launch_level_out(const Ctx &c, int l, int64_t nnz_cap, int32_t n_hint, hipStream_t s) {
    const LevelDesc *L = c.lv + l;
    {
        KAPPA_PROF("out_zero", s);
        hipLaunchKernelGGL(lv_out_zero_k, dim3(grid_for(n_hint, BLOCK * 4, 1024)), dim3(BLOCK), 0, s,
                           L, c.ms.out);
    }
    {
        KAPPA_PROF("tile_rows", s);
        hipLaunchKernelGGL(lv_tile_rows_k, dim3(grid_for(n_hint, BLOCK, 4096)), dim3(BLOCK), 0, s,
                           L, c.ms.tile_row);
    }
    KAPPA_PROF("out", s);
    int64_t nt_hint = etiles(nnz_cap);
    hipLaunchKernelGGL(lv_out_k, dim3(grid_for(nt_hint, 1, 8192)), dim3(BLOCK), 0, s, L,
                       c.ms.tile_row, c.ms.out);
}

// ---------------------------------------------------------------------------
// Ratings of every entry (Section 3.1).
// ---------------------------------------------------------------------------
template <int R>
__global__ void __launch_bounds__(BLOCK) rate_k(DevGraph g, const int32_t *tile_row,
                                                const uint32_t *out, uint64_t *num,
                                                uint64_t *den) {
    __shared__ int64_t s_off[ETILE_ROWS + 1];
    const int64_t ntiles = etiles(g.nnz);
    for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        TileCtx t = tile_begin(g, tile_row, tt, s_off);
        for (int i = 0; i < ETILE_ITEMS; ++i) {
            int64_t j = t.j0 + (int64_t)i * BLOCK + threadIdx.x;
            if (j >= t.j1) break;
            int32_t v = tile_row_of(g, t, s_off, j);
            int32_t u = g.adj[j];
            uint32_t ou = 0, ov = 0;
            if (R == KAPPA_INNER_OUTER) { ou = out[u]; ov = out[v]; }
            uint64_t a, b;
            rate<R>(g.ew[j], g.vw[u], g.vw[v], ou, ov, a, b);
            num[j] = a;
            den[j] = b;
        }
    }
}

void launch_rate(const DevGraph &g, const int32_t *tr, int rating, const uint32_t *out,
                 uint64_t *num, uint64_t *den, hipStream_t s) {
    int64_t nt = etiles(g.nnz);
    if (nt == 0) return;
    KAPPA_PROF("rate", s);
    dim3 gr(grid_for(nt, 1, 8192)), bl(BLOCK);
    switch (rating) {
    case KAPPA_INNER_OUTER: hipLaunchKernelGGL(rate_k<KAPPA_INNER_OUTER>, gr, bl, 0, s, g, tr, out, num, den); break;
    case KAPPA_WEIGHT: hipLaunchKernelGGL(rate_k<KAPPA_WEIGHT>, gr, bl, 0, s, g, tr, out, num, den); break;
    case KAPPA_EXPANSION: hipLaunchKernelGGL(rate_k<KAPPA_EXPANSION>, gr, bl, 0, s, g, tr, out, num, den); break;
    case KAPPA_EXPANSION_STAR: hipLaunchKernelGGL(rate_k<KAPPA_EXPANSION_STAR>, gr, bl, 0, s, g, tr, out, num, den); break;
    default: hipLaunchKernelGGL(rate_k<KAPPA_EXPANSION_STAR2>, gr, bl, 0, s, g, tr, out, num, den); break;
    }
}

// ---------------------------------------------------------------------------
// Matching check for externally supplied mate arrays.
// ---------------------------------------------------------------------------
__global__ void check_matching_k(DevGraph g, const int32_t *mate, uint32_t *flags) {
    bool bad = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t m = mate[v];
        if (m == -1) continue;
        if (m < 0 || m >= g.n || m == v || mate[m] != v) { bad = true; continue; }
        int64_t lo = g.xadj[v], hi = g.xadj[v + 1] - 1;
        bool found = false;
        while (lo <= hi) {
            int64_t mid = (lo + hi) >> 1;
            int32_t x = g.adj[mid];
            if (x == m) { found = true; break; }
            if (x < m) lo = mid + 1; else hi = mid - 1;
        }
        if (!found) bad = true;
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(flags, 1u);
}

void launch_check_matching(const DevGraph &g, const int32_t *mate, uint32_t *flags,
                           hipStream_t s) {
    if (g.n <= 0) return;
    KAPPA_PROF("check_matching", s);
    hipLaunchKernelGGL(check_matching_k, dim3(grid_for(g.n, BLOCK, 4096)), dim3(BLOCK), 0, s, g,
                       mate, flags);
}

// ---------------------------------------------------------------------------
// Initial partition stand-in and projection (Section 2, uncontraction).
// ---------------------------------------------------------------------------
__global__ void initial_partition_k(int32_t n, int32_t k, uint64_t seed, int32_t *part) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        part[x] = (int32_t)(mix64(seed + (uint64_t)x) % (uint64_t)k);
}

void launch_initial_partition(int32_t n, int32_t k, uint64_t seed, int32_t *part,
                              hipStream_t s) {
    if (n <= 0) return;
    KAPPA_PROF("initial_partition", s);
    hipLaunchKernelGGL(initial_partition_k, dim3(grid_for(n, BLOCK, 4096)), dim3(BLOCK), 0, s, n,
                       k, seed, part);
}

__global__ void project_k(const int32_t *cmap, int32_t n_fine, int32_t n_coarse,
                          const int32_t *part_coarse, int32_t *part_fine, uint32_t *flag) {
    bool bad = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_fine;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = cmap[v];
        if (c < 0 || c >= n_coarse) {
            part_fine[v] = -1;
            bad = true;
        } else {
            part_fine[v] = part_coarse[c];
        }
    }
    if (__ballot(bad) && lane_id() == 0 && flag) atomicOr(flag, 1u);
}

void launch_project(const int32_t *cmap, int32_t n_fine, int32_t n_coarse,
                    const int32_t *part_coarse, int32_t *part_fine, uint32_t *flag,
                    hipStream_t s) {
    if (n_fine <= 0) return;
    KAPPA_PROF("project", s);
    hipLaunchKernelGGL(project_k, dim3(grid_for(n_fine, BLOCK * 4, 2048)), dim3(BLOCK), 0, s, cmap,
                       n_fine, n_coarse, part_coarse, part_fine, flag);
}

// ---------------------------------------------------------------------------
// One level of the way back up (Section 2: uncontraction, then cut and
// balance; imbalance of Section 5.2), two kernels.
//   up_nodes:   the level's partition (projected through cmap, or the
//               stand-in initial partition, or given), block weights in an
//               LDS histogram, c(V) and max c(v), the entry tiles' rows
//   up_entries: the cut over entry tiles; the last block to finish sums the
//               shards, writes the result and clears the accumulators for
//               the next level
// Accumulators (zero on entry, zero again on exit): bw[BW_SHARDS][k],
// acc[3][NSHARD] (cut, c(V), max c(v)), arrive[ARRIVE_WORDS].
// flag bit 0: a map entry out of range; bit 1: a block id out of range.
// ---------------------------------------------------------------------------
constexpr int UP_NODE_BLOCKS = 512;

__global__ void __launch_bounds__(BLOCK) up_nodes_k(DevGraph g, int mode, const int32_t *cmap,
                                                    int32_t n_coarse, const int32_t *part_c,
                                                    uint64_t part_seed, int32_t *part, int32_t k,
                                                    int32_t *tile_row, uint64_t *bw, uint64_t *acc,
                                                    uint32_t *flag) {
    extern __shared__ uint64_t s_hist[];   // k entries
    __shared__ uint64_t sh[BLOCK / WAVE + 1];
    __shared__ uint32_t shm[BLOCK / WAVE];
    for (int i = threadIdx.x; i < k; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    const int64_t ntiles = etiles(g.nnz);
    uint64_t tot = 0;
    uint32_t mx = 0, bad = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t p;
        if (mode == UP_PROJECT) {
            const int32_t cx = cmap[v];
            if (cx < 0 || cx >= n_coarse) {
                p = -1;
                bad |= 1u;
            } else {
                p = part_c[cx];
            }
            part[v] = p;
        } else if (mode == UP_INITIAL) {
            p = (int32_t)(mix64(part_seed + (uint64_t)v) % (uint64_t)k);
            part[v] = p;
        } else {
            p = part[v];
        }
        const uint32_t c = g.vw[v];
        if (p < 0 || p >= k) {
            bad |= 2u;
        } else if (c) {
            atomicAdd((unsigned long long *)&s_hist[p], (unsigned long long)c);
        }
        tot += c;
        mx = c > mx ? c : mx;
        const int64_t b = g.xadj[v], e = g.xadj[v + 1];
        for (int64_t t = (b + ETILE - 1) / ETILE; t * ETILE < e && t < ntiles; ++t)
            tile_row[t] = (int32_t)v;
    }
    __syncthreads();
    uint64_t *bws = bw + (int64_t)(blockIdx.x % BW_SHARDS) * k;
    for (int i = threadIdx.x; i < k; i += blockDim.x)
        if (s_hist[i]) atomicAdd((unsigned long long *)&bws[i], (unsigned long long)s_hist[i]);
    tot = block_sum(tot, sh);
    mx = wave_max(mx);
    if (lane_id() == 0) shm[threadIdx.x / WAVE] = mx;
    for (int o = WAVE / 2; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, WAVE);
    if (bad && lane_id() == 0) atomicOr(flag, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int sd = shard_of_block();
        for (int i = 1; i < BLOCK / WAVE; ++i) mx = shm[i] > mx ? shm[i] : mx;
        if (tot) atomicAdd((unsigned long long *)&acc[1 * NSHARD + sd], (unsigned long long)tot);
        if (mx) atomicMax((unsigned long long *)&acc[2 * NSHARD + sd], (unsigned long long)mx);
    }
}

typedef unsigned __int128 u128;

// The sums, the exact L_max test, and cleared accumulators (one block, all
// threads call; the accumulators' writers have finished).
__device__ __forceinline__ void up_finalize(int32_t k, uint32_t eps_num, uint32_t eps_den,
                                            uint64_t *bw, uint64_t *acc, uint64_t *block_w_out,
                                            kappa_cut_result *res, uint64_t *sh, uint64_t *s_acc) {
    static_assert(BLOCK / WAVE >= 3 && NSHARD == WAVE, "one wave per sharded accumulator");
    uint64_t mxb = 0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        uint64_t part_w[BW_SHARDS];
#pragma unroll
        for (int q = 0; q < BW_SHARDS; ++q)
            part_w[q] = __hip_atomic_load(&bw[(int64_t)q * k + i], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        uint64_t w = 0;
#pragma unroll
        for (int q = 0; q < BW_SHARDS; ++q) {
            w += part_w[q];
            bw[(int64_t)q * k + i] = 0;
        }
        if (block_w_out) block_w_out[i] = w;
        mxb = w > mxb ? w : mxb;
    }
    mxb = wave_max(mxb);
    {
        const int w = threadIdx.x / WAVE;
        if (w < 3) {
            uint64_t *p = &acc[w * NSHARD + lane_id()];
            uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *p = 0;
            v = w == 2 ? wave_max(v) : wave_sum(v);
            if (lane_id() == 0) s_acc[w] = v;
        }
    }
    if (lane_id() == 0) sh[threadIdx.x / WAVE] = mxb;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < BLOCK / WAVE; ++i) mxb = sh[i] > mxb ? sh[i] : mxb;
    const uint64_t total = s_acc[1], maxc = s_acc[2];
    // L_max = (1 + eps) c(V) / k + max c(v) = lnum / lden, lden = k * eps_den
    const u128 lnum =
        (u128)((uint64_t)eps_den + eps_num) * total + (u128)((uint64_t)k * eps_den) * maxc;
    const u128 lden = (u128)k * eps_den;
    const u128 lhs = lden * mxb;
    res->cut = s_acc[0];
    res->total = total;
    res->max_block = mxb;
    res->max_node = maxc;
    res->lmax_num = (uint64_t)lnum;
    res->lmax_den = (uint64_t)lden;
    res->imb_num = lhs > lnum ? (uint64_t)(lhs - lnum) : 0;
    res->bal_num = (uint64_t)k * mxb;
    res->bal_den = total;
    res->feasible = lhs <= lnum ? 1 : 0;
}

// LAST: the block that finishes last finalizes (small grids); otherwise
// up_finalize_k runs next (a release per block costs more on large grids).
template <bool LAST>
__global__ void __launch_bounds__(BLOCK) up_entries_k(DevGraph g, const int32_t *tile_row,
                                                      const int32_t *part, int32_t k,
                                                      uint32_t eps_num, uint32_t eps_den,
                                                      uint64_t *bw, uint64_t *acc, unsigned *arrive,
                                                      uint64_t *block_w_out,
                                                      kappa_cut_result *res) {
    __shared__ int64_t s_off[ETILE_ROWS + 1];
    __shared__ uint64_t sh[BLOCK / WAVE + 1];
    __shared__ uint64_t s_acc[3];
    __shared__ int last;
    const int64_t ntiles = etiles(g.nnz);
    uint64_t cut = 0;
    for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        TileCtx t = tile_begin(g, tile_row, tt, s_off);
        int32_t vv[ETILE_ITEMS], uu[ETILE_ITEMS];
        uint32_t ww[ETILE_ITEMS];
#pragma unroll
        for (int i = 0; i < ETILE_ITEMS; ++i) {
            const int64_t j = t.j0 + (int64_t)i * BLOCK + threadIdx.x;
            uu[i] = -1;
            vv[i] = 0;
            ww[i] = 0;
            if (j < t.j1) {
                vv[i] = tile_row_of(g, t, s_off, j);
                uu[i] = g.adj[j];
                ww[i] = g.ew[j];
            }
        }
#pragma unroll
        for (int i = 0; i < ETILE_ITEMS; ++i)
            if (uu[i] > vv[i] && part[uu[i]] != part[vv[i]]) cut += ww[i];
    }
    cut = block_sum(cut, sh);
    if (threadIdx.x == 0 && cut)
        atomicAdd((unsigned long long *)&acc[shard_of_block()], (unsigned long long)cut);
    if (!LAST) return;
    __syncthreads();
    if (threadIdx.x == 0) last = arrive_last(arrive);
    __syncthreads();
    if (!last) return;
    up_finalize(k, eps_num, eps_den, bw, acc, block_w_out, res, sh, s_acc);
}

__global__ void __launch_bounds__(BLOCK) up_finalize_k(int32_t k, uint32_t eps_num,
                                                       uint32_t eps_den, uint64_t *bw,
                                                       uint64_t *acc, uint64_t *block_w_out,
                                                       kappa_cut_result *res) {
    __shared__ uint64_t sh[BLOCK / WAVE + 1];
    __shared__ uint64_t s_acc[3];
    up_finalize(k, eps_num, eps_den, bw, acc, block_w_out, res, sh, s_acc);
}

constexpr unsigned UP_LAST_BLOCKS = 64;   // grids up to this size finalize in their last block

void launch_up_level(const DevGraph &g, int mode, const int32_t *cmap, int32_t n_coarse,
                     const int32_t *part_c, uint64_t part_seed, int32_t *part, int32_t k,
                     uint32_t eps_num, uint32_t eps_den, int32_t *tile_row, const UpAcc &a,
                     uint64_t *block_w_out, kappa_cut_result *res, hipStream_t s) {
    {
        KAPPA_PROF("up_nodes", s);
        hipLaunchKernelGGL(up_nodes_k, dim3(grid_for(g.n, BLOCK * 4, UP_NODE_BLOCKS)), dim3(BLOCK),
                           (size_t)k * sizeof(uint64_t), s, g, mode, cmap, n_coarse, part_c,
                           part_seed, part, k, tile_row, a.bw, a.acc, a.flag);
    }
    const unsigned grid = grid_for(etiles(g.nnz), 1, ARRIVE_MAX_BLOCKS);
    if (grid <= UP_LAST_BLOCKS) {
        KAPPA_PROF("up_entries", s);
        hipLaunchKernelGGL(up_entries_k<true>, dim3(grid), dim3(BLOCK), 0, s, g, tile_row, part, k,
                           eps_num, eps_den, a.bw, a.acc, a.arrive, block_w_out, res);
        return;
    }
    {
        KAPPA_PROF("up_entries", s);
        hipLaunchKernelGGL(up_entries_k<false>, dim3(grid), dim3(BLOCK), 0, s, g, tile_row, part,
                           k, eps_num, eps_den, a.bw, a.acc, a.arrive, block_w_out, res);
    }
    KAPPA_PROF("up_finalize", s);
    hipLaunchKernelGGL(up_finalize_k, dim3(1), dim3(BLOCK), 0, s, k, eps_num, eps_den, a.bw, a.acc,
                       block_w_out, res);
}

void launch_up_clear(const UpAcc &a, int32_t k, hipStream_t s) {
    ZeroRanges z;
    z.add(a.bw, (int64_t)BW_SHARDS * k * 2);
    z.add(a.acc, 3 * NSHARD * 2);
    z.add(a.arrive, ARRIVE_WORDS);
    z.add(a.flag, 1);
    launch_zero(z, s);
}

}  // namespace kappa
