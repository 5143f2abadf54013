// k_contract.hip -- contraction of a matching (Section 2).
//
// Each matched pair {u, v} becomes one coarse node x with c(x) = c(u) + c(v);
// the rows of u and v are merged: neighbours are renamed to coarse ids,
// the contracted edge itself is dropped, and parallel edges are merged with
// summed weight.  Coarse ids: representatives (unmatched nodes and the smaller
// end of each matched edge) numbered in ascending fine id by a device scan.
//
// Steps:
//   1. scan of the representative flags -> cmap of representatives, rep_of
//   2. coarse_nodes: c(x), cmap of partners, bound(x) = deg(u) + deg(v) - 2,
//      row class by bound
//   3. scan of the bounds -> padded row offsets
//   4. merge of each coarse row into the padded buffer, by class:
//        small (<= 64 entries): 16 lanes per row, rank sort in LDS
//        mid (<= 4094):         one block per row, bitonic sort in LDS
//        large:                 dense per-slot accumulator + bitmap, read
//                               back in ascending id order
//      Equal coarse neighbours form runs of at most 4 entries (a coarse node
//      has at most two fine nodes on each side).
//   5. scan of the merged degrees -> coarse row offsets
//   6. compact: copy merged rows into the exact-size coarse arrays
#include "kappa_internal.h"

namespace kappa {

constexpr uint32_t INVALID_KEY = 0xffffffffu;
constexpr int SM_ROWS = BLOCK / ROW_SMALL_G;      // 16 small rows per block
constexpr int SM_CAP = ROW_SMALL_MAX + 2;        // entries incl. the dropped edge
constexpr int MID_P = 4096;

__device__ __forceinline__ int64_t nc_of(const int64_t *totals) { return totals[0]; }

// --- 1. representatives ---------------------------------------------------
struct RepF {
    const int32_t *mate;
    __device__ int64_t operator()(int64_t i) const {
        int32_t m = mate[i];
        return (m < 0 || i < m) ? 1 : 0;
    }
};
struct RepW {
    int32_t *cmap;
    int32_t *rep_of;
    __device__ void operator()(int64_t i, int64_t pre, int64_t v) const {
        if (v) {
            cmap[i] = (int32_t)pre;
            rep_of[pre] = (int32_t)i;
        }
    }
};

// --- 2. coarse nodes --------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) coarse_nodes_k(DevGraph g, const int32_t *mate,
                                                        int32_t *cmap, const int32_t *rep_of,
                                                        uint32_t *cvw, int32_t *cdeg,
                                                        int32_t *rows, int32_t *row_cnt,
                                                        const int64_t *totals) {
    int64_t nc = nc_of(totals);
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t wb0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1));
    for (int64_t wb = wb0; wb < nc; wb += stride) {
        int64_t x = wb + lane_id();
        int cls = -1;
        if (x < nc) {
            int32_t u = rep_of[x];
            int32_t w = mate[u];
            uint32_t c = g.vw[u];
            int64_t bnd = g.xadj[u + 1] - g.xadj[u];
            if (w >= 0) {
                cmap[w] = (int32_t)x;
                c += g.vw[w];
                bnd += g.xadj[w + 1] - g.xadj[w] - 2;
            }
            cvw[x] = c;
            cdeg[x] = (int32_t)bnd;
            cls = bnd == 0 ? -1 : (bnd <= ROW_SMALL_MAX ? 0 : (bnd <= ROW_MID_MAX ? 1 : 2));
        }
        wave_append(cls == 0, (int32_t)x, rows, &row_cnt[0]);
        wave_append(cls == 1, (int32_t)x, rows + g.n, &row_cnt[1]);
        wave_append(cls == 2, (int32_t)x, rows + 2 * (int64_t)g.n, &row_cnt[2]);
    }
}

// --- 3./5. scans over coarse rows ---------------------------------------------
struct DegF {
    const int32_t *deg;
    const int64_t *totals;
    __device__ int64_t operator()(int64_t i) const { return i < totals[0] ? deg[i] : 0; }
};
struct OffW {
    int64_t *off;
    const int64_t *totals;
    __device__ void operator()(int64_t i, int64_t pre, int64_t) const {
        if (i <= totals[0]) off[i] = pre;
    }
};

// The fine entries of coarse row x: row u, then row w (partner), each without
// the contracted edge.  t-th entry -> (coarse key, weight); INVALID_KEY for
// the contracted edge.
struct RowSrc {
    int32_t u, w;
    int64_t bu, du, bw;
    int64_t tot;
};
__device__ __forceinline__ RowSrc row_src(const DevGraph &g, const int32_t *mate,
                                          const int32_t *rep_of, int32_t x) {
    RowSrc r;
    r.u = rep_of[x];
    r.w = mate[r.u];
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

// --- 4a. small rows: 16 lanes per row, rank sort ------------------------------
__global__ void __launch_bounds__(BLOCK) fill_small_k(DevGraph g, const int32_t *mate,
                                                      const int32_t *cmap, const int32_t *rep_of,
                                                      const int64_t *tmp_off, int32_t *cdeg,
                                                      const int32_t *rows, const int32_t *row_cnt,
                                                      int32_t *tmp_adj, uint32_t *tmp_ew,
                                                      int64_t *totals) {
    __shared__ uint32_t sk[SM_ROWS][SM_CAP];
    __shared__ uint32_t sw[SM_ROWS][SM_CAP];
    __shared__ uint8_t sf[SM_ROWS][SM_CAP];
    const int grp = threadIdx.x / ROW_SMALL_G, sub = threadIdx.x % ROW_SMALL_G;
    const int64_t count = row_cnt[0];
    const int64_t gs = (int64_t)gridDim.x * SM_ROWS;
    const int64_t lim = (count + gs - 1) / gs * gs;
    int32_t dmax = 0;
    for (int64_t i = (int64_t)blockIdx.x * SM_ROWS + grp; i < lim; i += gs) {
        bool live = i < count;
        int32_t x = live ? rows[i] : 0;
        RowSrc r;
        r.tot = 0;
        if (live) r = row_src(g, mate, rep_of, x);
        for (int64_t t = sub; t < r.tot; t += ROW_SMALL_G) {
            uint32_t k, w;
            row_entry(g, cmap, r, t, k, w);
            sk[grp][t] = k;
            sw[grp][t] = w;
        }
        __syncthreads();
        int tot = (int)r.tot;
        for (int t = sub; t < tot; t += ROW_SMALL_G) {
            uint32_t k = sk[grp][t];
            bool lead = k != INVALID_KEY;
            for (int q = 0; q < t && lead; ++q) lead = sk[grp][q] != k;
            sf[grp][t] = lead;
        }
        __syncthreads();
        int nl = 0;
        int64_t off = live ? tmp_off[x] : 0;
        for (int t = sub; t < tot; t += ROW_SMALL_G) {
            if (!sf[grp][t]) continue;
            uint32_t k = sk[grp][t];
            int rank = 0;
            uint32_t sum = 0;
            for (int q = 0; q < tot; ++q) {
                uint32_t kq = sk[grp][q];
                rank += (sf[grp][q] && kq < k) ? 1 : 0;
                sum += kq == k ? sw[grp][q] : 0u;
            }
            tmp_adj[off + rank] = (int32_t)k;
            tmp_ew[off + rank] = sum;
            ++nl;
        }
        for (int o = ROW_SMALL_G / 2; o > 0; o >>= 1) nl += __shfl_xor(nl, o, ROW_SMALL_G);
        if (live && sub == 0) {
            cdeg[x] = nl;
            dmax = nl > dmax ? nl : dmax;
        }
        __syncthreads();
    }
    dmax = wave_max(dmax);
    if (lane_id() == 0 && dmax) atomicMax((unsigned long long *)&totals[3], (unsigned long long)dmax);
}

// --- 4b. mid rows: one block per row, bitonic sort in LDS -------------------------
__global__ void __launch_bounds__(BLOCK) fill_mid_k(DevGraph g, const int32_t *mate,
                                                    const int32_t *cmap, const int32_t *rep_of,
                                                    const int64_t *tmp_off, int32_t *cdeg,
                                                    const int32_t *rows, const int32_t *row_cnt,
                                                    int32_t *tmp_adj, uint32_t *tmp_ew,
                                                    int64_t *totals) {
    __shared__ uint64_t s[MID_P];
    __shared__ int64_t sh[BLOCK / WAVE + 1];
    const int64_t count = row_cnt[1];
    int32_t dmax = 0;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        int32_t x = rows[g.n + i];
        RowSrc r = row_src(g, mate, rep_of, x);
        int tot = (int)r.tot;
        int P = 2;
        while (P < tot) P <<= 1;
        for (int t = threadIdx.x; t < P; t += BLOCK) {
            uint64_t val = ~0ull;
            if (t < tot) {
                uint32_t k, w;
                row_entry(g, cmap, r, t, k, w);
                val = ((uint64_t)k << 32) | w;
            }
            s[t] = val;
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = threadIdx.x; t < P; t += BLOCK) {
                    int ixj = t ^ j;
                    if (ixj > t) {
                        uint64_t a = s[t], b = s[ixj];
                        bool up = (t & k) == 0;
                        if ((a > b) == up) { s[t] = b; s[ixj] = a; }
                    }
                }
                __syncthreads();
            }
        }
        // leaders: first entry of each run of equal keys
        const int ipt = (P + BLOCK - 1) / BLOCK;
        const int t0 = threadIdx.x * ipt;
        int64_t mine = 0;
        for (int q = 0; q < ipt; ++q) {
            int t = t0 + q;
            if (t >= P) break;
            uint32_t k = (uint32_t)(s[t] >> 32);
            if (k != INVALID_KEY && (t == 0 || (uint32_t)(s[t - 1] >> 32) != k)) ++mine;
        }
        int64_t total;
        int64_t rank = block_excl_scan(mine, sh, &total);
        int64_t off = tmp_off[x];
        for (int q = 0; q < ipt; ++q) {
            int t = t0 + q;
            if (t >= P) break;
            uint32_t k = (uint32_t)(s[t] >> 32);
            if (k == INVALID_KEY || (t > 0 && (uint32_t)(s[t - 1] >> 32) == k)) continue;
            uint32_t sum = 0;
            for (int e = t; e < P && (uint32_t)(s[e] >> 32) == k; ++e) sum += (uint32_t)s[e];
            tmp_adj[off + rank] = (int32_t)k;
            tmp_ew[off + rank] = sum;
            ++rank;
        }
        if (threadIdx.x == 0) {
            cdeg[x] = (int32_t)total;
            dmax = (int32_t)total > dmax ? (int32_t)total : dmax;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && dmax) atomicMax((unsigned long long *)&totals[3], (unsigned long long)dmax);
}

// --- 4c. large rows: dense accumulator per slot --------------------------------------
__global__ void __launch_bounds__(BLOCK) fill_large_k(DevGraph g, const int32_t *mate,
                                                      const int32_t *cmap, const int32_t *rep_of,
                                                      const int64_t *tmp_off, int32_t *cdeg,
                                                      const int32_t *rows, const int32_t *row_cnt,
                                                      int32_t *tmp_adj, uint32_t *tmp_ew,
                                                      uint32_t *hub_acc, uint32_t *hub_bits,
                                                      int64_t hub_words, int64_t *totals) {
    __shared__ int64_t s_wcnt[BLOCK / WAVE + 1];
    uint32_t *acc = hub_acc + (int64_t)blockIdx.x * g.n;
    uint32_t *bits = hub_bits + (int64_t)blockIdx.x * hub_words;
    const int64_t nc = nc_of(totals);
    const int64_t nwords = (nc + 31) / 32;
    const int64_t count = row_cnt[2];
    const int nw = BLOCK / WAVE, wv = threadIdx.x / WAVE;
    const int64_t span = (nwords + nw - 1) / nw;
    const int64_t lo = wv * span, hi = lo + span < nwords ? lo + span : nwords;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        int32_t x = rows[2 * (int64_t)g.n + i];
        RowSrc r = row_src(g, mate, rep_of, x);
        for (int64_t t = threadIdx.x; t < r.tot; t += BLOCK) {
            uint32_t k, w;
            row_entry(g, cmap, r, t, k, w);
            if (k == INVALID_KEY) continue;
            atomicAdd(&acc[k], w);
            atomicOr(&bits[k >> 5], 1u << (k & 31));
        }
        __threadfence();
        __syncthreads();
        // pass 1: set bits per wave range (L1-bypassing loads)
        int64_t c = 0;
        for (int64_t q = lo + lane_id(); q < hi; q += WAVE)
            c += __popc(__hip_atomic_load(&bits[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        c = wave_sum(c);
        if (lane_id() == 0) s_wcnt[wv] = c;
        __syncthreads();
        int64_t base = 0, total = 0;
        for (int q = 0; q < nw; ++q) {
            if (q < wv) base += s_wcnt[q];
            total += s_wcnt[q];
        }
        // pass 2: ascending walk, read-and-clear bits and accumulators
        int64_t off = tmp_off[x];
        for (int64_t q0 = lo; q0 < hi; q0 += WAVE) {
            int64_t q = q0 + lane_id();
            uint32_t word = q < hi ? atomicExch(&bits[q], 0u) : 0u;
            int64_t pc = __popc(word);
            int64_t inc = wave_incl_scan(pc);
            int64_t pos = base + inc - pc;
            while (word) {
                int b = __ffs(word) - 1;
                word &= word - 1;
                uint32_t key = (uint32_t)(q * 32 + b);
                tmp_adj[off + pos] = (int32_t)key;
                tmp_ew[off + pos] = atomicExch(&acc[key], 0u);
                ++pos;
            }
            base += __shfl(inc, WAVE - 1, WAVE);
        }
        if (threadIdx.x == 0) {
            cdeg[x] = (int32_t)total;
            atomicMax((unsigned long long *)&totals[3], (unsigned long long)total);
        }
        __threadfence();
        __syncthreads();
    }
}

// --- 6. compaction ----------------------------------------------------------------
__global__ void __launch_bounds__(BLOCK) compact_small_k(const int32_t *rows, const int32_t *row_cnt,
                                                         const int64_t *tmp_off, const int32_t *cdeg,
                                                         const int64_t *cxadj, const int32_t *tmp_adj,
                                                         const uint32_t *tmp_ew, int32_t *cadj,
                                                         uint32_t *cew) {
    const int grp = threadIdx.x / ROW_SMALL_G, sub = threadIdx.x % ROW_SMALL_G;
    const int64_t count = row_cnt[0];
    for (int64_t i = (int64_t)blockIdx.x * SM_ROWS + grp; i < count;
         i += (int64_t)gridDim.x * SM_ROWS) {
        int32_t x = rows[i];
        int64_t src = tmp_off[x], dst = cxadj[x];
        int32_t len = cdeg[x];
        for (int t = sub; t < len; t += ROW_SMALL_G) {
            cadj[dst + t] = tmp_adj[src + t];
            cew[dst + t] = tmp_ew[src + t];
        }
    }
}

__global__ void __launch_bounds__(BLOCK) compact_big_k(const int32_t *rows, int32_t n_fine,
                                                       const int32_t *row_cnt,
                                                       const int64_t *tmp_off, const int32_t *cdeg,
                                                       const int64_t *cxadj, const int32_t *tmp_adj,
                                                       const uint32_t *tmp_ew, int32_t *cadj,
                                                       uint32_t *cew) {
    const int64_t c1 = row_cnt[1], c2 = row_cnt[2];
    for (int64_t i = blockIdx.x; i < c1 + c2; i += gridDim.x) {
        int32_t x = i < c1 ? rows[n_fine + i] : rows[2 * (int64_t)n_fine + (i - c1)];
        int64_t src = tmp_off[x], dst = cxadj[x];
        int32_t len = cdeg[x];
        for (int t = threadIdx.x; t < len; t += BLOCK) {
            cadj[dst + t] = tmp_adj[src + t];
            cew[dst + t] = tmp_ew[src + t];
        }
    }
}

// ---------------------------------------------------------------------------------
__global__ void contract_reset_k(int32_t *row_cnt, int64_t *totals) {
    if (threadIdx.x < 4) { row_cnt[threadIdx.x] = 0; totals[threadIdx.x] = 0; }
}

void launch_contract_build(const DevGraph &g, const int32_t *mate, int64_t max_bound,
                           int32_t *cmap, uint32_t *cvw, int64_t *cxadj, ContractScratch &cs,
                           hipStream_t s) {
    {
        KAPPA_PROF("contract_reset", s);
        hipLaunchKernelGGL(contract_reset_k, dim3(1), dim3(WAVE), 0, s, cs.row_cnt, cs.totals);
    }
    if (g.n <= 0) {
        launch_scan((int64_t)1, DegF{cs.cdeg, cs.totals}, OffW{cxadj, cs.totals}, cs.partials,
                    cs.totals + 2, s);
        return;
    }
    launch_scan((int64_t)g.n, RepF{mate}, RepW{cmap, cs.rep_of}, cs.partials, cs.totals + 0, s);
    {
        KAPPA_PROF("coarse_nodes", s);
        hipLaunchKernelGGL(coarse_nodes_k, dim3(grid_for(g.n, BLOCK, 2048)), dim3(BLOCK), 0, s, g,
                           mate, cmap, cs.rep_of, cvw, cs.cdeg, cs.rows, cs.row_cnt, cs.totals);
    }
    launch_scan((int64_t)g.n + 1, DegF{cs.cdeg, cs.totals}, OffW{cs.tmp_off, cs.totals},
                cs.partials, cs.totals + 1, s);
    {
        KAPPA_PROF("fill_small", s);
        hipLaunchKernelGGL(fill_small_k, dim3(grid_for(g.n, SM_ROWS, 4096)), dim3(BLOCK), 0, s, g,
                           mate, cmap, cs.rep_of, cs.tmp_off, cs.cdeg, cs.rows, cs.row_cnt,
                           cs.tmp_adj, cs.tmp_ew, cs.totals);
    }
    if (max_bound > ROW_SMALL_MAX) {
        KAPPA_PROF("fill_mid", s);
        hipLaunchKernelGGL(fill_mid_k, dim3(grid_for(g.n, 1, 1024)), dim3(BLOCK), 0, s, g, mate,
                           cmap, cs.rep_of, cs.tmp_off, cs.cdeg, cs.rows, cs.row_cnt, cs.tmp_adj,
                           cs.tmp_ew, cs.totals);
    }
    if (max_bound > ROW_MID_MAX && cs.hub_acc) {
        KAPPA_PROF("fill_large", s);
        hipLaunchKernelGGL(fill_large_k, dim3(HUB_SLOTS), dim3(BLOCK), 0, s, g, mate, cmap,
                           cs.rep_of, cs.tmp_off, cs.cdeg, cs.rows, cs.row_cnt, cs.tmp_adj,
                           cs.tmp_ew, cs.hub_acc, cs.hub_bits, cs.hub_words, cs.totals);
    }
    launch_scan((int64_t)g.n + 1, DegF{cs.cdeg, cs.totals}, OffW{cxadj, cs.totals}, cs.partials,
                cs.totals + 2, s);
}

void launch_contract_compact(const ContractScratch &cs, int32_t n_fine, int64_t max_bound,
                             const int64_t *cxadj, int32_t *cadj, uint32_t *cew, hipStream_t s) {
    if (n_fine <= 0) return;
    {
        KAPPA_PROF("compact_small", s);
        hipLaunchKernelGGL(compact_small_k, dim3(grid_for(n_fine, SM_ROWS, 4096)), dim3(BLOCK), 0,
                           s, cs.rows, cs.row_cnt, cs.tmp_off, cs.cdeg, cxadj, cs.tmp_adj,
                           cs.tmp_ew, cadj, cew);
    }
    if (max_bound > ROW_SMALL_MAX) {
        KAPPA_PROF("compact_big", s);
        hipLaunchKernelGGL(compact_big_k, dim3(grid_for(n_fine, 1, 1024)), dim3(BLOCK), 0, s,
                           cs.rows, n_fine, cs.row_cnt, cs.tmp_off, cs.cdeg, cxadj, cs.tmp_adj,
                           cs.tmp_ew, cadj, cew);
    }
}

}  // namespace kappa
