// Pairwise refinement of a k-way partition (Section 5).
//
//   quotient:  Q has an edge {a, b} (a < b) when an edge of G joins blocks a
//              and b; a k x k bitmap built with LDS-aggregated ORs.
//   colouring: Q's edges in ascending (a, b) order, each taking the smallest
//              colour free at both ends (the sequential greedy colouring that
//              Section 5.1 parallelises); one workgroup, since each choice
//              depends on all earlier ones.  Pairs of one colour share no
//              block, so their local searches touch disjoint node sets and
//              disjoint block weights and run side by side.
//   collect:   per colour, the nodes of each pair's two blocks into one
//              region per pair (order inside a region does not matter).
//   fm:        one workgroup per pair of the colour.  Its two halves run the
//              two local searches of a local iteration (run seeds r = 0, 1)
//              in lockstep, one move per step: a reduction over the queued
//              nodes finds each queue's top under the strict order (gain,
//              then mix64(run_seed ^ v), then the smaller id), one lane picks
//              the queue (TopGain, MaxLoad when a block is overloaded) and
//              books the move, and the half updates the neighbours' gains
//              and queues (Section 5.2).  The better run is adopted; the
//              workgroup repeats local iterations until one improves nothing.
//              A run's first FM_QCAP queue entries live in LDS with everything
//              a move needs (gain, hash, id, side, c(v), row start and
//              degree), so a move touches memory only for the neighbours'
//              rows; later entries stay in memory with the same meaning.  A
//              moved node's entry is replaced by the last one, so the queue
//              holds only nodes that may still move.
//
// Every choice is a maximum under a strict total order, so the result does
// not depend on the order of reductions or of the region: it is bit-exact
// with the sequential definition.
#include <algorithm>

#include "kappa_internal.h"

namespace kappa {

constexpr int RQ_THREADS = 256;
constexpr int RC_ITEMS = 16;           // nodes per thread in collect
constexpr int FM_THREADS = 512;        // two halves of 256, one per run
constexpr int FM_HALF = FM_THREADS / 2;
constexpr int FM_WAVES = FM_HALF / WAVE;
constexpr int FM_QCAP = 2048;          // queue entries per run kept in LDS (the rest in memory)

__device__ __forceinline__ uint64_t run_seed_of(uint64_t seed, int32_t g, int32_t a, int32_t b,
                                                int32_t t, int32_t r) {
    uint64_t h = mix64(seed + (uint64_t)(uint32_t)g);
    h = mix64(h ^ (((uint64_t)(uint32_t)a << 32) | (uint32_t)b));
    return mix64(h + 2 * (uint64_t)(uint32_t)t + (uint64_t)(uint32_t)r);
}

// (gain, hash, id) above (gain, hash, id); id < 0 is "none", below all
__device__ __forceinline__ bool key_above(int64_t g1, uint64_t h1, int32_t v1, int64_t g2,
                                          uint64_t h2, int32_t v2) {
    if (v2 < 0) return v1 >= 0;
    if (v1 < 0) return false;
    if (g1 != g2) return g1 > g2;
    if (h1 != h2) return h1 > h2;
    return v1 < v2;
}

__device__ __forceinline__ bool state_below(int64_t i1, int64_t c1, int64_t i2, int64_t c2) {
    return i1 < i2 || (i1 == i2 && c1 < c2);
}

__device__ __forceinline__ int64_t pair_imb(int64_t w0, int64_t w1, int64_t S, int64_t L) {
    const int64_t x = S * (w0 > w1 ? w0 : w1) - L;
    return x > 0 ? x : 0;
}

// block weights and node counts, c(V), max c(v); flags a block id outside [0, k)
__global__ void __launch_bounds__(RQ_THREADS)
    ref_weights_k(const int32_t *__restrict__ part, const uint32_t *__restrict__ vw, int32_t n,
                  int32_t k, int64_t *bw, int32_t *bc, RefineCtl *ctl) {
    __shared__ unsigned long long s_w[REFINE_K_MAX];
    __shared__ int32_t s_c[REFINE_K_MAX];
    __shared__ unsigned long long s_tot, s_max;
    __shared__ uint32_t s_bad;
    for (int i = threadIdx.x; i < k; i += blockDim.x) { s_w[i] = 0; s_c[i] = 0; }
    if (threadIdx.x == 0) { s_tot = 0; s_max = 0; s_bad = 0; }
    __syncthreads();
    unsigned long long tot = 0, mx = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = part[v];
        const uint32_t c = vw[v];
        tot += c;
        mx = c > mx ? c : mx;
        if (p < 0 || p >= k) { s_bad = 1; continue; }
        atomicAdd(&s_w[p], (unsigned long long)c);
        atomicAdd(&s_c[p], 1);
    }
    atomicAdd(&s_tot, tot);
    atomicMax(&s_max, mx);
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        if (s_c[i]) {
            atomicAdd((unsigned long long *)&bw[i], s_w[i]);
            atomicAdd(&bc[i], s_c[i]);
        }
    }
    if (threadIdx.x == 0) {
        atomicAdd(&ctl->total, s_tot);
        atomicMax(&ctl->max_node, s_max);
        if (s_bad) atomicOr(&ctl->flags, 1u);
    }
}

// Q as a bitmap: row a, bit b for a < b
__global__ void __launch_bounds__(RQ_THREADS)
    ref_quotient_k(const int64_t *__restrict__ xadj, const int32_t *__restrict__ adj,
                   const int32_t *__restrict__ part, int32_t n, int32_t k,
                   unsigned long long *qbits) {
    __shared__ unsigned long long s_q[REFINE_K_MAX * REFINE_QW];
    const int qw = (k + 63) / 64;
    for (int i = threadIdx.x; i < k * qw; i += blockDim.x) s_q[i] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = part[v];
        if (a < 0 || a >= k) continue;   // reported by the weights pass
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            const int32_t b = part[adj[j]];
            if (a < b && b < k) atomicOr(&s_q[a * qw + (b >> 6)], 1ull << (b & 63));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k * qw; i += blockDim.x)
        if (s_q[i]) atomicOr(&qbits[i], s_q[i]);
}

// greedy edge colouring of Q; pairs sorted by colour (ascending (a, b) inside
// a colour) into cpairs, colour c at [col_off[c], col_off[c + 1])
__global__ void __launch_bounds__(RQ_THREADS)
    ref_colour_k(const unsigned long long *__restrict__ qbits, int32_t k, int32_t *tmp_pair,
                 int32_t *tmp_col, int32_t *cpairs, int32_t *col_off, int32_t *fill,
                 RefineCtl *ctl) {
    __shared__ unsigned long long s_used[REFINE_K_MAX * REFINE_CW];
    __shared__ int32_t s_cnt[REFINE_COLOURS + 1];
    const int qw = (k + 63) / 64;
    for (int i = threadIdx.x; i < k * REFINE_CW; i += blockDim.x) s_used[i] = 0;
    for (int i = threadIdx.x; i <= REFINE_COLOURS; i += blockDim.x) s_cnt[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = 0, ncol = 0;
        for (int32_t a = 0; a < k; ++a)
            for (int w = 0; w < qw; ++w) {
                unsigned long long bits = qbits[a * qw + w];
                while (bits) {
                    const int32_t b = w * 64 + __builtin_ctzll(bits);
                    bits &= bits - 1;
                    int32_t c = 0;
                    for (int x = 0; x < REFINE_CW; ++x) {
                        const unsigned long long fr = ~(s_used[a * REFINE_CW + x] |
                                                        s_used[b * REFINE_CW + x]);
                        if (fr) { c = x * 64 + __builtin_ctzll(fr); break; }
                    }
                    s_used[a * REFINE_CW + (c >> 6)] |= 1ull << (c & 63);
                    s_used[b * REFINE_CW + (c >> 6)] |= 1ull << (c & 63);
                    tmp_pair[m] = a | (b << 16);
                    tmp_col[m] = c;
                    ++s_cnt[c];
                    ++m;
                    ncol = c + 1 > ncol ? c + 1 : ncol;
                }
            }
        int32_t acc = 0;
        for (int32_t c = 0; c < ncol; ++c) {
            col_off[c] = acc;
            acc += s_cnt[c];
            s_cnt[c] = col_off[c];
        }
        col_off[ncol] = acc;
        for (int32_t i = 0; i < m; ++i) cpairs[s_cnt[tmp_col[i]]++] = tmp_pair[i];
        ctl->ncol = ncol;
        ctl->npairs = m;
    }
    __syncthreads();
    const int32_t m = ctl->npairs;
    for (int32_t i = threadIdx.x; i < m; i += blockDim.x) fill[i] = 0;
}

__global__ void __launch_bounds__(RQ_THREADS)
    ref_collect_k(const int32_t *__restrict__ part, int32_t n, int32_t k, int32_t c,
                  const int32_t *__restrict__ cpairs, const int32_t *__restrict__ col_off,
                  const int32_t *__restrict__ bc, int32_t *fill, int32_t *poff,
                  int32_t *region) {
    __shared__ int32_t s_map[REFINE_K_MAX];
    __shared__ int32_t s_off[REFINE_K_MAX / 2];
    __shared__ int32_t s_cnt[REFINE_K_MAX / 2];
    __shared__ int32_t s_base[REFINE_K_MAX / 2];
    const int32_t p0 = col_off[c], np = col_off[c + 1] - p0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) s_map[i] = -1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s_cnt[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        s_map[cpairs[p0 + i] & 0xffff] = i;
        s_map[cpairs[p0 + i] >> 16] = i;
    }
    if (threadIdx.x == 0) {
        int32_t off = 0;
        for (int32_t i = 0; i < np; ++i) {
            s_off[i] = off;
            off += bc[cpairs[p0 + i] & 0xffff] + bc[cpairs[p0 + i] >> 16];
            if (blockIdx.x == 0) poff[p0 + i] = s_off[i];
        }
    }
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * blockDim.x * RC_ITEMS;
    const int64_t hi = std::min<int64_t>(lo + (int64_t)blockDim.x * RC_ITEMS, n);
    for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        const int32_t j = s_map[part[v]];
        if (j >= 0) atomicAdd(&s_cnt[j], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        s_base[i] = s_cnt[i] ? atomicAdd(&fill[p0 + i], s_cnt[i]) : 0;
        s_cnt[i] = 0;
    }
    __syncthreads();
    for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        const int32_t j = s_map[part[v]];
        if (j < 0) continue;
        const int64_t pos = (int64_t)s_off[j] + s_base[j] + atomicAdd(&s_cnt[j], 1);
        if (pos < n) region[pos] = (int32_t)v;   // counts agree with part unless state is broken
    }
}

struct FmArgs {
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
    const int32_t *cpairs, *col_off, *poff, *fill;
    int64_t *bw;
    int32_t *bc;
    const int32_t *region;
    int32_t *dist;
    int64_t *gain;       // [2][n]
    uint8_t *status;     // [2][n]: 0 idle, 1 queued, 2 moved
    int32_t *qlist;      // [2][n] region-relative; entries from qcap on
    int32_t *mlog;       // [2][n] region-relative
    int32_t *slot;       // [2][n]: queue position of a queued node
    int32_t qcap;        // queue positions below qcap live in LDS (<= FM_QCAP)
    RefineCtl *ctl;
};

// per-run state of one local search, in LDS
constexpr int ROW_CHUNK = 8;

// the blocks and weights of row entries [e0, min(e0 + ROW_CHUNK, x1)): all
// neighbour loads first, then all block loads, so they overlap; entries past
// the row get block -1
__device__ __forceinline__ void row_chunk(const int32_t *adj, const uint32_t *ew,
                                          const int32_t *part, int64_t e0, int64_t x1,
                                          int32_t *pu, uint32_t *wu) {
    int32_t uu[ROW_CHUNK];
#pragma unroll
    for (int k = 0; k < ROW_CHUNK; ++k) {
        const bool in = e0 + k < x1;
        uu[k] = in ? adj[e0 + k] : -1;
        wu[k] = in ? ew[e0 + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < ROW_CHUNK; ++k) pu[k] = uu[k] >= 0 ? part[uu[k]] : -1;
}

// a finished search, published for the adoption
struct RunState {
    int64_t best_imb, best_cut, best_w[2];
    int32_t best_cnt[2], qn, m, kept;
};

// a thread's best queue entry of one block under (gain, hash, id)
struct Best {
    int64_t g = 0;
    uint64_t h = 0;
    int32_t v = -1, q = -1;
    __device__ __forceinline__ void offer(int64_t g2, uint64_t h2, int32_t v2, int32_t q2) {
        if (key_above(g2, h2, v2, g, h, v)) { g = g2; h = h2; v = v2; q = q2; }
    }
};

// the wave's best (gain, hash, id), carrying the queue position
// DPP lane moves inside a row of 16 lanes: quad_perm swaps of neighbours and
// of pairs, the mirror of each half-row, the mirror of the row.  Each pairs
// every lane with another, so after the four steps every lane holds its row's
// maximum.
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

template <int CTRL>
__device__ __forceinline__ int32_t dpp_i32(int32_t x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ void best_step_dpp(int64_t &g, uint64_t &h, int32_t &v, int32_t &q) {
    const int64_t g2 = (int64_t)(((uint64_t)(uint32_t)dpp_i32<CTRL>((int32_t)(g >> 32)) << 32) |
                                 (uint32_t)dpp_i32<CTRL>((int32_t)g));
    const uint64_t h2 = ((uint64_t)(uint32_t)dpp_i32<CTRL>((int32_t)(h >> 32)) << 32) |
                        (uint32_t)dpp_i32<CTRL>((int32_t)h);
    const int32_t v2 = dpp_i32<CTRL>(v), q2 = dpp_i32<CTRL>(q);
    if (key_above(g2, h2, v2, g, h, v)) { g = g2; h = h2; v = v2; q = q2; }
}

__device__ __forceinline__ void wave_best(int64_t &g, uint64_t &h, int32_t &v, int32_t &q) {
    best_step_dpp<DPP_XOR1>(g, h, v, q);
    best_step_dpp<DPP_XOR2>(g, h, v, q);
    best_step_dpp<DPP_HALF_MIRROR>(g, h, v, q);
    best_step_dpp<DPP_MIRROR>(g, h, v, q);
    for (int o = 16; o < WAVE; o <<= 1) {   // across rows
        const int64_t g2 = __shfl_xor(g, o);
        const uint64_t h2 = __shfl_xor(h, o);
        const int32_t v2 = __shfl_xor(v, o);
        const int32_t q2 = __shfl_xor(q, o);
        if (key_above(g2, h2, v2, g, h, v)) { g = g2; h = h2; v = v2; q = q2; }
    }
}

__global__ void __launch_bounds__(FM_THREADS) ref_fm_k(FmArgs A, int32_t gi, int32_t c) {
    __shared__ RunState rs[2];
    __shared__ int64_t s_wg[2][2][FM_WAVES];
    __shared__ uint64_t s_wh[2][2][FM_WAVES];
    __shared__ int32_t s_wv[2][2][FM_WAVES];
    __shared__ int32_t s_wq[2][2][FM_WAVES];
    // queue entries below qcap: gain, node, bit 0 side (1: block b), bit 1 moved
    // with c(v), the row start and the degree, so that a move needs no memory
    // access before the neighbours' rows
    __shared__ int64_t q_g[2][FM_QCAP];
    __shared__ int64_t q_x[2][FM_QCAP];
    __shared__ uint64_t q_h[2][FM_QCAP];   // mix64(run seed ^ node)
    __shared__ int32_t q_v[2][FM_QCAP];
    __shared__ uint32_t q_c[2][FM_QCAP];
    __shared__ int32_t q_d[2][FM_QCAP];
    __shared__ uint8_t q_s[2][FM_QCAP];
    __shared__ int32_t s_off, s_len, s_na, s_nb, s_nf, s_stop, s_pick, s_bc[2];
    __shared__ int32_t s_done[2], s_v[2], s_to[2], s_deg[2];
    __shared__ int64_t s_x0[2];
    __shared__ int64_t s_bw[2];
    __shared__ unsigned long long s_cut, s_bytes;
    const int32_t j = blockIdx.x, p = A.col_off[c] + j;
    const int32_t a = A.cpairs[p] & 0xffff, b = A.cpairs[p] >> 16;
    const int tid = threadIdx.x, r = tid / FM_HALF, lt = tid % FM_HALF;
    const int lane = lt % WAVE, wv = lt / WAVE;
    if (tid == 0) {
        s_bytes = 0;
        s_off = A.poff[p];
        s_bc[0] = A.bc[a];
        s_bc[1] = A.bc[b];
        s_bw[0] = A.bw[a];
        s_bw[1] = A.bw[b];
        s_len = s_bc[0] + s_bc[1];
    }
    __syncthreads();
    const int32_t off = s_off, len = s_len;
    if (A.fill[p] != len || (int64_t)off + len > A.n) {   // the region is not what the counts say
        if (tid == 0) atomicOr(&A.ctl->flags, 2u);
        return;
    }
    const int32_t *reg = A.region + off;
    const int64_t S = (int64_t)A.k * A.eps_den;
    const int64_t L = ((int64_t)A.eps_den + A.eps_num) * (int64_t)A.ctl->total +
                      S * (int64_t)A.ctl->max_node;
    int64_t *gain_r = A.gain + (size_t)r * A.n;
    uint8_t *st_r = A.status + (size_t)r * A.n;
    int32_t *q_r = A.qlist + (size_t)r * A.n + off;
    int32_t *m_r = A.mlog + (size_t)r * A.n + off;
    int32_t *sl_r = A.slot + (size_t)r * A.n;
    const int32_t qcap = A.qcap;
    int64_t *qg = q_g[r], *qx = q_x[r];
    uint64_t *qh = q_h[r];
    int32_t *qv = q_v[r], *qd = q_d[r];
    uint32_t *qcw = q_c[r];
    uint8_t *qs = q_s[r];

    unsigned long long ticks_init = 0, ticks_moves = 0, t0 = 0;
    // the BFS frontiers use the two move logs, which are free until the moves
    int32_t *fr[2] = {A.mlog + off, A.mlog + (size_t)A.n + off};
    for (int32_t t = 0; t < A.max_local; ++t) {
        if (tid == 0) {
            s_cut = 0; s_na = 0; s_nb = 0; s_nf = 0;
            rs[0].qn = rs[1].qn = 0;
            t0 = wall_clock64();
        }
        __syncthreads();
        // gains, boundary, cut and node counts of the current partition; the
        // boundary is the BFS's first frontier
        unsigned long long cut = 0, touched = 0;
        int32_t na = 0, nb = 0;
        for (int32_t i = tid; i < len; i += FM_THREADS) {
            const int32_t v = reg[i], pv = A.part[v];
            const int64_t x0 = A.xadj[v], x1 = A.xadj[v + 1];
            int64_t g = 0;
            bool bnd = false;
            // rows in chunks of ROW_CHUNK entries, each chunk's loads issued together
            for (int64_t e0 = x0; e0 < x1; e0 += ROW_CHUNK) {
                int32_t pu[ROW_CHUNK];
                uint32_t wu[ROW_CHUNK];
                row_chunk(A.adj, A.ew, A.part, e0, x1, pu, wu);
#pragma unroll
                for (int k = 0; k < ROW_CHUNK; ++k) {
                    if (pu[k] != a && pu[k] != b) continue;   // also the chunk's tail (-1)
                    if (pu[k] != pv) {
                        g += wu[k];
                        bnd = true;
                        if (pv == a) cut += wu[k];
                    } else {
                        g -= wu[k];
                    }
                }
            }
            A.gain[v] = g;
            A.gain[(size_t)A.n + v] = g;
            A.status[v] = 0;
            A.status[(size_t)A.n + v] = 0;
            A.dist[v] = bnd ? 0 : -1;
            if (bnd) fr[0][atomicAdd(&s_nf, 1)] = v;
            if (pv == a) ++na; else ++nb;
            touched += 40 + 12 * (unsigned long long)(x1 - x0);
        }
        atomicAdd(&s_bytes, touched);
        atomicAdd(&s_cut, cut);
        atomicAdd(&s_na, na);
        atomicAdd(&s_nb, nb);
        __syncthreads();
        // bounded BFS inside each block, one frontier per distance
        int32_t nf = s_nf;
        __syncthreads();   // every thread has read the count before the first step clears it
        for (int32_t d = 1; d <= A.depth && nf > 0; ++d) {
            const int32_t *cur = fr[(d - 1) & 1];
            int32_t *nxt = fr[d & 1];
            if (tid == 0) s_nf = 0;
            __syncthreads();
            for (int32_t i = tid; i < nf; i += FM_THREADS) {
                const int32_t v = cur[i], pv = A.part[v];
                const int64_t x1 = A.xadj[v + 1];
                for (int64_t e0 = A.xadj[v]; e0 < x1; e0 += ROW_CHUNK) {
                    int32_t uu[ROW_CHUNK], pu[ROW_CHUNK];
#pragma unroll
                    for (int k = 0; k < ROW_CHUNK; ++k) uu[k] = e0 + k < x1 ? A.adj[e0 + k] : -1;
#pragma unroll
                    for (int k = 0; k < ROW_CHUNK; ++k) pu[k] = uu[k] >= 0 ? A.part[uu[k]] : -1;
#pragma unroll
                    for (int k = 0; k < ROW_CHUNK; ++k)
                        if (pu[k] == pv && atomicCAS(&A.dist[uu[k]], -1, d) == -1)
                            nxt[atomicAdd(&s_nf, 1)] = uu[k];
                }
            }
            __syncthreads();
            nf = s_nf;
            __syncthreads();   // everyone has read the count before it is cleared
        }
        // both runs: queues start with the boundary
        const uint64_t rseed = run_seed_of(A.seed, gi, a, b, t, r);
        for (int32_t i = lt; i < len; i += FM_HALF) {
            const int32_t v = reg[i];
            if (A.dist[v] == 0) {
                st_r[v] = 1;
                const int32_t pos = atomicAdd(&rs[r].qn, 1);
                sl_r[v] = pos;
                if (pos < qcap) {
                    qv[pos] = v;
                    qg[pos] = gain_r[v];
                    qh[pos] = mix64(rseed ^ (uint64_t)(uint32_t)v);
                    qs[pos] = A.part[v] == b;
                    qx[pos] = A.xadj[v];
                    qd[pos] = (int32_t)(A.xadj[v + 1] - A.xadj[v]);
                    qcw[pos] = A.vw[v];
                } else {
                    q_r[pos] = v;
                }
            }
        }
        if (tid == 0) { s_done[0] = 0; s_done[1] = 0; }
        __syncthreads();
        const int64_t smaller = min(s_na, s_nb);
        const int64_t start_imb = pair_imb(s_bw[0], s_bw[1], S, L), start_cut = (int64_t)s_cut;
        // the state of a search, kept in the registers of its half's lane 0
        int64_t w0 = s_bw[0], w1 = s_bw[1], cur_cut = start_cut, best_imb = start_imb;
        int64_t best_cut = start_cut, bw0 = w0, bw1 = w1, since = 0;
        int32_t c0 = s_na, c1 = s_nb, bc0 = c0, bc1 = c1, m = 0, kept = 0;
        if (tid == 0) {
            const unsigned long long t1 = wall_clock64();
            ticks_init += t1 - t0;
            t0 = t1;
        }
        // the moves, both runs in lockstep
        for (;;) {
            if (s_done[0] && s_done[1]) break;
            const bool live = !s_done[r];
            Best b0, b1;   // the best queued node of block a and of block b
            if (live) {
                const int32_t qn = rs[r].qn, qc = min(qn, qcap);
                for (int32_t i = lt; i < qc; i += FM_HALF) {
                    const uint8_t st = qs[i];
                    if (st & 2) continue;
                    if (st & 1) b1.offer(qg[i], qh[i], qv[i], i);
                    else b0.offer(qg[i], qh[i], qv[i], i);
                }
                for (int32_t i = qcap + lt; i < qn; i += FM_HALF) {
                    const int32_t v = q_r[i];
                    if (st_r[v] != 1) continue;
                    const uint64_t h = mix64(rseed ^ (uint64_t)(uint32_t)v);
                    if (A.part[v] == b) b1.offer(gain_r[v], h, v, i);
                    else b0.offer(gain_r[v], h, v, i);
                }
            }
            wave_best(b0.g, b0.h, b0.v, b0.q);
            wave_best(b1.g, b1.h, b1.v, b1.q);
            if (lane == 0) {
                s_wg[r][0][wv] = b0.g; s_wh[r][0][wv] = b0.h; s_wv[r][0][wv] = b0.v; s_wq[r][0][wv] = b0.q;
                s_wg[r][1][wv] = b1.g; s_wh[r][1][wv] = b1.h; s_wv[r][1][wv] = b1.v; s_wq[r][1][wv] = b1.q;
            }
            __syncthreads();
            if (wv == 0 && live) {
                // lanes 0-3 take side 0 of the half's four waves, lanes 4-7
                // side 1; two quad swaps leave each side's best in lanes 0 and 4
                static_assert(FM_WAVES == 4, "one quad per side");
                int64_t g = 0;
                uint64_t h = 0;
                int32_t v = -1, q = -1;
                if (lane < 2 * FM_WAVES) {
                    const int sd = lane / FM_WAVES, x = lane % FM_WAVES;
                    g = s_wg[r][sd][x]; h = s_wh[r][sd][x]; v = s_wv[r][sd][x]; q = s_wq[r][sd][x];
                }
                best_step_dpp<DPP_XOR2>(g, h, v, q);
                best_step_dpp<DPP_XOR1>(g, h, v, q);
                const int64_t g1 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(g >> 32), FM_WAVES) << 32) |
                                             (uint32_t)__builtin_amdgcn_readlane((int32_t)g, FM_WAVES));
                const uint64_t h1 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(h >> 32), FM_WAVES) << 32) |
                                    (uint32_t)__builtin_amdgcn_readlane((int32_t)h, FM_WAVES);
                const int32_t v1 = __builtin_amdgcn_readlane(v, FM_WAVES);
                const int32_t q1 = __builtin_amdgcn_readlane(q, FM_WAVES);
                if (lane == 0) {
                    int32_t mv = -1;
                    bool stop = false;
                    if (v < 0 && v1 < 0) {
                        stop = true;
                    } else {
                        int from;
                        const bool over = S * w0 > L || S * w1 > L;
                        if (over && w0 != w1) {                           // MaxLoad
                            from = w0 > w1 ? 0 : 1;
                            if ((from ? v1 : v) < 0) from = 1 - from;
                        } else if (v < 0 || v1 < 0) {
                            from = v < 0 ? 1 : 0;
                        } else {                                          // TopGain
                            from = key_above(g, h, v, g1, h1, v1) ? 0 : 1;
                        }
                        mv = from ? v1 : v;
                        const int32_t mq = from ? q1 : q;
                        const int64_t mg = from ? g1 : g;
                        const int to = 1 - from;
                        st_r[mv] = 2;
                        int64_t cv, x0;
                        int32_t deg;
                        if (mq < qcap) {
                            cv = qcw[mq];
                            x0 = qx[mq];
                            deg = qd[mq];
                        } else {
                            cv = A.vw[mv];
                            x0 = A.xadj[mv];
                            deg = (int32_t)(A.xadj[mv + 1] - x0);
                        }
                        const int32_t qn = rs[r].qn;
                        atomicAdd(&s_bytes, 17ull * (unsigned long long)qn +
                                                25ull * (unsigned long long)deg);
                        // the queue stays dense: the last entry takes the moved
                        // node's place (the order of entries decides nothing)
                        const int32_t last = qn - 1;
                        if (mq != last) {
                            if (last < qcap) {
                                const int32_t lv = qv[last];
                                qv[mq] = lv; qg[mq] = qg[last]; qh[mq] = qh[last]; qs[mq] = qs[last];
                                qx[mq] = qx[last]; qd[mq] = qd[last]; qcw[mq] = qcw[last];
                                sl_r[lv] = mq;
                            } else {
                                const int32_t lv = q_r[last];
                                if (mq < qcap) {   // a memory entry moves on chip
                                    const int64_t lx0 = A.xadj[lv];
                                    qv[mq] = lv;
                                    qg[mq] = gain_r[lv];
                                    qh[mq] = mix64(rseed ^ (uint64_t)(uint32_t)lv);
                                    qs[mq] = A.part[lv] == b;
                                    qx[mq] = lx0;
                                    qd[mq] = (int32_t)(A.xadj[lv + 1] - lx0);
                                    qcw[mq] = A.vw[lv];
                                } else {
                                    q_r[mq] = lv;
                                }
                                sl_r[lv] = mq;
                            }
                        }
                        rs[r].qn = last;
                        if (from == 0) { w0 -= cv; w1 += cv; --c0; ++c1; }
                        else { w1 -= cv; w0 += cv; --c1; ++c0; }
                        cur_cut -= mg;
                        m_r[m++] = mv;
                        s_to[r] = to;
                        s_x0[r] = x0;
                        s_deg[r] = deg;
                        const int64_t imb = pair_imb(w0, w1, S, L);
                        if (state_below(imb, cur_cut, best_imb, best_cut)) {
                            best_imb = imb; best_cut = cur_cut;
                            bw0 = w0; bw1 = w1;
                            bc0 = c0; bc1 = c1;
                            kept = m;
                            since = 0;
                        } else {
                            since += 1;
                        }
                        if (since * (int64_t)A.alpha_den > (int64_t)A.alpha_num * smaller) stop = true;
                    }
                    s_v[r] = mv;
                    if (stop) s_done[r] = 1;
                }
            }
            __syncthreads();
            // neighbours of the moved node (its own side is not re-read: it is moved)
            const int32_t v = live ? s_v[r] : -1;
            if (v >= 0) {
                const int to = s_to[r];
                const int64_t x0 = s_x0[r], x1 = x0 + s_deg[r];
                for (int64_t e = x0 + lt; e < x1; e += FM_HALF) {
                    const int32_t u = A.adj[e];
                    const uint32_t wu = A.ew[e];
                    // everything about u in one round of loads (some unused)
                    const int32_t pu = A.part[u];
                    const uint8_t su_st = st_r[u];
                    const int32_t du = A.dist[u];
                    const int32_t sl = sl_r[u];
                    const int64_t gu = gain_r[u];
                    const int64_t ux0 = A.xadj[u], ux1 = A.xadj[u + 1];
                    const uint32_t cu = A.vw[u];
                    if (pu != a && pu != b) continue;
                    if (su_st == 2) continue;
                    const int su = pu == b;
                    const int64_t delta = su == to ? -2 * (int64_t)wu : 2 * (int64_t)wu;
                    if (su_st == 1) {
                        if (sl < qcap) qg[sl] += delta;
                        else gain_r[u] = gu + delta;
                    } else {
                        const int64_t g = gu + delta;
                        if (du >= 0) {
                            st_r[u] = 1;
                            const int32_t pos = atomicAdd(&rs[r].qn, 1);
                            sl_r[u] = pos;
                            if (pos < qcap) {
                                qv[pos] = u;
                                qg[pos] = g;
                                qh[pos] = mix64(rseed ^ (uint64_t)(uint32_t)u);
                                qs[pos] = (uint8_t)su;
                                qx[pos] = ux0;
                                qd[pos] = (int32_t)(ux1 - ux0);
                                qcw[pos] = cu;
                            } else {
                                q_r[pos] = u;
                                gain_r[u] = g;
                            }
                        } else {
                            gain_r[u] = g;
                        }
                    }
                }
            }
            __syncthreads();
        }
        // each half's lane 0 publishes its search
        if (lt == 0) {
            RunState &R = rs[r];
            R.best_imb = best_imb; R.best_cut = best_cut;
            R.best_w[0] = bw0; R.best_w[1] = bw1;
            R.best_cnt[0] = bc0; R.best_cnt[1] = bc1;
            R.kept = kept; R.m = m;
        }
        __syncthreads();
        // adopt the better run if it improves on the start
        if (tid == 0) {
            ticks_moves += wall_clock64() - t0;
            const int rb = state_below(rs[1].best_imb, rs[1].best_cut, rs[0].best_imb, rs[0].best_cut) ? 1 : 0;
            const bool imp = state_below(rs[rb].best_imb, rs[rb].best_cut, start_imb, start_cut);
            atomicAdd(&A.ctl->stats[1], 2ull);
            atomicAdd(&A.ctl->stats[2], (unsigned long long)(rs[0].m + rs[1].m));
            if (imp) {
                s_bytes += 12ull * (unsigned long long)rs[rb].kept;
                atomicAdd(&A.ctl->stats[3], (unsigned long long)rs[rb].kept);
                atomicAdd(&A.ctl->stats[4], 1ull);
                s_bw[0] = rs[rb].best_w[0];
                s_bw[1] = rs[rb].best_w[1];
                s_bc[0] = rs[rb].best_cnt[0];
                s_bc[1] = rs[rb].best_cnt[1];
                A.bw[a] = s_bw[0];
                A.bw[b] = s_bw[1];
                A.bc[a] = s_bc[0];
                A.bc[b] = s_bc[1];
            }
            s_stop = imp ? 0 : 1;
            s_pick = rb;
        }
        __syncthreads();
        if (s_stop) break;
        {
            const int rb = s_pick;
            const int32_t *mb = A.mlog + (size_t)rb * A.n + off;
            const int32_t kk = rs[rb].kept;
            for (int32_t i = tid; i < kk; i += FM_THREADS) {
                const int32_t v = mb[i];
                A.part[v] = A.part[v] == a ? b : a;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        atomicAdd(&A.ctl->stats[5], s_bytes);
        atomicAdd(&A.ctl->stats[6], ticks_init);
        atomicAdd(&A.ctl->stats[7], ticks_moves);
    }
}

void launch_refine_weights(const int32_t *part, const uint32_t *vw, int32_t n, int32_t k,
                           int64_t *bw, int32_t *bc, RefineCtl *ctl, hipStream_t s) {
    KAPPA_PROF("refine_weights", s);
    hipLaunchKernelGGL(ref_weights_k, dim3(grid_for(n, RQ_THREADS * 8, 1024)), dim3(RQ_THREADS), 0,
                       s, part, vw, n, k, bw, bc, ctl);
}

void launch_refine_colouring(const int64_t *xadj, const int32_t *adj, const int32_t *part,
                             int32_t n, int32_t k, unsigned long long *qbits, int32_t *tmp_pair,
                             int32_t *tmp_col, int32_t *cpairs, int32_t *col_off, int32_t *fill,
                             RefineCtl *ctl, hipStream_t s) {
    {
        KAPPA_PROF("refine_quotient", s);
        hipLaunchKernelGGL(ref_quotient_k, dim3(grid_for(n, RQ_THREADS * 8, 1024)),
                           dim3(RQ_THREADS), 0, s, xadj, adj, part, n, k, qbits);
    }
    KAPPA_PROF("refine_colour", s);
    hipLaunchKernelGGL(ref_colour_k, dim3(1), dim3(RQ_THREADS), 0, s, qbits, k, tmp_pair, tmp_col,
                       cpairs, col_off, fill, ctl);
}

void launch_refine_colour(const RefineLaunch &R, int32_t gi, int32_t c, int32_t npairs,
                          hipStream_t s) {
    {
        KAPPA_PROF("refine_collect", s);
        hipLaunchKernelGGL(ref_collect_k, dim3(grid_for(R.n, RQ_THREADS * RC_ITEMS, 1u << 30)),
                           dim3(RQ_THREADS), 0, s, R.part, R.n, R.k, c, R.cpairs, R.col_off, R.bc,
                           R.fill, R.poff, R.region);
    }
    FmArgs A;
    A.xadj = R.xadj; A.adj = R.adj; A.ew = R.ew; A.vw = R.vw; A.part = R.part;
    A.n = R.n; A.k = R.k; A.eps_num = R.eps_num; A.eps_den = R.eps_den; A.seed = R.seed;
    A.alpha_num = R.alpha_num; A.alpha_den = R.alpha_den; A.depth = R.depth;
    A.max_local = R.max_local; A.cpairs = R.cpairs; A.col_off = R.col_off; A.poff = R.poff;
    A.fill = R.fill;
    A.bw = R.bw;
    A.bc = R.bc; A.region = R.region; A.dist = R.dist; A.gain = R.gain; A.status = R.status;
    A.qlist = R.qlist; A.mlog = R.mlog; A.ctl = R.ctl;
    A.slot = R.slot;
    A.qcap = R.qcap < 0 || R.qcap > FM_QCAP ? FM_QCAP : R.qcap;
    KAPPA_PROF("refine_fm", s);
    hipLaunchKernelGGL(ref_fm_k, dim3(npairs), dim3(FM_THREADS), 0, s, A, gi, c);
}

}  // namespace kappa
