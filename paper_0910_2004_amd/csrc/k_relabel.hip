// Locality relabelling (Section 3.3: the preliminary partition by recursive
// coordinate bisection of nodes with 2D coordinates).
//
//   rcb order:  depth by depth, every box of more than `leaf` points is sorted
//               stably by x (even depths) or y (odd depths) and cut after its
//               first half.  Boxes are contiguous ranges of the order, so a
//               depth is a stable sort of all positions by (box, key): a
//               stable radix sort by key, then one by box.  The key is the
//               coordinate in a box that is cut and the position itself in a
//               box that is not, which therefore keeps its order.
//   relabel:    node x of the new numbering is node order[x] of the old one;
//               rows move, neighbours are renamed through the inverse, and
//               the entries are sorted by (row, new neighbour): by neighbour,
//               then stably by row.
//
// The sorts are the library's own stable LSD radix sorts (k_sort.hip), the
// offsets its device exclusive sum.
#include <vector>

#include "kappa_internal.h"

namespace kappa {

// Order-preserving 64-bit key of a double (-0.0 as +0.0).
__device__ __forceinline__ uint64_t sortable(double x) {
    if (x == 0.0) x = 0.0;
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ int32_t box_at(const int32_t *beg, int32_t nbox, int32_t i) {
    int32_t lo = 0, hi = nbox - 1;   // the last box whose start is <= i
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (beg[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Depth pass 1 input: the key of position i and i itself.
__global__ void rcb_keys_k(const double *xy, const int32_t *order, const int32_t *beg,
                           const uint8_t *cut, int32_t nbox, int32_t n, int axis, uint64_t *keys,
                           int32_t *pos) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = box_at(beg, nbox, (int32_t)i);
        keys[i] = cut[b] ? sortable(xy[2 * (int64_t)order[i] + axis]) : (uint64_t)i;
        pos[i] = (int32_t)i;
    }
}

// Depth pass 2 input: the box of the position each item came from.
__global__ void rcb_box_keys_k(const int32_t *pos, const int32_t *beg, int32_t nbox, int32_t n,
                               uint32_t *bkey) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bkey[i] = (uint32_t)box_at(beg, nbox, pos[i]);
}

__global__ void gather_i32_k(const int32_t *src, const int32_t *idx, int64_t n, int32_t *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

__global__ void iota_k(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// --- relabel ----------------------------------------------------------------
// inv[order[x]] = x; a value out of range or seen twice sets the flag.
__global__ void relabel_inverse_k(const int32_t *order, int32_t n, int32_t *inv, uint32_t *seen,
                                  uint32_t *flag) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = order[x];
        if ((uint32_t)v >= (uint32_t)n) {
            atomicOr(flag, 1u);
            continue;
        }
        if (atomicAdd(&seen[v], 1u) != 0u) atomicOr(flag, 1u);
        inv[v] = (int32_t)x;
    }
}

// New degree and node weight of every new node (deg[n] = 0 closes the scan).
__global__ void relabel_rows_k(DevGraph g, const int32_t *order, int64_t *deg, uint32_t *vw) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= g.n;
         x += (int64_t)gridDim.x * blockDim.x) {
        if (x == g.n) {
            deg[x] = 0;
            continue;
        }
        const int32_t v = order[x];
        deg[x] = g.xadj[v + 1] - g.xadj[v];
        vw[x] = g.vw[v];
    }
}

// The new rows' entries in the old order, renamed, with their row and
// position (one wave per row).
__global__ void relabel_fill_k(DevGraph g, const int32_t *order, const int32_t *inv,
                               const int64_t *nx, int32_t *adj, uint32_t *ew, uint32_t *row,
                               int32_t *pos) {
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
    for (int64_t x = w0; x < g.n; x += nw) {
        const int32_t v = order[x];
        const int64_t b = g.xadj[v], e = g.xadj[v + 1], d = nx[x];
        for (int64_t j = b + lane_id(); j < e; j += WAVE) {
            const int64_t t = d + (j - b);
            adj[t] = inv[g.adj[j]];
            ew[t] = g.ew[j];
            row[t] = (uint32_t)x;
            pos[t] = (int32_t)t;
        }
    }
}

__global__ void relabel_gather_k(const int32_t *adj0, const uint32_t *ew0, const int32_t *idx,
                                 int64_t m, int32_t *adj, uint32_t *ew) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = idx[j];
        adj[j] = adj0[s];
        ew[j] = ew0[s];
    }
}

static int bits_for(int64_t count) {   // bits of the largest value count - 1
    int b = 1;
    while (b < 63 && ((int64_t)1 << b) < count) ++b;
    return b;
}

// The boxes of every depth (host): beg[d] holds the box starts of depth d,
// cut[d] whether each box is cut (sorted) at that depth.
void rcb_boxes(int32_t n, int32_t leaf, std::vector<std::vector<int32_t>> &beg,
               std::vector<std::vector<uint8_t>> &cut) {
    std::vector<std::pair<int32_t, int32_t>> boxes = {{0, n}};
    for (;;) {
        bool any = false;
        for (auto &bx : boxes) any = any || bx.second - bx.first > leaf;
        if (!any) break;
        std::vector<int32_t> b;
        std::vector<uint8_t> c;
        std::vector<std::pair<int32_t, int32_t>> next;
        for (auto &bx : boxes) {
            b.push_back(bx.first);
            const bool k = bx.second - bx.first > leaf;
            c.push_back(k ? 1 : 0);
            if (k) {
                const int32_t mid = bx.first + (bx.second - bx.first) / 2;
                next.push_back({bx.first, mid});
                next.push_back({mid, bx.second});
            } else {
                next.push_back(bx);
            }
        }
        beg.push_back(b);
        cut.push_back(c);
        boxes.swap(next);
    }
}

#define HCHK(expr)                                    \
    do {                                              \
        if ((expr) != hipSuccess) return KAPPA_E_HIP; \
    } while (0)

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// ws == nullptr: only *need is set.  Synchronous (the box tables are host
// vectors read by the queued copies).
kappa_status rcb_order_impl(const double *xy, int32_t n, int32_t leaf, int32_t *order,
                            hipStream_t s, char *ws, size_t ws_bytes, size_t *need) {
    std::vector<std::vector<int32_t>> beg;
    std::vector<std::vector<uint8_t>> cut;
    rcb_boxes(n, leaf, beg, cut);
    size_t maxbox = 1;
    for (auto &b : beg) maxbox = std::max(maxbox, b.size());
    const size_t nn = (size_t)std::max(n, 1);
    const size_t t1 = radix_sort_ws_bytes((int64_t)nn, 8), t2 = radix_sort_ws_bytes((int64_t)nn, 4);
    const size_t o_k0 = 0, o_k1 = al256(o_k0 + 8 * nn), o_p0 = al256(o_k1 + 8 * nn),
                 o_p1 = al256(o_p0 + 4 * nn), o_b0 = al256(o_p1 + 4 * nn),
                 o_b1 = al256(o_b0 + 4 * nn), o_p2 = al256(o_b1 + 4 * nn),
                 o_ord = al256(o_p2 + 4 * nn), o_beg = al256(o_ord + 4 * nn),
                 o_cut = al256(o_beg + 4 * maxbox), o_tmp = al256(o_cut + maxbox),
                 total = al256(o_tmp + std::max(t1, t2));
    *need = total;
    if (!ws) return KAPPA_OK;
    if (ws_bytes < total) return KAPPA_E_NOMEM;
    uint64_t *k0 = (uint64_t *)(ws + o_k0), *k1 = (uint64_t *)(ws + o_k1);
    int32_t *p0 = (int32_t *)(ws + o_p0), *p1 = (int32_t *)(ws + o_p1), *p2 = (int32_t *)(ws + o_p2);
    uint32_t *b0 = (uint32_t *)(ws + o_b0), *b1 = (uint32_t *)(ws + o_b1);
    int32_t *ord2 = (int32_t *)(ws + o_ord), *dbeg = (int32_t *)(ws + o_beg);
    uint8_t *dcut = (uint8_t *)(ws + o_cut);
    void *tmp = ws + o_tmp;
    if (n <= 0) return KAPPA_OK;
    hipLaunchKernelGGL(iota_k, dim3(grid_for(n, BLOCK, 4096)), dim3(BLOCK), 0, s, order, (int64_t)n);
    for (size_t d = 0; d < beg.size(); ++d) {
        const int32_t nbox = (int32_t)beg[d].size();
        // small tables from pageable memory: the runtime stages them before
        // the copy call returns
        HCHK(hipMemcpyAsync(dbeg, beg[d].data(), (size_t)nbox * 4, hipMemcpyHostToDevice, s));
        HCHK(hipMemcpyAsync(dcut, cut[d].data(), (size_t)nbox, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(rcb_keys_k, dim3(grid_for(n, BLOCK, 4096)), dim3(BLOCK), 0, s, xy, order,
                           dbeg, dcut, nbox, n, (int)(d & 1), k0, p0);
        kappa_status st = radix_sort_pairs<uint64_t>(k0, k1, (const uint32_t *)p0, (uint32_t *)p1,
                                                     n, 0, 64, (char *)tmp, s);
        if (st != KAPPA_OK) return st;
        hipLaunchKernelGGL(rcb_box_keys_k, dim3(grid_for(n, BLOCK, 4096)), dim3(BLOCK), 0, s, p1,
                           dbeg, nbox, n, b0);
        st = radix_sort_pairs<uint32_t>(b0, b1, (const uint32_t *)p1, (uint32_t *)p2, n, 0,
                                        bits_for(nbox), (char *)tmp, s);
        if (st != KAPPA_OK) return st;
        hipLaunchKernelGGL(gather_i32_k, dim3(grid_for(n, BLOCK, 4096)), dim3(BLOCK), 0, s, order,
                           p2, (int64_t)n, ord2);
        HCHK(hipMemcpyAsync(order, ord2, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    }
    HCHK(hipGetLastError());
    HCHK(hipStreamSynchronize(s));
    return KAPPA_OK;
}

// ws == nullptr: only *need is set.  hflag: pinned host word.  Synchronous.
kappa_status relabel_impl(const DevGraph &g, const int32_t *order, int64_t *nx, int32_t *nadj,
                          uint32_t *new_ew, uint32_t *nvw, hipStream_t s, char *ws,
                          size_t ws_bytes, size_t *need, uint32_t *hflag) {
    const size_t nn = (size_t)std::max(g.n, 1), ne = (size_t)std::max<int64_t>(g.nnz, 1);
    const size_t ts = exclusive_sum_ws_bytes((int64_t)nn + 1), t1 = radix_sort_ws_bytes((int64_t)ne, 4);
    const size_t o_inv = 0, o_seen = al256(4 * nn), o_flag = al256(o_seen + 4 * nn),
                 o_deg = al256(o_flag + 4), o_a = al256(o_deg + 8 * (nn + 1)),
                 o_w = al256(o_a + 4 * ne), o_row = al256(o_w + 4 * ne),
                 o_p0 = al256(o_row + 4 * ne), o_k1 = al256(o_p0 + 4 * ne),
                 o_p1 = al256(o_k1 + 4 * ne), o_r1 = al256(o_p1 + 4 * ne),
                 o_p2 = al256(o_r1 + 4 * ne), o_tmp = al256(o_p2 + 4 * ne),
                 total = al256(o_tmp + std::max(ts, t1));
    *need = total;
    if (!ws) return KAPPA_OK;
    if (ws_bytes < total) return KAPPA_E_NOMEM;
    int32_t *inv = (int32_t *)(ws + o_inv);
    uint32_t *seen = (uint32_t *)(ws + o_seen), *flag = (uint32_t *)(ws + o_flag);
    int64_t *deg = (int64_t *)(ws + o_deg);
    int32_t *a0 = (int32_t *)(ws + o_a), *p0 = (int32_t *)(ws + o_p0);
    uint32_t *w0 = (uint32_t *)(ws + o_w), *row = (uint32_t *)(ws + o_row);
    uint32_t *k1 = (uint32_t *)(ws + o_k1), *r1 = (uint32_t *)(ws + o_r1);
    int32_t *p1 = (int32_t *)(ws + o_p1), *p2 = (int32_t *)(ws + o_p2);
    void *tmp = ws + o_tmp;
    ZeroRanges z;
    z.add(seen, g.n);
    z.add(flag, 1);
    launch_zero(z, s);
    if (g.n > 0)
        hipLaunchKernelGGL(relabel_inverse_k, dim3(grid_for(g.n, BLOCK, 4096)), dim3(BLOCK), 0, s,
                           order, g.n, inv, seen, flag);
    HCHK(hipMemcpyAsync(hflag, flag, 4, hipMemcpyDeviceToHost, s));
    HCHK(hipStreamSynchronize(s));
    if (*hflag) return KAPPA_E_ARG;   // not a permutation of 0 .. n-1
    hipLaunchKernelGGL(relabel_rows_k, dim3(grid_for((int64_t)g.n + 1, BLOCK, 4096)), dim3(BLOCK), 0,
                       s, g, order, deg, nvw);
    kappa_status st = exclusive_sum_i64(deg, nx, (int64_t)g.n + 1, (char *)tmp, s);
    if (st != KAPPA_OK) return st;
    if (g.n > 0 && g.nnz > 0) {
        hipLaunchKernelGGL(relabel_fill_k, dim3(grid_for(g.n, BLOCK / WAVE, 4096)), dim3(BLOCK), 0, s,
                           g, order, inv, nx, a0, w0, row, p0);
        // by new neighbour, then stably by row
        st = radix_sort_pairs<uint32_t>((const uint32_t *)a0, k1, (const uint32_t *)p0,
                                        (uint32_t *)p1, g.nnz, 0, bits_for(g.n), (char *)tmp, s);
        if (st != KAPPA_OK) return st;
        hipLaunchKernelGGL(gather_i32_k, dim3(grid_for(g.nnz, BLOCK, 4096)), dim3(BLOCK), 0, s,
                           (const int32_t *)row, p1, g.nnz, (int32_t *)k1);
        st = radix_sort_pairs<uint32_t>(k1, r1, (const uint32_t *)p1, (uint32_t *)p2, g.nnz, 0,
                                        bits_for(g.n), (char *)tmp, s);
        if (st != KAPPA_OK) return st;
        hipLaunchKernelGGL(relabel_gather_k, dim3(grid_for(g.nnz, BLOCK, 4096)), dim3(BLOCK), 0, s,
                           a0, w0, p2, g.nnz, nadj, new_ew);
    }
    HCHK(hipGetLastError());
    HCHK(hipStreamSynchronize(s));
    return KAPPA_OK;
}

}  // namespace kappa
