// k_sort.hip -- stable LSD radix sort of (key, value) pairs on the device,
// 8 bits per pass, and the device exclusive sum used beside it.
//
// A pass over n items in tiles of RS_TILE:
//   1. rs_hist_k:    the digit histogram of every tile, stored digit-major
//                    (hist[d * tiles + t]) so that one exclusive scan of the
//                    whole array gives, for digit d of tile t, the position of
//                    its first item in the output;
//   2. the library's device scan over hist, in place;
//   3. rs_scatter_k: every tile ranks its items stably (items in input order:
//                    step s of a tile holds items s * RS_THREADS + thread;
//                    within a step, lanes of one digit are found with eight
//                    ballots and counted by wave) and writes each item to its
//                    digit's position.
// Keys are uint32 or uint64; values are 32-bit.  Passes alternate between the
// output arrays and one scratch pair so that the last lands in the output;
// the input is not modified.
#include "kappa_internal.h"

namespace kappa {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_BINS = 256;
constexpr int RS_WAVES = RS_THREADS / WAVE;

template <class KT>
__global__ void __launch_bounds__(RS_THREADS) rs_hist_k(const KT *keys, int64_t n, int shift,
                                                        int32_t *hist) {
    __shared__ int32_t cnt[RS_BINS];
    const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {   // block-uniform
        cnt[threadIdx.x] = 0;
        __syncthreads();
        const int64_t base = tile * RS_TILE;
        uint32_t d[RS_ITEMS];
#pragma unroll
        for (int s = 0; s < RS_ITEMS; ++s) {
            const int64_t i = base + (int64_t)s * RS_THREADS + threadIdx.x;
            d[s] = i < n ? (uint32_t)((keys[i] >> shift) & (RS_BINS - 1)) : RS_BINS;
        }
#pragma unroll
        for (int s = 0; s < RS_ITEMS; ++s)
            if (d[s] < RS_BINS) atomicAdd(&cnt[d[s]], 1);
        __syncthreads();
        hist[(int64_t)threadIdx.x * tiles + tile] = cnt[threadIdx.x];
        __syncthreads();   // cnt is cleared for the next tile
    }
}

template <class KT>
__global__ void __launch_bounds__(RS_THREADS) rs_scatter_k(const KT *kin, const uint32_t *vin,
                                                           KT *kout, uint32_t *vout, int64_t n,
                                                           int shift, const int32_t *hist) {
    __shared__ int32_t base_of[RS_BINS];          // this tile's first output position per digit
    __shared__ int32_t wcnt[RS_WAVES][RS_BINS];   // items of a digit per wave in the current step
    const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    const int wv = threadIdx.x / WAVE;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {   // block-uniform
        base_of[threadIdx.x] = hist[(int64_t)threadIdx.x * tiles + tile];
        for (int w = 0; w < RS_WAVES; ++w) wcnt[w][threadIdx.x] = 0;
        const int64_t base = tile * RS_TILE;
        KT key[RS_ITEMS];
        uint32_t val[RS_ITEMS];
#pragma unroll
        for (int s = 0; s < RS_ITEMS; ++s) {
            const int64_t i = base + (int64_t)s * RS_THREADS + threadIdx.x;
            key[s] = i < n ? kin[i] : (KT)0;
            val[s] = i < n ? vin[i] : 0u;
        }
        __syncthreads();
        for (int s = 0; s < RS_ITEMS; ++s) {
            const int64_t i = base + (int64_t)s * RS_THREADS + threadIdx.x;
            const bool live = i < n;
            const uint32_t d = (uint32_t)((key[s] >> shift) & (RS_BINS - 1));
            // lanes of the wave holding the same digit
            uint64_t same = __ballot(live);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                same &= bit ? m : ~m;
            }
            const int before = (int)__popcll(same & lanemask_lt());
            if (live && before == 0) wcnt[wv][d] = (int32_t)__popcll(same);
            __syncthreads();
            if (live) {
                int32_t r = base_of[d] + before;
                for (int w = 0; w < wv; ++w) r += wcnt[w][d];
                kout[r] = key[s];
                vout[r] = val[s];
            }
            __syncthreads();
            {
                int32_t add = 0;
                for (int w = 0; w < RS_WAVES; ++w) {
                    add += wcnt[w][threadIdx.x];
                    wcnt[w][threadIdx.x] = 0;
                }
                base_of[threadIdx.x] += add;
            }
            __syncthreads();
        }
    }
}

// Exclusive scan of the histogram in place (values are item counts < 2^31).
struct HistF {
    int32_t *h;
    int64_t len;
    __device__ int64_t size() const { return len; }
    __device__ int64_t operator()(int64_t i) const { return h[i]; }
    __device__ void post(int64_t) const {}
};
struct HistW {
    int32_t *h;
    struct Pre {};
    struct Bound {
        int32_t *h;
        __device__ Pre prefetch(int64_t, int64_t) const { return Pre{}; }
        __device__ void operator()(int64_t i, int64_t pre, int64_t, const Pre &) const {
            h[i] = (int32_t)pre;
        }
    };
    __device__ Bound bind() const { return Bound{h}; }
};

static int64_t rs_tiles(int64_t n) { return (n + RS_TILE - 1) / RS_TILE; }

size_t radix_sort_ws_bytes(int64_t n, size_t key_bytes) {
    const int64_t nn = n > 0 ? n : 1;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t hist = (int64_t)RS_BINS * rs_tiles(nn);
    return al(key_bytes * nn) + al(4 * nn) + al(4 * hist) + al(8 * (scan_tiles(hist) + 1)) +
           al(4 * ARRIVE_WORDS);
}

template <class KT>
kappa_status radix_sort_pairs(const KT *kin, KT *kout, const uint32_t *vin, uint32_t *vout,
                              int64_t n, int begin_bit, int end_bit, char *ws, hipStream_t s) {
    if (n <= 0) return KAPPA_OK;
    if (n >= ((int64_t)1 << 31) || begin_bit < 0 || end_bit > (int)(8 * sizeof(KT)) ||
        begin_bit >= end_bit || kin == kout || vin == vout)
        return KAPPA_E_ARG;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t tiles = rs_tiles(n), hlen = (int64_t)RS_BINS * tiles;
    char *p = ws;
    KT *ktmp = (KT *)p;
    p += al(sizeof(KT) * n);
    uint32_t *vtmp = (uint32_t *)p;
    p += al(4 * n);
    int32_t *hist = (int32_t *)p;
    p += al(4 * hlen);
    int64_t *partials = (int64_t *)p;
    p += al(8 * (scan_tiles(hlen) + 1));
    unsigned *arrive = (unsigned *)p;
    ZeroRanges z;
    z.add(arrive, ARRIVE_WORDS);
    launch_zero(z, s);
    const int passes = (end_bit - begin_bit + 7) / 8;
    KT *kb[2] = {kout, ktmp};
    uint32_t *vb[2] = {vout, vtmp};
    const unsigned grid = grid_for(tiles, 1, 2048);
    for (int q = 0; q < passes; ++q) {
        const int shift = begin_bit + 8 * q;
        const KT *ksrc = q == 0 ? kin : kb[(passes - q) & 1];
        const uint32_t *vsrc = q == 0 ? vin : vb[(passes - q) & 1];
        KT *kdst = kb[(passes - 1 - q) & 1];
        uint32_t *vdst = vb[(passes - 1 - q) & 1];
        {
            KAPPA_PROF("sort_hist", s);
            hipLaunchKernelGGL(rs_hist_k<KT>, dim3(grid), dim3(RS_THREADS), 0, s, ksrc, n, shift, hist);
        }
        launch_scan(hlen, HistF{hist, hlen}, HistW{hist}, partials, arrive, nullptr, s);
        KAPPA_PROF("sort_scatter", s);
        hipLaunchKernelGGL(rs_scatter_k<KT>, dim3(grid), dim3(RS_THREADS), 0, s, ksrc, vsrc, kdst, vdst,
                           n, shift, hist);
    }
    return hipGetLastError() == hipSuccess ? KAPPA_OK : KAPPA_E_HIP;
}

template kappa_status radix_sort_pairs<uint32_t>(const uint32_t *, uint32_t *, const uint32_t *,
                                                 uint32_t *, int64_t, int, int, char *, hipStream_t);
template kappa_status radix_sort_pairs<uint64_t>(const uint64_t *, uint64_t *, const uint32_t *,
                                                 uint32_t *, int64_t, int, int, char *, hipStream_t);

// Exclusive sum of n int64 values (out[i] = sum of in[0 .. i-1]) by the
// library's device scan.  ws: exclusive_sum_ws_bytes(n) bytes.
struct SumF {
    const int64_t *in;
    int64_t len;
    __device__ int64_t size() const { return len; }
    __device__ int64_t operator()(int64_t i) const { return in[i]; }
    __device__ void post(int64_t) const {}
};
struct SumW {
    int64_t *out;
    struct Pre {};
    struct Bound {
        int64_t *out;
        __device__ Pre prefetch(int64_t, int64_t) const { return Pre{}; }
        __device__ void operator()(int64_t i, int64_t pre, int64_t, const Pre &) const { out[i] = pre; }
    };
    __device__ Bound bind() const { return Bound{out}; }
};

size_t exclusive_sum_ws_bytes(int64_t n) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(8 * (scan_tiles(n > 0 ? n : 1) + 1)) + al(4 * ARRIVE_WORDS);
}

kappa_status exclusive_sum_i64(const int64_t *in, int64_t *out, int64_t n, char *ws, hipStream_t s) {
    if (n <= 0) return KAPPA_OK;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    int64_t *partials = (int64_t *)ws;
    unsigned *arrive = (unsigned *)(ws + al(8 * (scan_tiles(n) + 1)));
    ZeroRanges z;
    z.add(arrive, ARRIVE_WORDS);
    launch_zero(z, s);
    launch_scan(n, SumF{in, n}, SumW{out}, partials, arrive, nullptr, s);
    return hipGetLastError() == hipSuccess ? KAPPA_OK : KAPPA_E_HIP;
}

}  // namespace kappa
