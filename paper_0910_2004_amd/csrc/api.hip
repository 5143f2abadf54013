// api.hip -- the C ABI (include/kappa.h): argument checks, stream-ordered
// device memory, the multilevel loop and the way back up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kappa_internal.h"

using namespace kappa;

// ===========================================================================
// Profiling: HIP events around library launches (enabled on request).
// ===========================================================================
namespace {

struct ProfRec {
    int id;
    hipEvent_t a, b;
};
struct Profiler {
    bool on = false;
    std::vector<const char *> names;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    std::vector<int64_t> launches;
    std::vector<double> ms;
    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    int id_of(const char *name) {
        for (size_t i = 0; i < names.size(); ++i)
            if (names[i] == name || std::strcmp(names[i], name) == 0) return (int)i;
        names.push_back(name);
        launches.push_back(0);
        ms.push_back(0.0);
        return (int)names.size() - 1;
    }
    void collect() {
        if (recs.empty()) return;
        (void)hipDeviceSynchronize();
        for (auto &r : recs) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, r.a, r.b);
            launches[r.id] += 1;
            ms[r.id] += t;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
};
Profiler g_prof;

}  // namespace

namespace kappa {
ProfScope::ProfScope(const char *name, hipStream_t st) : id(-1), s(st) {
    if (!g_prof.on) return;
    id = g_prof.id_of(name);
    ProfRec r{id, g_prof.take(), g_prof.take()};
    (void)hipEventRecord(r.a, s);
    g_prof.recs.push_back(r);
}
ProfScope::~ProfScope() {
    if (id < 0) return;
    (void)hipEventRecord(g_prof.recs.back().b, s);
}
}  // namespace kappa

extern "C" void kappa_profile_enable(int32_t on) { g_prof.on = on != 0; }
extern "C" void kappa_profile_reset(void) {
    g_prof.collect();
    std::fill(g_prof.launches.begin(), g_prof.launches.end(), 0);
    std::fill(g_prof.ms.begin(), g_prof.ms.end(), 0.0);
}
extern "C" int32_t kappa_profile_read(const char **names, int64_t *launches, double *ms,
                                      int32_t cap) {
    g_prof.collect();
    int32_t n = (int32_t)g_prof.names.size();
    for (int32_t i = 0; i < n && i < cap; ++i) {
        if (names) names[i] = g_prof.names[i];
        if (launches) launches[i] = g_prof.launches[i];
        if (ms) ms[i] = g_prof.ms[i];
    }
    return n;
}

// ===========================================================================
// Device memory: stream-ordered pool allocations.
// ===========================================================================
namespace {

std::once_flag g_pool_once;

void pool_init() {
    std::call_once(g_pool_once, [] {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    });
}

// A list of stream-ordered allocations released together.
struct Arena {
    hipStream_t s = nullptr;
    std::vector<void *> ptrs;
    bool failed = false;
    explicit Arena(hipStream_t st) : s(st) { pool_init(); }
    template <class T>
    T *get(int64_t count) {
        if (count <= 0) count = 1;
        void *p = nullptr;
        if (hipMallocAsync(&p, (size_t)count * sizeof(T), s) != hipSuccess || !p) {
            failed = true;
            return nullptr;
        }
        ptrs.push_back(p);
        return (T *)p;
    }
    void release() {
        for (void *p : ptrs) (void)hipFreeAsync(p, s);
        ptrs.clear();
    }
    ~Arena() { release(); }
};

// Pinned host memory for read-backs, per thread, kept for the process.
// Fixed regions so that read-backs of different kinds never alias.
enum PinnedRegion { PIN_SMALL = 0, PIN_MATCH = 1, PIN_RESULTS = 2 };
constexpr size_t PIN_REGION_BYTES = 96 * 1024;
void *pinned(size_t bytes, PinnedRegion region = PIN_SMALL) {
    thread_local char *buf = nullptr;
    if (bytes > PIN_REGION_BYTES) return nullptr;
    if (!buf) {
        void *p = nullptr;
        if (hipHostMalloc(&p, 3 * PIN_REGION_BYTES, hipHostMallocDefault) != hipSuccess) return nullptr;
        buf = (char *)p;
    }
    return buf + (size_t)region * PIN_REGION_BYTES;
}

inline hipStream_t S(kappa_stream_t s) { return (hipStream_t)s; }

bool graph_args_ok(const kappa_graph *g) {
    if (!g || g->n < 0 || g->nnz < 0 || !g->xadj) return false;
    if (g->n > 0 && !g->vw) return false;
    if (g->nnz > 0 && (!g->adj || !g->ew)) return false;
    return true;
}

DevGraph dev(const kappa_graph *g) {
    DevGraph d;
    d.n = g->n;
    d.nnz = g->nnz;
    d.xadj = g->xadj;
    d.adj = g->adj;
    d.ew = g->ew;
    d.vw = g->vw;
    return d;
}

#define HIPCHK(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return KAPPA_E_HIP; \
    } while (0)

// Validation + max degree, one read-back.
kappa_status validate_impl(const DevGraph &g, hipStream_t s, int32_t *maxdeg_out) {
    Arena ar(s);
    // [0] flags (u32) [1] maxdeg (i32) | sums (2 x u64)
    uint32_t *small = ar.get<uint32_t>(2);
    uint64_t *sums = ar.get<uint64_t>(2);
    int32_t *tr = ar.get<int32_t>(tile_rows_needed(g.nnz));
    if (ar.failed) return KAPPA_E_NOMEM;
    launch_fill_u32(small, 2, 0, s);
    launch_fill_u64(sums, 2, 0, s);
    launch_validate(g, tr, small, sums, s);
    launch_max_degree(g, (int32_t *)(small + 1), s);
    struct RB {
        uint32_t small[2];
        uint64_t sums[2];
    };
    RB *rb = (RB *)pinned(sizeof(RB));
    if (!rb) return KAPPA_E_NOMEM;
    HIPCHK(hipMemcpyAsync(rb->small, small, sizeof(rb->small), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rb->sums, sums, sizeof(rb->sums), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    uint32_t f = rb->small[0];
    if (maxdeg_out) *maxdeg_out = (int32_t)rb->small[1];
    if (f & 3u) return KAPPA_E_GRAPH;
    if ((f & 4u) || rb->sums[0] > 0xffffffffull || rb->sums[1] > 0xffffffffull)
        return KAPPA_E_RANGE;
    return KAPPA_OK;
}

int32_t max_degree_sync(const DevGraph &g, hipStream_t s, kappa_status *st) {
    Arena ar(s);
    int32_t *d = ar.get<int32_t>(1);
    if (ar.failed) { *st = KAPPA_E_NOMEM; return 0; }
    launch_fill_u32((uint32_t *)d, 1, 0, s);
    launch_max_degree(g, d, s);
    int32_t *h = (int32_t *)pinned(sizeof(int32_t));
    if (hipMemcpyAsync(h, d, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        *st = KAPPA_E_HIP;
        return 0;
    }
    *st = KAPPA_OK;
    return *h;
}

// ---------------------------------------------------------------------------
// Matching driver: batches of rounds, one read-back per batch.
// ---------------------------------------------------------------------------
constexpr int STAT_KEEP = 64;   // rounds of statistics kept per level

struct MatchResult {
    int32_t rounds = 0;
    int64_t matched = 0;
    std::vector<int64_t> pointing, degsum;
};

kappa_status run_matching(const DevGraph &g, int rating, uint64_t seed, int32_t maxdeg,
                          int32_t *mate, MatchScratch &ms, hipStream_t s, MatchResult &res) {
    static_assert(sizeof(MatchState) <= PIN_REGION_BYTES, "read-back region too small");
    launch_match_begin(g, rating, mate, ms, s);
    MatchState *rb = (MatchState *)pinned(sizeof(MatchState), PIN_MATCH);
    if (!rb) return KAPPA_E_NOMEM;
    const size_t head = offsetof(MatchState, stat);
    int r = 1, chunk = 8;
    for (;;) {
        launch_match_rounds(g, rating, seed, maxdeg, mate, ms, r, chunk, s);
        r += chunk;
        HIPCHK(hipMemcpyAsync(rb, ms.state, head, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (rb->handoff == -2 || g.n == 0) break;
        // -3: the finisher hit its round cap; more than n/2 + 1 rounds cannot
        // happen (each round with a pointing node matches a pair)
        if (rb->handoff == -3 || (int64_t)r > (int64_t)g.n + 256) return KAPPA_E_HIP;
        chunk = std::min(chunk * 2, 64);
    }
    res.rounds = rb->rounds;
    res.matched = rb->matched;
    int keep = std::min(res.rounds, STAT_KEEP);
    res.pointing.assign(keep, 0);
    res.degsum.assign(keep, 0);
    if (keep > 0) {
        HIPCHK(hipMemcpyAsync(&rb->stat[0][0], &ms.state->stat[0][0], sizeof(int64_t) * 2 * keep,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < keep; ++i) {
            res.pointing[i] = rb->stat[i][0];
            res.degsum[i] = rb->stat[i][1];
        }
    }
    return KAPPA_OK;
}

bool alloc_match_scratch(Arena &ar, const DevGraph &g, int rating, MatchScratch &ms) {
    ms.best = ar.get<int32_t>(g.n);
    ms.lists = ar.get<int32_t>(6 * (int64_t)g.n);
    ms.out = rating == KAPPA_INNER_OUTER ? ar.get<uint32_t>(g.n) : nullptr;
    ms.tile_row = rating == KAPPA_INNER_OUTER ? ar.get<int32_t>(tile_rows_needed(g.nnz)) : nullptr;
    ms.state = ar.get<MatchState>(1);
    return !ar.failed;
}

bool alloc_contract_scratch(Arena &ar, const DevGraph &g, ContractScratch &cs) {
    cs.rep_of = ar.get<int32_t>(g.n);
    cs.tmp_off = ar.get<int64_t>((int64_t)g.n + 1);
    cs.cdeg = ar.get<int32_t>(g.n);
    cs.rows = ar.get<int32_t>(3 * (int64_t)g.n);
    cs.row_cnt = ar.get<int32_t>(4);
    cs.tmp_adj = ar.get<int32_t>(g.nnz);
    cs.tmp_ew = ar.get<uint32_t>(g.nnz);
    cs.partials = ar.get<int64_t>(scan_tiles((int64_t)g.n + 1) + 2);
    cs.totals = ar.get<int64_t>(4);
    cs.hub_acc = nullptr;
    cs.hub_bits = nullptr;
    cs.hub_words = (int64_t)g.n / 32 + 1;
    return !ar.failed;
}

bool alloc_hubs(Arena &ar, int32_t n, ContractScratch &cs, hipStream_t s) {
    cs.hub_words = (int64_t)n / 32 + 1;
    cs.hub_acc = ar.get<uint32_t>((int64_t)HUB_SLOTS * n);
    cs.hub_bits = ar.get<uint32_t>((int64_t)HUB_SLOTS * cs.hub_words);
    if (ar.failed) return false;
    launch_fill_u32(cs.hub_acc, (int64_t)HUB_SLOTS * n, 0, s);
    launch_fill_u32(cs.hub_bits, (int64_t)HUB_SLOTS * cs.hub_words, 0, s);
    return true;
}

inline int64_t bound_of(int32_t maxdeg) { return maxdeg > 0 ? 2 * (int64_t)maxdeg - 2 : 0; }

}  // namespace

// ===========================================================================
// Hierarchy
// ===========================================================================
struct kappa_level {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t maxdeg = 0;
    const int64_t *xadj = nullptr;
    const int32_t *adj = nullptr;
    const uint32_t *ew = nullptr;
    const uint32_t *vw = nullptr;
    int32_t *cmap = nullptr;   // to the next level
    int32_t *mate = nullptr;
    int32_t rounds = 0;
    int64_t matched = 0;
    int32_t stop = KAPPA_STOP_NONE;
    std::vector<int64_t> pointing, degsum;
};

struct kappa_hierarchy {
    hipStream_t s = nullptr;
    std::vector<kappa_level> levels;
    std::vector<void *> owned;
    ~kappa_hierarchy() {
        for (void *p : owned) (void)hipFreeAsync(p, s);
    }
    template <class T>
    T *alloc(int64_t count) {
        if (count <= 0) count = 1;
        void *p = nullptr;
        if (hipMallocAsync(&p, (size_t)count * sizeof(T), s) != hipSuccess || !p) return nullptr;
        owned.push_back(p);
        return (T *)p;
    }
};

static DevGraph dev_level(const kappa_level &L) {
    DevGraph d;
    d.n = L.n;
    d.nnz = L.nnz;
    d.xadj = L.xadj;
    d.adj = L.adj;
    d.ew = L.ew;
    d.vw = L.vw;
    return d;
}

// ===========================================================================
// Entry points
// ===========================================================================
extern "C" kappa_status kappa_validate(const kappa_graph *g, kappa_stream_t stream) {
    if (!graph_args_ok(g)) return KAPPA_E_ARG;
    return validate_impl(dev(g), S(stream), nullptr);
}

extern "C" kappa_status kappa_rate(const kappa_graph *g, int32_t rating, uint64_t *num,
                                   uint64_t *den, kappa_stream_t stream) {
    if (!graph_args_ok(g) || rating < 0 || rating > 4) return KAPPA_E_ARG;
    if (g->nnz > 0 && (!num || !den)) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d = dev(g);
    Arena ar(s);
    int32_t *tr = ar.get<int32_t>(tile_rows_needed(d.nnz));
    uint32_t *out = rating == KAPPA_INNER_OUTER ? ar.get<uint32_t>(d.n) : nullptr;
    if (ar.failed) return KAPPA_E_NOMEM;
    launch_tile_rows(d, tr, s);
    if (out) launch_out(d, tr, out, s);
    launch_rate(d, tr, rating, out, num, den, s);
    HIPCHK(hipGetLastError());
    return KAPPA_OK;
}

extern "C" kappa_status kappa_match(const kappa_graph *g, int32_t rating, uint64_t level_seed,
                                    int32_t *mate, int32_t *rounds_out, int64_t *matched_out,
                                    kappa_stream_t stream) {
    if (!graph_args_ok(g) || rating < 0 || rating > 4) return KAPPA_E_ARG;
    if (g->n > 0 && !mate) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d = dev(g);
    kappa_status st;
    int32_t maxdeg = max_degree_sync(d, s, &st);
    if (st != KAPPA_OK) return st;
    Arena ar(s);
    MatchScratch ms;
    if (!alloc_match_scratch(ar, d, rating, ms)) return KAPPA_E_NOMEM;
    if (ms.tile_row) launch_tile_rows(d, ms.tile_row, s);
    MatchResult res;
    st = run_matching(d, rating, level_seed, maxdeg, mate, ms, s, res);
    if (st != KAPPA_OK) return st;
    if (rounds_out) *rounds_out = res.rounds;
    if (matched_out) *matched_out = res.matched;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_contract(const kappa_graph *g, const int32_t *mate, int32_t *cmap,
                                       kappa_graph_out *coarse, kappa_stream_t stream) {
    if (!graph_args_ok(g) || !coarse) return KAPPA_E_ARG;
    if (g->n > 0 && (!mate || !cmap || !coarse->vw)) return KAPPA_E_ARG;
    if (!coarse->xadj || coarse->cap_n < 0 || coarse->cap_nnz < 0) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d = dev(g);
    kappa_status st;
    int32_t maxdeg = max_degree_sync(d, s, &st);
    if (st != KAPPA_OK) return st;
    Arena ar(s);
    uint32_t *flag = ar.get<uint32_t>(1);
    ContractScratch cs;
    if (!alloc_contract_scratch(ar, d, cs)) return KAPPA_E_NOMEM;
    int64_t mb = bound_of(maxdeg);
    if (mb > ROW_MID_MAX && !alloc_hubs(ar, d.n, cs, s)) return KAPPA_E_NOMEM;
    // the coarse row offsets and weights need n' (+1) entries; n' <= n
    int64_t *cx = ar.get<int64_t>((int64_t)d.n + 1);
    uint32_t *cv = ar.get<uint32_t>(d.n);
    if (ar.failed) return KAPPA_E_NOMEM;
    launch_fill_u32(flag, 1, 0, s);
    launch_check_matching(d, mate, flag, s);
    uint32_t *hf = (uint32_t *)pinned(sizeof(uint32_t));
    HIPCHK(hipMemcpyAsync(hf, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*hf) return KAPPA_E_ARG;
    launch_contract_build(d, mate, mb, cmap, cv, cx, cs, s);
    int64_t *tot = (int64_t *)pinned(4 * sizeof(int64_t));
    HIPCHK(hipMemcpyAsync(tot, cs.totals, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t nc = (int32_t)tot[0];
    int64_t nnzc = tot[2];
    coarse->n = nc;
    coarse->nnz = nnzc;
    if (nc > coarse->cap_n || nnzc > coarse->cap_nnz) return KAPPA_E_CAPACITY;
    if (nnzc > 0 && (!coarse->adj || !coarse->ew)) return KAPPA_E_ARG;
    launch_contract_compact(cs, d.n, mb, cx, coarse->adj, coarse->ew, s);
    HIPCHK(hipMemcpyAsync(coarse->xadj, cx, ((size_t)nc + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToDevice, s));
    if (nc > 0)
        HIPCHK(hipMemcpyAsync(coarse->vw, cv, (size_t)nc * sizeof(uint32_t),
                              hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return KAPPA_OK;
}

extern "C" kappa_status kappa_coarsen(const kappa_graph *g, const kappa_coarsen_params *p,
                                      kappa_hierarchy **out, kappa_stream_t stream) {
    if (!out) return KAPPA_E_ARG;
    *out = nullptr;
    if (!graph_args_ok(g) || !p) return KAPPA_E_ARG;
    if (p->rating < 0 || p->rating > 4 || p->max_levels < 0 || p->max_levels > 256 ||
        (p->stall_num > 0 && p->stall_den == 0))
        return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d0 = dev(g);
    int32_t maxdeg = 0;
    kappa_status st = validate_impl(d0, s, &maxdeg);
    if (st != KAPPA_OK) return st;

    kappa_hierarchy *H = new (std::nothrow) kappa_hierarchy();
    if (!H) return KAPPA_E_NOMEM;
    H->s = s;
    kappa_level L0;
    L0.n = d0.n; L0.nnz = d0.nnz; L0.maxdeg = maxdeg;
    L0.xadj = d0.xadj; L0.adj = d0.adj; L0.ew = d0.ew; L0.vw = d0.vw;
    H->levels.push_back(L0);

    Arena ar(s);
    MatchScratch ms;
    ContractScratch cs;
    if (!alloc_match_scratch(ar, d0, p->rating, ms) || !alloc_contract_scratch(ar, d0, cs)) {
        delete H;
        return KAPPA_E_NOMEM;
    }
    bool hubs = false;
    int64_t *tot = (int64_t *)pinned(4 * sizeof(int64_t));

    for (int32_t l = 0;; ++l) {
        kappa_level &cur = H->levels.back();
        if (cur.n <= p->stop_n) { cur.stop = KAPPA_STOP_SIZE; break; }
        if (l == p->max_levels) { cur.stop = KAPPA_STOP_MAXLEVEL; break; }
        DevGraph d = dev_level(cur);
        uint64_t seed_l = mix64(p->seed + (uint64_t)l);
        cur.mate = H->alloc<int32_t>(d.n);
        if (!cur.mate) { delete H; return KAPPA_E_NOMEM; }
        if (ms.tile_row) launch_tile_rows(d, ms.tile_row, s);
        MatchResult mr;
        st = run_matching(d, p->rating, seed_l, cur.maxdeg, cur.mate, ms, s, mr);
        if (st != KAPPA_OK) { delete H; return st; }
        cur.rounds = mr.rounds;
        cur.matched = mr.matched;
        cur.pointing = mr.pointing;
        cur.degsum = mr.degsum;
        if (mr.matched == 0) { cur.stop = KAPPA_STOP_EMPTY; break; }

        int64_t mb = bound_of(cur.maxdeg);
        if (mb > ROW_MID_MAX && !hubs) {
            if (!alloc_hubs(ar, d0.n, cs, s)) { delete H; return KAPPA_E_NOMEM; }
            hubs = true;
        }
        cur.cmap = H->alloc<int32_t>(d.n);
        int64_t *cx = H->alloc<int64_t>((int64_t)d.n + 1);
        uint32_t *cv = H->alloc<uint32_t>(d.n);
        if (!cur.cmap || !cx || !cv) { delete H; return KAPPA_E_NOMEM; }
        launch_contract_build(d, cur.mate, mb, cur.cmap, cv, cx, cs, s);
        HIPCHK(hipMemcpyAsync(tot, cs.totals, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        kappa_level nxt;
        nxt.n = (int32_t)tot[0];
        nxt.nnz = tot[2];
        nxt.maxdeg = (int32_t)tot[3];
        int32_t *ca = H->alloc<int32_t>(nxt.nnz);
        uint32_t *ce = H->alloc<uint32_t>(nxt.nnz);
        if (!ca || !ce) { delete H; return KAPPA_E_NOMEM; }
        launch_contract_compact(cs, d.n, mb, cx, ca, ce, s);
        nxt.xadj = cx; nxt.adj = ca; nxt.ew = ce; nxt.vw = cv;
        int32_t n_prev = cur.n;
        H->levels.push_back(nxt);
        if (p->stall_num > 0 &&
            (uint64_t)(n_prev - nxt.n) * p->stall_den < (uint64_t)p->stall_num * (uint64_t)n_prev) {
            H->levels.back().stop = KAPPA_STOP_STALL;
            break;
        }
    }
    if (hipGetLastError() != hipSuccess) { delete H; return KAPPA_E_HIP; }
    HIPCHK(hipStreamSynchronize(s));
    *out = H;
    return KAPPA_OK;
}

extern "C" int32_t kappa_hierarchy_levels(const kappa_hierarchy *h) {
    return h ? (int32_t)h->levels.size() : 0;
}

extern "C" kappa_status kappa_hierarchy_level(const kappa_hierarchy *h, int32_t l, kappa_graph *g,
                                              const int32_t **cmap, kappa_level_info *info) {
    if (!h || l < 0 || l >= (int32_t)h->levels.size()) return KAPPA_E_ARG;
    const kappa_level &L = h->levels[l];
    if (g) {
        g->n = L.n; g->nnz = L.nnz; g->xadj = L.xadj; g->adj = L.adj; g->ew = L.ew; g->vw = L.vw;
    }
    if (cmap) *cmap = L.cmap;
    if (info) {
        info->n = L.n;
        info->nnz = L.nnz;
        info->rounds = L.rounds;
        info->matched = L.matched;
        info->stop_reason = L.stop;
    }
    return KAPPA_OK;
}

extern "C" int32_t kappa_hierarchy_round_stats(const kappa_hierarchy *h, int32_t l,
                                               int64_t *pointing, int64_t *degsum, int32_t cap) {
    if (!h || l < 0 || l >= (int32_t)h->levels.size() || cap < 0) return KAPPA_E_ARG;
    const kappa_level &L = h->levels[l];
    int32_t k = std::min<int32_t>(cap, (int32_t)L.pointing.size());
    for (int32_t i = 0; i < k; ++i) {
        if (pointing) pointing[i] = L.pointing[i];
        if (degsum) degsum[i] = L.degsum[i];
    }
    return L.rounds;
}

extern "C" void kappa_hierarchy_free(kappa_hierarchy *h) { delete h; }

extern "C" kappa_status kappa_initial_partition(int32_t n, int32_t k, uint64_t seed, int32_t *part,
                                                kappa_stream_t stream) {
    if (n < 0 || k < 1 || k > 4096 || (n > 0 && !part)) return KAPPA_E_ARG;
    launch_initial_partition(n, k, seed, part, S(stream));
    HIPCHK(hipGetLastError());
    return KAPPA_OK;
}

extern "C" kappa_status kappa_project(const int32_t *cmap, int32_t n_fine, int32_t n_coarse,
                                      const int32_t *part_coarse, int32_t *part_fine,
                                      kappa_stream_t stream) {
    if (n_fine < 0 || n_coarse < 0) return KAPPA_E_ARG;
    if (n_fine > 0 && (!cmap || !part_fine || (n_coarse > 0 && !part_coarse))) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    Arena ar(s);
    uint32_t *flag = ar.get<uint32_t>(1);
    if (ar.failed) return KAPPA_E_NOMEM;
    launch_fill_u32(flag, 1, 0, s);
    launch_project(cmap, n_fine, n_coarse, part_coarse, part_fine, flag, s);
    uint32_t *hf = (uint32_t *)pinned(sizeof(uint32_t));
    HIPCHK(hipMemcpyAsync(hf, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return *hf ? KAPPA_E_RANGE : KAPPA_OK;
}

static bool cut_args_ok(int32_t k, uint32_t eps_num, uint32_t eps_den) {
    return k >= 1 && k <= 4096 && eps_den >= 1 && eps_den <= 1000000u && eps_num <= 16000000u;
}

extern "C" kappa_status kappa_cut_balance(const kappa_graph *g, const int32_t *part, int32_t k,
                                          uint32_t eps_num, uint32_t eps_den, uint64_t *block_w,
                                          kappa_cut_result *out, kappa_stream_t stream) {
    if (!graph_args_ok(g) || !out || !cut_args_ok(k, eps_num, eps_den)) return KAPPA_E_ARG;
    if (g->n > 0 && !part) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d = dev(g);
    Arena ar(s);
    uint64_t *bw = block_w ? block_w : ar.get<uint64_t>(k);
    uint64_t *acc = ar.get<uint64_t>(3);
    uint32_t *flag = ar.get<uint32_t>(1);
    kappa_cut_result *rd = ar.get<kappa_cut_result>(1);
    int32_t *tr = ar.get<int32_t>(tile_rows_needed(d.nnz));
    if (ar.failed) return KAPPA_E_NOMEM;
    launch_fill_u32(flag, 1, 0, s);
    launch_tile_rows(d, tr, s);
    launch_cut_balance(d, tr, part, k, eps_num, eps_den, bw, acc, flag, rd, s);
    struct RB {
        kappa_cut_result r;
        uint32_t f;
    };
    RB *rb = (RB *)pinned(sizeof(RB));
    HIPCHK(hipMemcpyAsync(&rb->r, rd, sizeof(kappa_cut_result), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&rb->f, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (rb->f) return KAPPA_E_RANGE;
    *out = rb->r;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_uncoarsen(const kappa_hierarchy *h, int32_t k, uint64_t part_seed,
                                        uint32_t eps_num, uint32_t eps_den, int32_t *part0,
                                        kappa_cut_result *results, kappa_stream_t stream) {
    if (!h || h->levels.empty() || !cut_args_ok(k, eps_num, eps_den)) return KAPPA_E_ARG;
    if (h->levels[0].n > 0 && !part0) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    const int32_t nl = (int32_t)h->levels.size();
    Arena ar(s);
    std::vector<int32_t *> part(nl, nullptr);
    part[0] = part0;
    for (int32_t l = 1; l < nl; ++l) part[l] = ar.get<int32_t>(h->levels[l].n);
    kappa_cut_result *rd = ar.get<kappa_cut_result>(nl);
    uint64_t *bw = ar.get<uint64_t>(k);
    uint64_t *acc = ar.get<uint64_t>(3);
    uint32_t *flag = ar.get<uint32_t>(1);
    int32_t *tr = ar.get<int32_t>(tile_rows_needed(h->levels[0].nnz));
    if (ar.failed) return KAPPA_E_NOMEM;
    launch_fill_u32(flag, 1, 0, s);
    const int32_t L = nl - 1;
    launch_initial_partition(h->levels[L].n, k, part_seed, part[L], s);
    for (int32_t l = L; l >= 0; --l) {
        const kappa_level &lv = h->levels[l];
        if (l < L)
            launch_project(lv.cmap, lv.n, h->levels[l + 1].n, part[l + 1], part[l], flag, s);
        DevGraph d = dev_level(lv);
        launch_tile_rows(d, tr, s);
        launch_cut_balance(d, tr, part[l], k, eps_num, eps_den, bw, acc, flag, rd + l, s);
    }
    uint32_t *hf = (uint32_t *)pinned(sizeof(kappa_cut_result) * nl + 8, PIN_RESULTS);
    if (!hf) return KAPPA_E_ARG;
    kappa_cut_result *hr = (kappa_cut_result *)((char *)hf + 8);
    HIPCHK(hipMemcpyAsync(hf, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hr, rd, sizeof(kappa_cut_result) * nl, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*hf) return KAPPA_E_RANGE;
    if (results) std::memcpy(results, hr, sizeof(kappa_cut_result) * nl);
    return KAPPA_OK;
}

extern "C" const char *kappa_status_str(kappa_status st) {
    switch (st) {
    case KAPPA_OK: return "ok";
    case KAPPA_E_ARG: return "invalid argument";
    case KAPPA_E_GRAPH: return "graph is not a symmetric simple CSR with ascending rows";
    case KAPPA_E_RANGE: return "value out of range (weight, weight sum, block id or map entry)";
    case KAPPA_E_NOMEM: return "device allocation failed";
    case KAPPA_E_CAPACITY: return "output buffer too small";
    case KAPPA_E_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

extern "C" const char *kappa_version(void) { return "kappa-mi355x 0.1 (gfx950)"; }
