// api.hip -- the C ABI (include/kappa.h): argument checks, stream-ordered
// device memory, the multilevel driver and the way back up.
//
// The multilevel loop runs on device state (k_level.hip): the host enqueues a
// batch of levels, then reads the control block once; levels whose stop rule
// has fired turn into no-ops on the device.  All levels live in one arena
// owned by the hierarchy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include <dlfcn.h>

#include <string>

#include "kappa_internal.h"

using namespace kappa;

// ===========================================================================
// Tuning table: the thresholds of kappa_tuning.  Defaults are the compiled
// values; at load the library reads the table at $KAPPA_TUNING (a path;
// "none" skips it) or else kappa_tuning.txt beside the library, if present.
// A bad file leaves the defaults.
// ===========================================================================
namespace {
std::mutex g_tune_mu;
Tune g_tune;

bool tune_ok(const kappa_tuning &t) {
    return t.bin_small_max >= 1 && t.bin_small_max <= BIN_SMALL_MAX && t.tail_max >= 0 &&
           t.tail_max <= FINISH_MAX && t.finish_max >= 0 && t.finish_max <= (1 << 20) &&
           t.finish_max_big >= 0 && t.finish_max_big <= (1 << 16) && t.row_small_max >= 2 &&
           t.row_small_max <= ROW_SMALL_MAX && t.scan_one_block_max >= 0 &&
           t.scan_one_block_max <= (1 << 22) && t.rounds_base >= 1 && t.rounds_base <= 16 &&
           t.rounds_n0 >= 1 && t.rounds_n0 <= (1 << 24) && t.rounds_growth >= 2 &&
           t.rounds_growth <= 1024 && t.rounds_cap >= t.rounds_base && t.rounds_cap <= 32;
}
kappa_tuning to_abi(const Tune &u) {
    kappa_tuning t;
    t.bin_small_max = u.bin_small_max;
    t.tail_max = u.tail_max;
    t.finish_max = u.finish_max;
    t.finish_max_big = u.finish_max_big;
    t.row_small_max = u.row_small_max;
    t.scan_one_block_max = u.scan_one_block_max;
    t.rounds_base = u.rounds_base;
    t.rounds_n0 = u.rounds_n0;
    t.rounds_growth = u.rounds_growth;
    t.rounds_cap = u.rounds_cap;
    return t;
}
Tune from_abi(const kappa_tuning &t) {
    Tune u;
    u.bin_small_max = t.bin_small_max;
    u.tail_max = t.tail_max;
    u.finish_max = t.finish_max;
    u.finish_max_big = t.finish_max_big;
    u.row_small_max = t.row_small_max;
    u.scan_one_block_max = t.scan_one_block_max;
    u.rounds_base = t.rounds_base;
    u.rounds_n0 = t.rounds_n0;
    u.rounds_growth = t.rounds_growth;
    u.rounds_cap = t.rounds_cap;
    return u;
}
// "name value" lines ('#' starts a comment); every name must be known.
kappa_status tune_parse(const char *path, kappa_tuning *out) {
    FILE *f = std::fopen(path, "r");
    if (!f) return KAPPA_E_ARG;
    kappa_tuning t = *out;
    struct Field {
        const char *name;
        int32_t *p;
    } fields[] = {{"bin_small_max", &t.bin_small_max},   {"tail_max", &t.tail_max},
                  {"finish_max", &t.finish_max},         {"finish_max_big", &t.finish_max_big},
                  {"row_small_max", &t.row_small_max},   {"scan_one_block_max", &t.scan_one_block_max},
                  {"rounds_base", &t.rounds_base},       {"rounds_n0", &t.rounds_n0},
                  {"rounds_growth", &t.rounds_growth},   {"rounds_cap", &t.rounds_cap}};
    char line[512];
    kappa_status st = KAPPA_OK;
    while (st == KAPPA_OK && std::fgets(line, sizeof line, f)) {
        char *hash = std::strchr(line, '#');
        if (hash) *hash = 0;
        char name[128];
        long long v = 0;
        char extra[8];
        const int got = std::sscanf(line, "%127s %lld %7s", name, &v, extra);
        if (got <= 0) continue;   // blank or comment
        if (got != 2 || v < INT32_MIN || v > INT32_MAX) {
            st = KAPPA_E_ARG;
            break;
        }
        bool known = false;
        for (auto &fd : fields)
            if (std::strcmp(fd.name, name) == 0) {
                *fd.p = (int32_t)v;
                known = true;
            }
        if (!known) st = KAPPA_E_ARG;
    }
    std::fclose(f);
    if (st == KAPPA_OK && !tune_ok(t)) st = KAPPA_E_RANGE;
    if (st == KAPPA_OK) *out = t;
    return st;
}
struct TuneInit {
    TuneInit() {
        const char *e = std::getenv("KAPPA_TUNING");
        std::string path;
        if (e && e[0]) {
            if (std::strcmp(e, "none") == 0) return;
            path = e;
        } else {
            Dl_info info;
            if (!dladdr((void *)&tune_ok, &info) || !info.dli_fname) return;
            path = info.dli_fname;
            const size_t slash = path.rfind('/');
            path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) +
                   "/kappa_tuning.txt";
        }
        kappa_tuning t = to_abi(Tune{});
        if (tune_parse(path.c_str(), &t) == KAPPA_OK) g_tune = from_abi(t);
    }
} g_tune_init;
}  // namespace

Tune kappa::tuning_now() {
    std::lock_guard<std::mutex> g(g_tune_mu);
    return g_tune;
}

extern "C" kappa_status kappa_tuning_get(kappa_tuning *out) {
    if (!out) return KAPPA_E_ARG;
    *out = to_abi(tuning_now());
    return KAPPA_OK;
}

extern "C" kappa_status kappa_tuning_set(const kappa_tuning *t) {
    if (!t) return KAPPA_E_ARG;
    if (!tune_ok(*t)) return KAPPA_E_RANGE;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune = from_abi(*t);
    return KAPPA_OK;
}

extern "C" kappa_status kappa_tuning_load(const char *path) {
    if (!path) return KAPPA_E_ARG;
    kappa_tuning t = to_abi(tuning_now());
    const kappa_status st = tune_parse(path, &t);
    if (st != KAPPA_OK) return st;
    return kappa_tuning_set(&t);
}

// ===========================================================================
// Profiling: HIP events around library launches (enabled on request).
// ===========================================================================
namespace {

struct ProfRec {
    int id;
    hipEvent_t a, b;
};
struct Profiler {
    std::atomic<bool> on{false};
    std::mutex mu;   // records are taken by every thread that launches
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
// set while an allocation-free entry point runs on this thread: the profiler
// records nothing then (its events would be created on demand)
thread_local bool g_no_alloc_call = false;

ProfScope::ProfScope(const char *name, hipStream_t st) : id(-1), rec(0), s(st) {
    if (!g_prof.on || g_no_alloc_call) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    id = g_prof.id_of(name);
    ProfRec r{id, g_prof.take(), g_prof.take()};
    (void)hipEventRecord(r.a, s);
    rec = g_prof.recs.size();
    g_prof.recs.push_back(r);
}
ProfScope::~ProfScope() {
    if (id < 0) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    (void)hipEventRecord(g_prof.recs[rec].b, s);
}
}  // namespace kappa

extern "C" void kappa_profile_enable(int32_t on) { g_prof.on = on != 0; }
extern "C" void kappa_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.collect();
    std::fill(g_prof.launches.begin(), g_prof.launches.end(), 0);
    std::fill(g_prof.ms.begin(), g_prof.ms.end(), 0.0);
}
extern "C" int32_t kappa_profile_read(const char **names, int64_t *launches, double *ms,
                                      int32_t cap) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
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
// Device memory.  Per stream, the library keeps one grow-only workspace for
// call-local buffers (held under a host lock while a call uses it) and a few
// released hierarchy arenas for reuse, so that a call on a warm stream
// allocates nothing.  All are stream-ordered allocations from the device's
// default pool.
// ===========================================================================
namespace {

bool debug_on();

// Under KAPPA_DEBUG, names a failed allocation on stderr.
void alloc_failed(const char *what, size_t bytes, hipError_t e) {
    if (debug_on())
        fprintf(stderr, "kappa: %s of %zu bytes failed: %s\n", what, bytes, hipGetErrorString(e));
}

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

constexpr size_t KEEP_ARENAS = 4;

// The device allocator (kappa_set_allocator); the default is the device's
// stream-ordered pool.  Every block remembers the allocator it came from.
struct Allocator {
    kappa_alloc_fn alloc = nullptr;
    kappa_free_fn dealloc = nullptr;
    void *ctx = nullptr;
    bool operator==(const Allocator &o) const {
        return alloc == o.alloc && dealloc == o.dealloc && ctx == o.ctx;
    }
};
std::mutex g_alloc_mu;
Allocator g_alloc;

Allocator current_allocator() {
    std::lock_guard<std::mutex> g(g_alloc_mu);
    return g_alloc;
}

void *dev_alloc(size_t bytes, hipStream_t s, const Allocator &al, const char *what) {
    void *p = nullptr;
    if (al.alloc) {
        p = al.alloc(bytes, (kappa_stream_t)s, al.ctx);
        if (!p) alloc_failed(what, bytes, hipErrorOutOfMemory);
        return p;
    }
    pool_init();
    const hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess || !p) {
        alloc_failed(what, bytes, e);
        return nullptr;
    }
    return p;
}

// idle: the device has no work left that uses p (free at once, no stream).
void dev_free(void *p, size_t bytes, hipStream_t s, const Allocator &al, bool idle = false) {
    if (!p) return;
    if (al.dealloc)
        al.dealloc(p, bytes, (kappa_stream_t)s, al.ctx);
    else if (idle)
        (void)hipFree(p);
    else
        (void)hipFreeAsync(p, s);
}

struct CachedArena {
    void *p;
    size_t bytes;
    Allocator al;
};

struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;      // nullptr: capture failed, run directly
    uint64_t last_use;
};

struct StreamCache {
    hipStream_t s = nullptr;
    std::mutex mu;            // held by the call using `ws` (and the graph cache)
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Allocator ws_al;          // the allocator of `ws`
    std::mutex amu;           // guards `arenas`
    std::vector<CachedArena> arenas;
    // launch sequences replayed as graphs (see run_seq)
    hipStream_t side = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<GraphEntry> graphs;
    std::vector<std::vector<uint64_t>> seen;
    uint64_t clock = 0;
};

std::mutex g_cache_mu;
std::vector<StreamCache *> g_caches;

StreamCache *cache_of(hipStream_t s) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    for (StreamCache *c : g_caches)
        if (c->s == s) return c;
    StreamCache *c = new StreamCache();
    c->s = s;
    g_caches.push_back(c);
    return c;
}

// 256-byte aligned sub-buffers of one block; with base == nullptr it only
// measures the layout.
struct Carve {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *get(int64_t count) {
        if (count <= 0) count = 1;
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += (size_t)count * sizeof(T);
        return p;
    }
};

// The stream's workspace, locked, at least `bytes` large (base == nullptr if
// it could not be allocated).  Calls on one stream are stream-ordered, so
// the next holder may reuse the memory while earlier kernels still run.
struct Workspace {
    StreamCache *c;
    std::unique_lock<std::mutex> lk;
    char *base = nullptr;
    Workspace(hipStream_t s, size_t bytes) : c(cache_of(s)), lk(c->mu) {
        const Allocator al = current_allocator();
        if (c->ws_bytes < bytes || !(c->ws_al == al)) {
            dev_free(c->ws, c->ws_bytes, s, c->ws_al);
            c->ws = nullptr;
            c->ws_bytes = 0;
            size_t want = bytes + bytes / 4 + 4096;
            void *p = dev_alloc(want, s, al, "workspace");
            if (!p) return;
            c->ws = (char *)p;
            c->ws_bytes = want;
            c->ws_al = al;
        }
        base = c->ws;
    }
};

// Runs `layout(Carve&)` once to measure and once on the locked workspace.
template <class L>
bool carve_workspace(hipStream_t s, std::unique_ptr<Workspace> &w, L &&layout) {
    Carve m;
    layout(m);
    w.reset(new (std::nothrow) Workspace(s, m.off));
    if (!w || !w->base) return false;
    Carve r;
    r.base = w->base;
    layout(r);
    return true;
}

// An arena of at least `bytes` from the current allocator (recycled if the
// stream's cache has one); *got: its size, *al: its allocator.
void *take_arena(hipStream_t s, size_t bytes, size_t *got, Allocator *al) {
    StreamCache *c = cache_of(s);
    *al = current_allocator();
    {
        std::lock_guard<std::mutex> g(c->amu);
        int best = -1;
        for (size_t i = 0; i < c->arenas.size(); ++i)
            if (c->arenas[i].bytes >= bytes && c->arenas[i].al == *al &&
                (best < 0 || c->arenas[i].bytes < c->arenas[best].bytes))
                best = (int)i;
        if (best >= 0) {
            void *p = c->arenas[best].p;
            *got = c->arenas[best].bytes;
            c->arenas.erase(c->arenas.begin() + best);
            return p;
        }
    }
    void *p = dev_alloc(bytes, s, *al, "arena");
    if (!p) return nullptr;
    *got = bytes;
    return p;
}

void give_arena(hipStream_t s, void *p, size_t bytes, const Allocator &al) {
    if (!p) return;
    StreamCache *c = cache_of(s);
    {
        std::lock_guard<std::mutex> g(c->amu);
        if (c->arenas.size() < KEEP_ARENAS && al == current_allocator()) {
            c->arenas.push_back(CachedArena{p, bytes, al});
            return;
        }
    }
    dev_free(p, bytes, s, al);
}

// ---------------------------------------------------------------------------
// Launch sequences (a batch of levels, the way back up) as HIP graphs.  A
// sequence is keyed by everything its kernel arguments and grids depend on
// (the workspace address included).  The first call with a key launches
// directly; the second captures the sequence on the stream's side stream and
// instantiates it; later calls replay it.  Replays run on the side stream,
// ordered against the caller's stream by an event each way.  The sequences
// hold kernel launches only.
// ---------------------------------------------------------------------------
bool debug_on();
bool g_graphs_on = false;   // measured slower than direct launches on gfx950 (ROCm 7)
bool g_tail_on = false;     // small levels in one workgroup (tail_k): measured slower
constexpr size_t KEEP_GRAPHS = 24, KEEP_SEEN = 48;

template <class E>
hipError_t run_seq(StreamCache *c, hipStream_t s, const std::vector<uint64_t> &key, E &&enqueue) {
    if (!g_graphs_on || g_prof.on || g_persistent_on) {   // cooperative launches are not captured
        enqueue(s);
        return hipGetLastError();
    }
    ++c->clock;
    GraphEntry *hit = nullptr;
    for (GraphEntry &e : c->graphs)
        if (e.key == key) hit = &e;
    if (!hit) {
        bool again = false;
        for (auto &k : c->seen) again = again || k == key;
        if (!again) {
            if (c->seen.size() >= KEEP_SEEN) c->seen.erase(c->seen.begin());
            c->seen.push_back(key);
            enqueue(s);
            return hipGetLastError();
        }
        if (!c->side) {
            if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess) {
                enqueue(s);
                return hipGetLastError();
            }
        }
        if (c->graphs.size() >= KEEP_GRAPHS) {
            size_t old = 0;
            for (size_t i = 1; i < c->graphs.size(); ++i)
                if (c->graphs[i].last_use < c->graphs[old].last_use) old = i;
            (void)hipStreamSynchronize(c->side);
            if (c->graphs[old].exec) (void)hipGraphExecDestroy(c->graphs[old].exec);
            c->graphs.erase(c->graphs.begin() + old);
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        bool ok = hipStreamBeginCapture(c->side, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            enqueue(c->side);
            ok = hipStreamEndCapture(c->side, &g) == hipSuccess && g;
            ok = ok && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess && ex;
            if (g) (void)hipGraphDestroy(g);
        }
        (void)hipGetLastError();
        if (!ok && ex) {
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
        }
        c->graphs.push_back(GraphEntry{key, ex, c->clock});
        hit = &c->graphs.back();
        if (debug_on() && !ex) fprintf(stderr, "kappa: graph capture failed; launching directly\n");
    }
    hit->last_use = c->clock;
    if (!hit->exec) {
        enqueue(s);
        return hipGetLastError();
    }
    hipError_t e = hipEventRecord(c->ev_in, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(hit->exec, c->side);
    if (e == hipSuccess) e = hipEventRecord(c->ev_out, c->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_out, 0);
    return e;
}

inline uint64_t pkey(const void *p) { return (uint64_t)(uintptr_t)p; }

// First-attempt arena size of kappa_coarsen / kappa_coarsen_batch (0: sized
// from level 0), with the cursor capped at exactly that size.
std::atomic<uint64_t> g_arena_first{0};

// Returns an arena to the stream's cache unless released to a hierarchy.
struct ArenaHold {
    hipStream_t s;
    void *p;
    size_t bytes;
    Allocator al;
    ~ArenaHold() { give_arena(s, p, bytes, al); }
    void *release() {
        void *q = p;
        p = nullptr;
        return q;
    }
};

// Pinned host memory for read-backs, per thread, kept for the process.
// Fixed regions so that read-backs of different kinds never alias.
enum PinnedRegion { PIN_SMALL = 0, PIN_LEVELS = 1, PIN_RESULTS = 2 };
constexpr size_t PIN_REGION_BYTES = 320 * 1024;
void *pinned(size_t bytes, PinnedRegion region = PIN_SMALL) {
    thread_local char *buf = nullptr;
    if (bytes > PIN_REGION_BYTES) return nullptr;
    if (!buf) {
        void *p = nullptr;
        const hipError_t e = hipHostMalloc(&p, 3 * PIN_REGION_BYTES, hipHostMallocDefault);
        if (e != hipSuccess) {
            alloc_failed("pinned host buffer", 3 * PIN_REGION_BYTES, e);
            return nullptr;
        }
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

// KAPPA_DEBUG=1 in the environment prints the HIP call or device flag behind
// an error status to stderr.
bool debug_on() {
    static int on = -1;
    if (on < 0) {
        const char *e = getenv("KAPPA_DEBUG");
        on = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return on == 1;
}

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            if (debug_on())                                                           \
                fprintf(stderr, "kappa: %s failed: %s (%s:%d)\n", #expr,              \
                        hipGetErrorString(_e), __FILE__, __LINE__);                   \
            return KAPPA_E_HIP;                                                       \
        }                                                                             \
    } while (0)

// Validation + max degree, one read-back.  trusted: the caller has validated
// the graph (KAPPA_COARSEN_TRUSTED); only the offsets pass runs (offsets,
// c(V) and the maximum degree), and no entry is checked.
kappa_status validate_impl(const DevGraph &g, hipStream_t s, int32_t *maxdeg_out,
                           bool trusted = false) {
    // the kernels' outputs in one block: zeroed by one launch, read back by one copy
    struct RB {
        uint32_t flags;
        int32_t mdeg[NSHARD];
        uint64_t sums[4 * NSHARD];
    };
    static_assert(sizeof(RB) % 4 == 0, "zeroed as words");
    RB *dv = nullptr;
    int32_t *tr = nullptr;
    char *sort_ws = nullptr;
    const size_t sort_bytes = trusted ? 0 : val_sort_ws_bytes(g.n, g.nnz);
    std::unique_ptr<Workspace> w;
    bool ok = carve_workspace(s, w, [&](Carve &cv) {
        dv = cv.get<RB>(1);
        tr = cv.get<int32_t>(tile_rows_needed(g.nnz));
        sort_ws = sort_bytes ? cv.get<char>((int64_t)sort_bytes) : nullptr;
    });
    if (!ok) return KAPPA_E_NOMEM;
    ZeroRanges z;
    z.add(dv, sizeof(RB) / 4);
    launch_zero(z, s);
    RB *rb = (RB *)pinned(sizeof(RB));
    if (!rb) return KAPPA_E_NOMEM;
    if (sort_ws) {
        // large graphs: the maximum degree decides between the sorted symmetry
        // test and the binary searches (one read-back more)
        launch_validate(g, tr, &dv->flags, dv->sums, dv->mdeg, s, true);
        HIPCHK(hipMemcpyAsync(rb->mdeg, dv->mdeg, sizeof(rb->mdeg), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int32_t md0 = 0;
        for (int i = 0; i < NSHARD; ++i) md0 = std::max(md0, rb->mdeg[i]);
        launch_validate(g, tr, &dv->flags, dv->sums, dv->mdeg, s, false,
                        md0 > VAL_SORT_MIN_DEG ? sort_ws : nullptr, true);
    } else {
        launch_validate(g, tr, &dv->flags, dv->sums, dv->mdeg, s, trusted, nullptr);
    }
    HIPCHK(hipMemcpyAsync(rb, dv, sizeof(RB), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    uint64_t tot[4] = {0, 0, 0, 0};
    int32_t md = 0;
    for (int i = 0; i < NSHARD; ++i) {
        for (int q = 0; q < 4; ++q) tot[q] += rb->sums[q * NSHARD + i];
        md = std::max(md, rb->mdeg[i]);
    }
    if (maxdeg_out) *maxdeg_out = md;
    uint32_t f = rb->flags;
    if (trusted) return (f & 1u) ? KAPPA_E_GRAPH : (tot[1] > 0xffffffffull ? KAPPA_E_RANGE : KAPPA_OK);
    if ((f & 3u) || tot[2] != tot[3]) return KAPPA_E_GRAPH;
    if ((f & 4u) || tot[0] > 0xffffffffull || tot[1] > 0xffffffffull) return KAPPA_E_RANGE;
    return KAPPA_OK;
}

// ---------------------------------------------------------------------------
// Scratch shared by every level (sized for level 0), carved from the
// workspace.  After the real pass the caller zeroes `arrive` (and the hub
// arrays) with fill_scratch.
// ---------------------------------------------------------------------------
// chunks: scan rows above BIN_MID_MAX entries in chunks of HUB_CHUNK (the
// graph has such rows at level 0; coarse levels of other graphs rarely do,
// and their long rows are then scanned by one block each).
void carve_scratch(Carve &cv, const DevGraph &g, int rating, bool hubs, Ctx &c,
                   bool chunks = false, bool tail = false) {
    MatchScratch &ms = c.ms;
    ContractScratch &cs = c.cs;
    ms.best = cv.get<int32_t>(g.n);
    ms.lv = cv.get<int32_t>(6 * (int64_t)g.n);
    ms.lb = cv.get<int32_t>(6 * (int64_t)g.n);
    ms.ld = cv.get<int32_t>(6 * (int64_t)g.n);
    ms.nrec = cv.get<int2>(g.n);
    ms.out = rating == KAPPA_INNER_OUTER ? cv.get<uint32_t>(g.n) : nullptr;
    ms.tile_row = rating == KAPPA_INNER_OUTER ? cv.get<int32_t>(tile_rows_needed(g.nnz)) : nullptr;
    ms.state = cv.get<MatchState>(1);
    ms.coop_bar = cv.get<unsigned>(2 + ARRIVE_WORDS);
    cs.rep_of = cv.get<int32_t>(g.n);
    cs.partner = cv.get<int32_t>(g.n);
    cs.cdeg = cv.get<int32_t>(g.n);
    cs.rows = cv.get<int32_t>(4 * (int64_t)g.n);
    cs.row_cnt = cv.get<int32_t>(8);
    cs.tmp_adj = cv.get<int32_t>(g.nnz);
    cs.tmp_ew = cv.get<uint32_t>(g.nnz);
    cs.partials = cv.get<int64_t>(scan_tiles((int64_t)g.n + 1) + 1);
    cs.arrive = cv.get<unsigned>(ARRIVE_WORDS);
    cs.totals = cv.get<int64_t>(4);
    cs.hub_w1 = (int64_t)g.n / 32 + 1;
    cs.hub_words = cs.hub_w1 + cs.hub_w1 / 32 + 1;
    // as many hub slots as the accumulator budget allows (more long rows
    // merged at once), between HUB_SLOTS and HUB_SLOTS_MAX
    cs.hub_slots = (int32_t)std::max<int64_t>(
        HUB_SLOTS, std::min<int64_t>(HUB_SLOTS_MAX, HUB_BUDGET / (4 * ((int64_t)g.n + 1))));
    // large rows: the key-bucket merge wherever it applies (graphs with long
    // rows, or any graph once a large row has turned up); the dense hub
    // accumulators only where it may not (more than HUGE_NC_MAX nodes) and
    // for the one-workgroup tail, which merges every large row densely
    c.huge = (hubs || c.big_rows) ? 1 : 0;
    const bool dense = hubs && (g.n > HUGE_NC_MAX || tail);
    cs.hub_acc = dense ? cv.get<uint32_t>((int64_t)cs.hub_slots * g.n) : nullptr;
    cs.hub_bits = dense ? cv.get<uint32_t>((int64_t)cs.hub_slots * cs.hub_words) : nullptr;
    // rows whose bound exceeds ROW_MID_MAX at most (the bounds sum to at
    // most nnz): every row the key buckets may take
    cs.hg_rows = g.nnz / (ROW_MID_MAX + 1) + 64;
    cs.hg_cap = g.nnz / HG_WIN_MIN + 2 * cs.hg_rows;         // groups at most
    cs.hg_adj = c.huge ? cv.get<int32_t>(g.nnz) : nullptr;
    cs.hg_ew = c.huge ? cv.get<uint32_t>(g.nnz) : nullptr;
    cs.hg_small = c.huge ? cv.get<int4>(cs.hg_cap) : nullptr;
    cs.hg_big = c.huge ? cv.get<int4>(cs.hg_cap) : nullptr;
    cs.hg_slot = c.huge ? cv.get<int2>(cs.hg_cap) : nullptr;
    cs.hg_row = c.huge ? cv.get<int2>(cs.hg_rows) : nullptr;
    cs.hg_cnt = c.huge ? cv.get<int32_t>(4) : nullptr;
    // two-phase matcher (c.block_bits set before carving)
    ms.loc = c.block_bits >= 0 ? cv.get<int32_t>(g.n) : nullptr;
    ms.lkey = c.block_bits >= 0 ? cv.get<LocKey>(g.n) : nullptr;
    ms.hub = HubChunks{nullptr, nullptr, nullptr, 0, nullptr, nullptr};
    if (chunks) {
        ms.hub.cap = hub_chunk_cap(g.nnz);
        ms.hub.rec = cv.get<int2>(2 * ms.hub.cap);
        ms.hub.first = cv.get<int32_t>(2 * (int64_t)g.n);
        ms.hub.part = cv.get<Cand>(ms.hub.cap);
        ms.hub.scan = cv.get<int2>(2 * (int64_t)g.n);
        ms.hub.kfirst = cv.get<int32_t>(g.n);
    }
}

void fill_scratch(const DevGraph &g, const Ctx &c, hipStream_t s) {
    ZeroRanges z;
    z.add(c.cs.arrive, ARRIVE_WORDS);
    z.add(c.cs.row_cnt, 8);
    z.add(c.cs.totals, 4 * 2);
    z.add(c.ms.coop_bar, 2 + ARRIVE_WORDS);
    z.add(c.cs.hg_cnt, 4);
    // the matching state: list counters, round statistics, merge counts
    static_assert(sizeof(MatchState) % 4 == 0, "zeroed as words");
    z.add(c.ms.state, sizeof(MatchState) / 4);
    if (c.cs.hub_acc) {
        z.add(c.cs.hub_acc, (int64_t)c.cs.hub_slots * g.n);
        z.add(c.cs.hub_bits, (int64_t)c.cs.hub_slots * c.cs.hub_words);
    }
    launch_zero(z, s);
}

// Host-side level size estimate (grid sizing only; any value is correct):
// the newest level size the host has read back, shrunk geometrically by the
// ratio observed so far (0.6 per level before any read-back; power-law graphs
// shrink far more slowly than meshes).
struct SizeHint {
    int32_t n0, known_l = 0, known_n;
    double ratio = 0.6;
    explicit SizeHint(int32_t n) : n0(n), known_n(n) {}
    int32_t at(int l) const {
        double v = (double)known_n * std::pow(ratio, std::max(0, l - known_l));
        return (int32_t)std::max(1.0, std::min((double)n0, v));
    }
    void seen(int l, int32_t n) {
        if (l <= known_l || n <= 0) return;
        double r = std::pow((double)n / std::max(1, known_n), 1.0 / (l - known_l));
        ratio = std::min(1.0, std::max(0.3, r));
        known_l = l;
        known_n = n;
    }
};

// Multi-block matching rounds before the one-workgroup finisher: rounds_base
// for a level of at most rounds_n0 nodes, one more per factor rounds_growth,
// at most rounds_cap (the tuning table).  The compiled defaults (3, 2048, 8,
// 8) were measured on random geometric graphs: three rounds bring a level of
// ~2 K nodes below the finisher's threshold, and each further round covers
// about 8x more nodes.  A round launched after the pending set is small is a
// no-op of two launches; one not launched leaves more nodes to the finisher.
inline int rounds_for(int32_t n_hint, const Tune &t) {
    if (n_hint <= t.rounds_n0) return t.rounds_base;
    int r = t.rounds_base +
            (int)std::ceil(std::log((double)n_hint / t.rounds_n0) / std::log((double)t.rounds_growth));
    return std::min(r, t.rounds_cap);
}

struct HostControl {
    Control c;
};

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
    const int32_t *gid = nullptr;   // batched levels: graph of each node
    int32_t rounds = 0, grid_rounds = 0;
    int64_t matched = 0;
    int32_t stop = KAPPA_STOP_NONE;
    std::vector<int64_t> pointing, degsum;
    std::vector<int64_t> rescan, rescan_deg;   // rows rescanned per round, their degree sum
};

struct kappa_hierarchy {
    hipStream_t s = nullptr;
    std::vector<kappa_level> levels;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    Allocator al;   // the allocator of `arena`
    std::vector<std::shared_ptr<void>> holds;   // served form: the step arenas its levels live in
    ~kappa_hierarchy() { give_arena(s, arena, arena_bytes, al); }
};

namespace {

// Inputs of the batched form (a disjoint union of `count` graphs).
struct BatchIn {
    int32_t count;
    const int32_t *node_off;   // host, count + 1
    const int32_t *stop_n;     // host, count
    // served steps (BatchCtx): host arrays of count entries, the host flag
    // (device-visible address) and the levels of the first launch batch
    const uint64_t *gbase = nullptr;
    const int32_t *lmax = nullptr;
    const uint32_t *interrupt = nullptr;
    const uint32_t *interrupt_host = nullptr;   // the same flag, host address
    int first_batch = 0;
};
// Per-graph results of the batched form.
struct BatchOut {
    std::vector<std::vector<int32_t>> noff;   // per union level: first node of each graph
    std::vector<int32_t> coarsest, reason;    // per graph
};

// One attempt at the whole contraction phase with an arena of *arena_io
// bytes (raised to at least what level 0 needs; the size used is written
// back).  exact_cap: the device cursor stops at that size even if a larger
// recycled arena is handed out.  Returns KAPPA_OK and fills H, or a status;
// *retry_flags gets the control flags asking for another attempt (arena too
// small, hub accumulators).
kappa_status coarsen_attempt(const DevGraph &d0, int32_t maxdeg0, const kappa_coarsen_params *p,
                             hipStream_t s, uint64_t *arena_io, bool exact_cap, bool hubs,
                             const BatchIn *bi, kappa_hierarchy *H, BatchOut *bo,
                             uint32_t *retry_flags) {
    *retry_flags = 0;
    Ctx c;
    c.rating = p->rating;
    c.seed = p->seed;
    c.seed_direct = 0;
    c.block_bits = (p->flags & KAPPA_COARSEN_TWO_PHASE) ? p->block_bits : -1;
    // rows above BIN_MID_MAX get a block each per round: many blocks when the
    // graph has many (power-law graphs), few otherwise
    c.big_blocks = maxdeg0 > BIN_MID_MAX ? 1024 : 64;
    // graphs without long rows at level 0 rarely grow rows of thousands of
    // entries: such rows then take the hub accumulators (no big-row launch)
    c.big_rows = maxdeg0 > BIN_MID_MAX ? 1 : 0;
    c.rescan_stats = g_prof.on ? 1 : 0;
    const int maxl = p->max_levels;
    const int32_t count = bi ? bi->count : 0;
    uint32_t *bflag = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) {
            c.ctrl = cv.get<Control>(1);
            c.lv = cv.get<LevelDesc>(maxl + 2);
            carve_scratch(cv, d0, p->rating, hubs, c, maxdeg0 > BIN_MID_MAX,
                          !bi && g_tail_on && c.block_bits < 0);
            if (bi) {
                c.b.count = count;
                c.b.stall_num = p->stall_num;
                c.b.stall_den = p->stall_den;
                c.b.stop_n = cv.get<int32_t>(count);
                c.b.active = cv.get<uint8_t>(count);
                c.b.coarsest = cv.get<int32_t>(count);
                c.b.reason = cv.get<int32_t>(count);
                c.b.excl = cv.get<int32_t>(d0.n);
                if (bi->gbase) {
                    c.b.gbase = cv.get<uint64_t>(count);
                    c.b.gseed = cv.get<uint64_t>(count);
                    c.b.lmax = cv.get<int32_t>(count);
                    c.b.stop_seen = cv.get<uint32_t>(1);
                    c.b.interrupt = bi->interrupt;
                }
                bflag = cv.get<uint32_t>(1);
            }
        }))
        return KAPPA_E_NOMEM;
    // level 0's mate and cmap (and, batched, its graph ids and offsets)
    // open the arena
    const uint64_t n_al = ((uint64_t)d0.n * 4 + 255) & ~(uint64_t)255;
    const uint64_t g_al = ((uint64_t)(count + 1) * 4 + 255) & ~(uint64_t)255;
    const uint64_t opening = bi ? 3 * n_al + g_al : 2 * n_al;
    const uint64_t arena_bytes = std::max<uint64_t>(*arena_io, opening);
    *arena_io = arena_bytes;
    size_t arena_got = 0;
    Allocator arena_al;
    void *arena = take_arena(s, arena_bytes, &arena_got, &arena_al);
    if (!arena) return KAPPA_E_NOMEM;
    // a recycled arena may be larger than asked for: all of it is usable
    const uint64_t cap = exact_cap ? arena_bytes : arena_got;
    ArenaHold hold{s, arena, arena_got, arena_al};
    fill_scratch(d0, c, s);

    // control block and level 0
    struct Init {
        Control ctrl;
        LevelDesc l0;
    };
    Init *in = (Init *)pinned(sizeof(Init));
    std::memset(in, 0, sizeof(Init));
    in->ctrl.done = 0;
    in->ctrl.nlevels = 1;
    in->ctrl.flags = 0;
    int32_t *gid0 = bi ? (int32_t *)((char *)arena + 2 * n_al) : nullptr;
    int32_t *noff0 = bi ? (int32_t *)((char *)arena + 3 * n_al) : nullptr;
    in->ctrl.cursor = opening;
    in->ctrl.cap = cap;
    in->ctrl.base = (char *)arena;
    // batched: size and stall rules apply per graph (batch_begin / batch_end)
    in->ctrl.stop_n = bi ? -1 : p->stop_n;
    in->ctrl.max_levels = maxl;
    in->ctrl.stall_num = bi ? 0 : p->stall_num;
    in->ctrl.stall_den = p->stall_den;
    in->l0.n = d0.n;
    in->l0.maxdeg = maxdeg0;
    in->l0.nnz = d0.nnz;
    in->l0.xadj = const_cast<int64_t *>(d0.xadj);
    in->l0.adj = const_cast<int32_t *>(d0.adj);
    in->l0.ew = const_cast<uint32_t *>(d0.ew);
    in->l0.vw = const_cast<uint32_t *>(d0.vw);
    in->l0.mate = (int32_t *)arena;
    in->l0.cmap = (int32_t *)((char *)arena + n_al);
    in->l0.gid = gid0;
    in->l0.noff = noff0;
    in->l0.phase = PH_IDLE;
    if (bi) {
        HIPCHK(hipMemcpyAsync(noff0, bi->node_off, (size_t)(count + 1) * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync((void *)c.b.stop_n, bi->stop_n, (size_t)count * 4,
                              hipMemcpyHostToDevice, s));
        if (bi->gbase) {
            HIPCHK(hipMemcpyAsync((void *)c.b.gbase, bi->gbase, (size_t)count * 8,
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync((void *)c.b.lmax, bi->lmax, (size_t)count * 4,
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemsetAsync(c.b.stop_seen, 0, sizeof(uint32_t), s));
        }
        HIPCHK(hipMemsetAsync(c.b.active, 1, (size_t)count, s));
        HIPCHK(hipMemsetAsync(c.b.coarsest, 0xff, (size_t)count * 4, s));
        HIPCHK(hipMemsetAsync(c.b.reason, 0, (size_t)count * 4, s));
        HIPCHK(hipMemsetAsync(bflag, 0, sizeof(uint32_t), s));
        launch_batch_gid(noff0, count, d0.n, gid0, s);
        DevGraph db = d0;
        db.gid = gid0;
        db.noff = noff0;
        launch_batch_check(db, bflag, s);
        uint32_t *hf = (uint32_t *)pinned(sizeof(uint32_t));
        HIPCHK(hipMemcpyAsync(hf, bflag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (*hf) return KAPPA_E_GRAPH;   // an edge joins two graphs of the batch
    }
    // every descriptor past level 0 starts idle (zero): kernels of levels not
    // built yet are no-ops
    launch_init_levels(c.ctrl, c.lv, maxl + 2, in->ctrl, in->l0, s);

    // levels in batches; one read-back per batch
    const int32_t n0 = d0.n;
    int first = (int)std::ceil(std::log(std::max(2.0, (double)n0 / std::max(1, p->stop_n))) /
                               std::log(1.0 / 0.6)) + 2;
    if (bi && bi->first_batch > 0) first = bi->first_batch;
    int launched = 0, batch = std::max(1, std::min(first, maxl + 1));
    // The tail kernel is tried ahead of each level past level 0 whose size
    // estimate is near its limit; once the estimate is within twice the limit
    // the batch ends on the tail launch (it most likely finishes the loop).
    // If it did not take that level, the next batch runs the level in full.
    const bool tail_on = !bi && g_tail_on && c.block_bits < 0;
    int tail_end = -1;   // level at which the previous batch ended on a tail launch
    // a level whose finisher handed it back (CF_EXTEND): the next batch
    // starts by giving it more grid rounds after round ext_round
    int ext_level = -1, ext_round = 0, ext_times = 0, ext_seen = -1;
    // served steps: the host saw the interrupt, so the next launch is the
    // next level's start alone (it ends the step there)
    bool begin_only = false;
    // power-law graphs hand levels back: small batches keep the levels
    // launched behind a handed-back one (no-ops then) few
    if (c.big_blocks > 64) batch = std::min(batch, 2);
    Control *hc = (Control *)pinned(sizeof(Control));
    SizeHint hint(n0);
    for (;;) {
        const int l_end = std::min(launched + batch, maxl + 1);
        int next = l_end;
        uint64_t ratio_bits;
        std::memcpy(&ratio_bits, &hint.ratio, sizeof ratio_bits);
        const std::vector<uint64_t> key = {1, pkey(w->base), (uint64_t)n0, (uint64_t)d0.nnz,
                                           (uint64_t)hint.known_l, (uint64_t)hint.known_n, ratio_bits,
                                           (uint64_t)p->rating, p->seed, (uint64_t)maxl,
                                           (uint64_t)hubs, (uint64_t)launched, (uint64_t)l_end,
                                           (uint64_t)count, (uint64_t)tail_on,
                                           (uint64_t)(int64_t)tail_end,
                                           (uint64_t)(int64_t)c.block_bits,
                                           (uint64_t)(int64_t)ext_level, (uint64_t)ext_round,
                                           (uint64_t)begin_only};
        HIPCHK(run_seq(w->c, s, key, [&](hipStream_t q) {
            if (begin_only) {
                launch_batch_begin(c, launched, q);
                next = launched;
                return;
            }
            for (int l = launched; l < l_end; ++l) {
                int32_t nh = hint.at(l);
                if (l == ext_level) {
                    launch_level_extend(c, l, nh, n0, ext_round,
                                        EXTEND_ROUNDS << std::min(ext_times, 3), true, q);
                    continue;
                }
                const bool try_tail = tail_on && l >= 1 && nh <= 8 * TAIL_MAX_N;
                if (try_tail) launch_tail(c, l, q);
                if (try_tail && nh <= 2 * TAIL_MAX_N && l != tail_end) {
                    next = l;
                    break;
                }
                // innerOuter on unit input weights ranks edges by degree
                // sums, which chains level 0 over many rounds (17 grid rounds
                // on the random geometric graph of 2^20 nodes); the finisher
                // completes any remainder
                int rounds = rounds_for(nh, c.t);
                if (l == 0 && p->rating == KAPPA_INNER_OUTER) rounds = 18;
                launch_level(c, l, nh, d0.nnz, n0, rounds, q);
            }
        }));
        if (next < l_end && !begin_only) tail_end = next;
        launched = next;
        HIPCHK(hipMemcpyAsync(hc, c.ctrl, sizeof(Control), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        hint.seen(hc->nlevels - 1, hc->last_n);
        ext_level = -1;
        if ((hc->flags & CF_EXTEND) && !(hc->flags & ~(uint32_t)CF_EXTEND)) {
            // resume the level on the grid; the kernels after it in this
            // batch were no-ops (the level was still matching)
            ext_level = hc->ext_level;
            ext_round = hc->ext_round;
            ext_times = ext_level == ext_seen ? ext_times + 1 : 0;
            ext_seen = ext_level;
            hc->flags &= ~(uint32_t)CF_EXTEND;
            hc->done = 0;
            HIPCHK(hipMemcpyAsync(c.ctrl, hc, sizeof(Control), hipMemcpyHostToDevice, s));
            launched = ext_level;
            batch = 1;   // the resumed level alone: it may be handed back again
            continue;
        }
        if (hc->done || launched > maxl) break;
        batch = c.big_blocks > 64 ? 2 : 4;
        if (bi && bi->gbase) {
            // served steps end at the next boundary once a graph stops or the
            // host interrupts: launch two levels at a time (each launched
            // level costs its kernels' launches even when it turns out idle),
            // and only the next level's start once the host has interrupted
            // (if that start did not end the step, the level runs in full)
            const bool intr = !begin_only && launched > 0 && bi->interrupt_host &&
                              __atomic_load_n(bi->interrupt_host, __ATOMIC_ACQUIRE) != 0;
            begin_only = intr;
            batch = 2;
        }
    }
    if (hc->flags && debug_on())
        fprintf(stderr, "kappa: coarsen control flags 0x%x (levels %d)\n", hc->flags, hc->nlevels);
    if (hc->flags & (CF_ARENA | CF_HUBS)) {
        *retry_flags = hc->flags;
        return KAPPA_E_NOMEM;
    }
    if (hc->flags & (CF_ROUNDS | CF_STATE)) {
        return KAPPA_E_HIP;
    }
    // read the level descriptors back
    const int nl = hc->nlevels;
    if ((size_t)nl * sizeof(LevelDesc) > PIN_REGION_BYTES) {
        return KAPPA_E_NOMEM;
    }
    LevelDesc *hl = (LevelDesc *)pinned((size_t)nl * sizeof(LevelDesc), PIN_LEVELS);
    HIPCHK(hipMemcpyAsync(hl, c.lv, (size_t)nl * sizeof(LevelDesc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    H->levels.clear();
    for (int l = 0; l < nl; ++l) {
        kappa_level L;
        L.n = hl[l].n;
        L.nnz = hl[l].nnz;
        L.maxdeg = hl[l].maxdeg;
        L.xadj = hl[l].xadj;
        L.adj = hl[l].adj;
        L.ew = hl[l].ew;
        L.vw = hl[l].vw;
        L.cmap = l + 1 < nl ? hl[l].cmap : nullptr;
        L.mate = hl[l].mate;
        L.gid = hl[l].gid;
        L.rounds = hl[l].rounds;
        L.grid_rounds = hl[l].grid_rounds;
        L.matched = hl[l].matched;
        L.stop = hl[l].stop;
        if (l + 1 < nl || L.stop == KAPPA_STOP_EMPTY) {
            int keep = std::min(L.rounds, STAT_ROUNDS);
            for (int i = 0; i < keep; ++i) {
                L.pointing.push_back(hl[l].stat[i][0]);
                L.degsum.push_back(hl[l].stat[i][1]);
                L.rescan.push_back(hl[l].stat[i][2]);
                L.rescan_deg.push_back(hl[l].stat[i][3]);
            }
        } else {
            L.rounds = 0;
            L.grid_rounds = 0;
            L.matched = 0;
        }
        if (l + 1 < nl) L.stop = KAPPA_STOP_NONE;
        H->levels.push_back(L);
    }
    if (bi) {
        bo->noff.assign(nl, std::vector<int32_t>(count + 1));
        for (int l = 0; l < nl; ++l)
            HIPCHK(hipMemcpyAsync(bo->noff[l].data(), hl[l].noff, (size_t)(count + 1) * 4,
                                  hipMemcpyDeviceToHost, s));
        bo->coarsest.assign(count, 0);
        bo->reason.assign(count, 0);
        HIPCHK(hipMemcpyAsync(bo->coarsest.data(), c.b.coarsest, (size_t)count * 4,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(bo->reason.data(), c.b.reason, (size_t)count * 4,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const int32_t last_stop = hl[nl - 1].stop;
        for (int32_t g = 0; g < count; ++g)
            if (bo->coarsest[g] < 0) {   // still coarsening when the union stopped
                bo->coarsest[g] = nl - 1;
                bo->reason[g] = last_stop;
            }
    }
    H->arena = hold.release();
    H->arena_bytes = arena_got;
    H->al = arena_al;
    return KAPPA_OK;
}

}  // namespace

namespace {
// two_phase_ok: the two-phase matcher may be asked for (single-graph forms)
bool params_ok(const kappa_coarsen_params *p, bool two_phase_ok) {
    const uint32_t known = KAPPA_COARSEN_TRUSTED | (two_phase_ok ? KAPPA_COARSEN_TWO_PHASE : 0u);
    if (!p || p->rating < 0 || p->rating > 4 || p->max_levels < 0 || p->max_levels > MAX_LEVELS ||
        (p->stall_num > 0 && p->stall_den == 0) || (p->flags & ~known))
        return false;
    return !(p->flags & KAPPA_COARSEN_TWO_PHASE) ||
           (p->block_bits >= 0 && p->block_bits <= BM_BITS_MAX);
}
}  // namespace

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
    int32_t *tr = nullptr;
    uint32_t *out = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) {
            tr = cv.get<int32_t>(tile_rows_needed(d.nnz));
            out = rating == KAPPA_INNER_OUTER ? cv.get<uint32_t>(d.n) : nullptr;
        }))
        return KAPPA_E_NOMEM;
    launch_tile_rows(d, tr, s);
    if (out) launch_out(d, tr, out, s);
    launch_rate(d, tr, rating, out, num, den, s);
    HIPCHK(hipGetLastError());
    return KAPPA_OK;
}

extern "C" kappa_status kappa_coarsen(const kappa_graph *g, const kappa_coarsen_params *p,
                                      kappa_hierarchy **out, kappa_stream_t stream) {
    if (!out) return KAPPA_E_ARG;
    *out = nullptr;
    if (!graph_args_ok(g) || !p) return KAPPA_E_ARG;
    if (!params_ok(p, true)) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d0 = dev(g);
    int32_t maxdeg = 0;
    kappa_status st = validate_impl(d0, s, &maxdeg, (p->flags & KAPPA_COARSEN_TRUSTED) != 0);
    if (st != KAPPA_OK) return st;

    kappa_hierarchy *H = new (std::nothrow) kappa_hierarchy();
    if (!H) return KAPPA_E_NOMEM;
    H->s = s;
    // arena: every level's nodes (vw, xadj, mate, cmap: 24 B) and entries
    // (adj, ew: 8 B), three times level 0 to start with
    uint64_t lvl0 = (uint64_t)d0.n * 24 + (uint64_t)d0.nnz * 8 + 4096;
    const uint64_t forced = g_arena_first.load();
    // graphs with rows above BIN_MID_MAX entries (power-law graphs) shrink
    // slowly: their hierarchies take five to six times level 0
    uint64_t arena = forced ? forced : (maxdeg > BIN_MID_MAX ? 8 : 3) * lvl0 + (1u << 20);
    bool hubs = 2 * (int64_t)maxdeg - 2 > ROW_MID_MAX / 8;
    for (int attempt = 0; attempt < 6; ++attempt) {
        uint32_t retry = 0;
        st = coarsen_attempt(d0, maxdeg, p, s, &arena, forced != 0, hubs, nullptr, H, nullptr,
                             &retry);
        if (debug_on())
            fprintf(stderr, "kappa: coarsen attempt %d arena %llu: status %d, retry flags 0x%x\n",
                    attempt, (unsigned long long)arena, (int)st, retry);
        if (st == KAPPA_OK) break;
        if (!retry) break;
        if (retry & CF_ARENA) arena *= 4;
        if (retry & CF_HUBS) hubs = true;
    }
    if (st != KAPPA_OK) {
        delete H;
        return st;
    }
    *out = H;
    return KAPPA_OK;
}

// ===========================================================================
// Batched form
// ===========================================================================
struct kappa_batch {
    kappa_hierarchy union_h;   // the union's levels (owns the arena)
    int32_t count = 0;
    BatchOut out;
    // the union itself when the library built it (kappa_coarsen_graphs)
    void *umem = nullptr;
    size_t umem_bytes = 0;
    Allocator umem_al;
    ~kappa_batch() { give_arena(union_h.s, umem, umem_bytes, umem_al); }
};

namespace {


// The batched coarsening of union u into B (B->union_h.s set); arguments checked.
kappa_status batch_impl(const kappa_graph *u, int32_t count, const int32_t *node_off,
                        const int32_t *stop_n, const kappa_coarsen_params *p, kappa_batch *B,
                        hipStream_t s) {
    DevGraph d0 = dev(u);
    int32_t maxdeg = 0;
    kappa_status st = validate_impl(d0, s, &maxdeg, (p->flags & KAPPA_COARSEN_TRUSTED) != 0);
    if (st != KAPPA_OK) return st;
    std::vector<int32_t> sn(count, p->stop_n);
    if (stop_n) sn.assign(stop_n, stop_n + count);
    BatchIn bi{count, node_off, sn.data()};
    B->count = count;
    // arena: every level's nodes (vw, xadj, mate, cmap, graph id: 28 B),
    // entries (8 B) and graph offsets, three times level 0 to start with
    uint64_t lvl0 = (uint64_t)d0.n * 28 + (uint64_t)d0.nnz * 8 + (uint64_t)(count + 1) * 4 + 8192;
    const uint64_t forced = g_arena_first.load();
    uint64_t arena = forced ? forced : 3 * lvl0 + (uint64_t)(count + 1) * 4 * 64 + (1u << 20);
    bool hubs = 2 * (int64_t)maxdeg - 2 > ROW_MID_MAX / 8;
    for (int attempt = 0; attempt < 6; ++attempt) {
        uint32_t retry = 0;
        st = coarsen_attempt(d0, maxdeg, p, s, &arena, forced != 0, hubs, &bi, &B->union_h,
                             &B->out, &retry);
        if (debug_on())
            fprintf(stderr, "kappa: batch attempt %d arena %llu: status %d, retry flags 0x%x\n",
                    attempt, (unsigned long long)arena, (int)st, retry);
        if (st == KAPPA_OK) break;
        if (!retry) break;
        if (retry & CF_ARENA) arena *= 4;
        if (retry & CF_HUBS) hubs = true;
    }
    return st;
}

}  // namespace

extern "C" kappa_status kappa_coarsen_batch(const kappa_graph *u, int32_t count,
                                            const int32_t *node_off, const int32_t *stop_n,
                                            const kappa_coarsen_params *p, kappa_batch **out,
                                            kappa_stream_t stream) {
    if (!out) return KAPPA_E_ARG;
    *out = nullptr;
    if (!graph_args_ok(u) || !params_ok(p, false) || count < 1 || !node_off) return KAPPA_E_ARG;
    if (node_off[0] != 0 || node_off[count] != u->n) return KAPPA_E_ARG;
    for (int32_t g = 0; g < count; ++g)
        if (node_off[g + 1] < node_off[g]) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    kappa_batch *B = new (std::nothrow) kappa_batch();
    if (!B) return KAPPA_E_NOMEM;
    B->union_h.s = s;
    const kappa_status st = batch_impl(u, count, node_off, stop_n, p, B, s);
    if (st != KAPPA_OK) {
        delete B;
        return st;
    }
    *out = B;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_coarsen_graphs(const kappa_graph *graphs, int32_t count,
                                             const int32_t *stop_n, const kappa_coarsen_params *p,
                                             kappa_batch **out, kappa_stream_t stream) {
    if (!out) return KAPPA_E_ARG;
    *out = nullptr;
    if (!graphs || count < 1 || !params_ok(p, false)) return KAPPA_E_ARG;
    std::vector<int64_t> off(2 * ((size_t)count + 1), 0);   // node offsets, then entry offsets
    int64_t *noff = off.data(), *eoff = off.data() + count + 1;
    std::vector<UnionSrc> src(count);
    for (int32_t g = 0; g < count; ++g) {
        if (!graph_args_ok(&graphs[g])) return KAPPA_E_ARG;
        noff[g + 1] = noff[g] + graphs[g].n;
        eoff[g + 1] = eoff[g] + graphs[g].nnz;
        src[g] = UnionSrc{graphs[g].xadj, graphs[g].adj, graphs[g].ew, graphs[g].vw};
    }
    const int64_t n = noff[count], nnz = eoff[count];
    if (n > INT32_MAX) return KAPPA_E_ARG;
    std::vector<int32_t> node_off(count + 1);
    for (int32_t g = 0; g <= count; ++g) node_off[g] = (int32_t)noff[g];
    hipStream_t s = S(stream);
    kappa_batch *B = new (std::nothrow) kappa_batch();
    if (!B) return KAPPA_E_NOMEM;
    B->union_h.s = s;
    // the union's arrays (library-owned, freed with the batch)
    Carve lay;
    int64_t *uxadj = nullptr;
    int32_t *uadj = nullptr;
    uint32_t *uew = nullptr, *uvw = nullptr;
    auto layout = [&](Carve &cv) {
        uxadj = cv.get<int64_t>(n + 1);
        uadj = cv.get<int32_t>(nnz);
        uew = cv.get<uint32_t>(nnz);
        uvw = cv.get<uint32_t>(n);
    };
    layout(lay);
    size_t got = 0;
    B->umem = take_arena(s, lay.off, &got, &B->umem_al);
    if (!B->umem) {
        delete B;
        return KAPPA_E_NOMEM;
    }
    B->umem_bytes = got;
    Carve real;
    real.base = (char *)B->umem;
    layout(real);
    {
        UnionSrc *dsrc = nullptr;
        int64_t *doff = nullptr;
        std::unique_ptr<Workspace> w;
        if (!carve_workspace(s, w, [&](Carve &cv) {
                dsrc = cv.get<UnionSrc>(count);
                doff = cv.get<int64_t>(2 * ((int64_t)count + 1));
            })) {
            delete B;
            return KAPPA_E_NOMEM;
        }
        kappa_status st = KAPPA_OK;
        if (hipMemcpyAsync(dsrc, src.data(), sizeof(UnionSrc) * count, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice,
                           s) != hipSuccess)
            st = KAPPA_E_HIP;
        if (st == KAPPA_OK) {
            launch_union_build(dsrc, count, doff, doff + count + 1, n, nnz, uxadj, uadj, uew, uvw, s);
            if (hipGetLastError() != hipSuccess) st = KAPPA_E_HIP;
        }
        // the descriptors are read by the union kernels before the next holder
        // of the workspace (stream order); the host vectors must outlive the
        // copies, which are staged from pageable memory before they return
        if (st != KAPPA_OK) {
            delete B;
            return st;
        }
    }
    kappa_graph u{(int32_t)n, nnz, uxadj, uadj, uew, uvw};
    const kappa_status st = batch_impl(&u, count, node_off.data(), stop_n, p, B, s);
    if (st != KAPPA_OK) {
        delete B;
        return st;
    }
    *out = B;
    return KAPPA_OK;
}

extern "C" int32_t kappa_batch_count(const kappa_batch *b) { return b ? b->count : 0; }

extern "C" kappa_status kappa_batch_graph_info(const kappa_batch *b, int32_t g, int32_t *levels,
                                               int32_t *stop_reason) {
    if (!b || g < 0 || g >= b->count) return KAPPA_E_ARG;
    if (levels) *levels = b->out.coarsest[g] + 1;
    if (stop_reason) *stop_reason = b->out.reason[g];
    return KAPPA_OK;
}

extern "C" kappa_status kappa_batch_hierarchy(const kappa_batch *b, int32_t g,
                                              kappa_hierarchy **out, kappa_stream_t stream) {
    if (!out) return KAPPA_E_ARG;
    *out = nullptr;
    if (!b || g < 0 || g >= b->count) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    const int32_t L = b->out.coarsest[g];
    const auto &U = b->union_h.levels;
    // node and entry ranges of the graph on every level
    std::vector<int32_t> na(L + 1), nb(L + 1);
    std::vector<int64_t> ea(L + 1), eb(L + 1);
    for (int32_t l = 0; l <= L; ++l) {
        na[l] = b->out.noff[l][g];
        nb[l] = b->out.noff[l][g + 1];
        int64_t e2[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(&e2[0], U[l].xadj + na[l], sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&e2[1], U[l].xadj + nb[l], sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ea[l] = e2[0];
        eb[l] = e2[1];
    }
    Carve lay;
    struct Arr {
        int64_t *xadj;
        int32_t *adj, *cmap, *mate;
        uint32_t *ew, *vw;
    };
    std::vector<Arr> arr(L + 1);
    auto layout = [&](Carve &cv) {
        for (int32_t l = 0; l <= L; ++l) {
            const int64_t n = nb[l] - na[l], nnz = eb[l] - ea[l];
            arr[l].xadj = cv.get<int64_t>(n + 1);
            arr[l].adj = cv.get<int32_t>(nnz);
            arr[l].ew = cv.get<uint32_t>(nnz);
            arr[l].vw = cv.get<uint32_t>(n);
            arr[l].cmap = cv.get<int32_t>(n);
            arr[l].mate = cv.get<int32_t>(n);
        }
    };
    layout(lay);
    std::unique_ptr<kappa_hierarchy> H(new (std::nothrow) kappa_hierarchy());
    if (!H) return KAPPA_E_NOMEM;
    H->s = s;
    size_t got = 0;
    void *arena = take_arena(s, lay.off, &got, &H->al);
    if (!arena) return KAPPA_E_NOMEM;
    H->arena = arena;
    H->arena_bytes = got;
    Carve real;
    real.base = (char *)arena;
    layout(real);
    for (int32_t l = 0; l <= L; ++l) {
        const kappa_level &src = U[l];
        DevGraph du;
        du.n = src.n; du.nnz = src.nnz; du.xadj = src.xadj; du.adj = src.adj; du.ew = src.ew;
        du.vw = src.vw;
        const bool has_next = l < L;
        launch_batch_extract(du, has_next ? src.cmap : nullptr, has_next ? src.mate : nullptr,
                             na[l], nb[l], ea[l], eb[l] - ea[l], has_next ? b->out.noff[l + 1][g] : 0,
                             arr[l].xadj, arr[l].adj, arr[l].ew, arr[l].vw, arr[l].cmap,
                             arr[l].mate, s);
        kappa_level lv;
        lv.n = nb[l] - na[l];
        lv.nnz = eb[l] - ea[l];
        lv.xadj = arr[l].xadj;
        lv.adj = arr[l].adj;
        lv.ew = arr[l].ew;
        lv.vw = arr[l].vw;
        lv.cmap = has_next ? arr[l].cmap : nullptr;
        lv.mate = has_next ? arr[l].mate : nullptr;
        lv.matched = has_next ? (int64_t)lv.n - (b->out.noff[l + 1][g + 1] - b->out.noff[l + 1][g]) : 0;
        lv.rounds = 0;   // rounds are counted for the union, not per graph
        lv.stop = has_next ? KAPPA_STOP_NONE : b->out.reason[g];
        H->levels.push_back(lv);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    *out = H.release();
    return KAPPA_OK;
}

extern "C" void kappa_batch_free(kappa_batch *b) { delete b; }

namespace {
// One matching of g (block_bits < 0: local-max rounds; otherwise the
// two-phase matcher, whose block matching is copied to block_mate if given).
kappa_status match_once(const kappa_graph *g, int32_t rating, uint64_t level_seed,
                        int32_t block_bits, int32_t *mate, int32_t *block_mate,
                        int32_t *rounds_out, int64_t *matched_out, kappa_stream_t stream) {
    if (!graph_args_ok(g) || rating < 0 || rating > 4) return KAPPA_E_ARG;
    if (g->n > 0 && !mate) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d = dev(g);
    Ctx c;
    c.rating = rating;
    c.seed = level_seed;   // used as is: h(e) = mix64(level_seed ^ eid)
    c.seed_direct = 1;
    c.block_bits = block_bits;
    int32_t *cm = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) {
            c.ctrl = cv.get<Control>(1);
            c.lv = cv.get<LevelDesc>(2);
            cm = cv.get<int32_t>(d.n);
            carve_scratch(cv, d, rating, false, c, true);
        }))
        return KAPPA_E_NOMEM;
    fill_scratch(d, c, s);
    struct Init {
        Control ctrl;
        LevelDesc l0;
    };
    Init *in = (Init *)pinned(sizeof(Init));
    std::memset(in, 0, sizeof(Init));
    in->ctrl.nlevels = 1;
    in->ctrl.stop_n = -1;
    in->ctrl.max_levels = MAX_LEVELS;
    in->l0.n = d.n;
    in->l0.nnz = d.nnz;
    in->l0.xadj = const_cast<int64_t *>(d.xadj);
    in->l0.adj = const_cast<int32_t *>(d.adj);
    in->l0.ew = const_cast<uint32_t *>(d.ew);
    in->l0.vw = const_cast<uint32_t *>(d.vw);
    in->l0.mate = mate;
    in->l0.cmap = cm;
    in->l0.phase = PH_IDLE;
    launch_init_levels(c.ctrl, c.lv, 2, in->ctrl, in->l0, s);
    launch_level_match(c, 0, d.n, d.nnz, 24, false, true, s);
    LevelDesc *hl = (LevelDesc *)pinned(sizeof(LevelDesc), PIN_LEVELS);
    Control *hc = (Control *)pinned(sizeof(Control));
    for (;;) {
        HIPCHK(hipMemcpyAsync(hl, c.lv, sizeof(LevelDesc), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hc, c.ctrl, sizeof(Control), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!(hc->flags & CF_EXTEND)) break;
        // the finisher handed the matching back: more grid rounds
        const int r_from = hc->ext_round;
        hc->flags &= ~(uint32_t)CF_EXTEND;
        hc->done = 0;
        HIPCHK(hipMemcpyAsync(c.ctrl, hc, sizeof(Control), hipMemcpyHostToDevice, s));
        launch_level_extend(c, 0, d.n, d.n, r_from, EXTEND_ROUNDS, false, s);
    }
    if (hc->flags & (CF_ROUNDS | CF_STATE)) {
        if (debug_on()) fprintf(stderr, "kappa: match control flags 0x%x\n", hc->flags);
        return KAPPA_E_HIP;
    }
    if (block_mate && d.n > 0) {
        HIPCHK(hipMemcpyAsync(block_mate, c.ms.loc, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (rounds_out) *rounds_out = hl->rounds;
    if (matched_out) *matched_out = hl->matched;
    return KAPPA_OK;
}
}  // namespace

extern "C" kappa_status kappa_match(const kappa_graph *g, int32_t rating, uint64_t level_seed,
                                    int32_t *mate, int32_t *rounds_out, int64_t *matched_out,
                                    kappa_stream_t stream) {
    return match_once(g, rating, level_seed, -1, mate, nullptr, rounds_out, matched_out, stream);
}

extern "C" kappa_status kappa_match_two_phase(const kappa_graph *g, int32_t rating,
                                              uint64_t level_seed, int32_t block_bits,
                                              int32_t *mate, int32_t *block_mate,
                                              int64_t *matched_out, kappa_stream_t stream) {
    if (block_bits < 0 || block_bits > BM_BITS_MAX) return KAPPA_E_ARG;
    return match_once(g, rating, level_seed, block_bits, mate, block_mate, nullptr, matched_out,
                      stream);
}

extern "C" kappa_status kappa_rcb_order(const double *xy, int32_t n, int32_t leaf, int32_t *order,
                                        kappa_stream_t stream) {
    if (n < 0 || leaf < 1 || (n > 0 && (!xy || !order))) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    size_t need = 0;
    kappa_status st = rcb_order_impl(xy, n, leaf, order, s, nullptr, 0, &need);
    if (st != KAPPA_OK) return st;
    char *buf = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) { buf = cv.get<char>((int64_t)need); }))
        return KAPPA_E_NOMEM;
    return rcb_order_impl(xy, n, leaf, order, s, buf, need, &need);
}

extern "C" kappa_status kappa_relabel(const kappa_graph *g, const int32_t *order,
                                      kappa_graph_out *out, kappa_stream_t stream) {
    if (!graph_args_ok(g) || !out) return KAPPA_E_ARG;
    if (g->n > 0 && (!order || !out->vw)) return KAPPA_E_ARG;
    if (!out->xadj || (g->nnz > 0 && (!out->adj || !out->ew))) return KAPPA_E_ARG;
    if (g->nnz > INT32_MAX) return KAPPA_E_ARG;   // the radix sorts count items in int
    if (out->cap_n < g->n || out->cap_nnz < g->nnz) return KAPPA_E_CAPACITY;
    hipStream_t s = S(stream);
    DevGraph d = dev(g);
    size_t need = 0;
    kappa_status st = relabel_impl(d, order, out->xadj, out->adj, out->ew, out->vw, s, nullptr, 0,
                                   &need, nullptr);
    if (st != KAPPA_OK) return st;
    uint32_t *hflag = (uint32_t *)pinned(sizeof(uint32_t));
    if (!hflag) return KAPPA_E_NOMEM;
    char *buf = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) { buf = cv.get<char>((int64_t)need); }))
        return KAPPA_E_NOMEM;
    st = relabel_impl(d, order, out->xadj, out->adj, out->ew, out->vw, s, buf, need, &need, hflag);
    if (st != KAPPA_OK) return st;
    out->n = g->n;
    out->nnz = g->nnz;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_contract(const kappa_graph *g, const int32_t *mate, int32_t *cmap,
                                       kappa_graph_out *coarse, kappa_stream_t stream) {
    if (!graph_args_ok(g) || !coarse) return KAPPA_E_ARG;
    if (g->n > 0 && (!mate || !cmap || !coarse->vw)) return KAPPA_E_ARG;
    if (!coarse->xadj || coarse->cap_n < 0 || coarse->cap_nnz < 0) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    DevGraph d = dev(g);
    // the coarse level: vw, xadj, mate, cmap (20 B per node), adj, ew
    const uint64_t arena_bytes = (uint64_t)d.n * 20 + (uint64_t)d.nnz * 8 + 8192;
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool hubs = attempt > 0;
        uint32_t *flag = nullptr;
        char *arena = nullptr;
        Ctx c;
        c.rating = 0;
        c.seed = 0;
        c.seed_direct = 0;
        std::unique_ptr<Workspace> w;
        if (!carve_workspace(s, w, [&](Carve &cv) {
                flag = cv.get<uint32_t>(1);
                c.ctrl = cv.get<Control>(1);
                c.lv = cv.get<LevelDesc>(2);
                carve_scratch(cv, d, 0, hubs, c);
                arena = cv.get<char>((int64_t)arena_bytes);
            }))
            return KAPPA_E_NOMEM;
        if (attempt == 0) {
            launch_fill_u32(flag, 1, 0, s);
            launch_check_matching(d, mate, flag, s);
            uint32_t *hf = (uint32_t *)pinned(sizeof(uint32_t));
            HIPCHK(hipMemcpyAsync(hf, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (*hf) return KAPPA_E_ARG;
        }
        fill_scratch(d, c, s);
        struct Init {
            Control ctrl;
            LevelDesc l0;
        };
        Init *in = (Init *)pinned(sizeof(Init));
        std::memset(in, 0, sizeof(Init));
        in->ctrl.nlevels = 1;
        in->ctrl.stop_n = -1;
        in->ctrl.max_levels = MAX_LEVELS;
        in->ctrl.cap = arena_bytes;
        in->ctrl.base = arena;
        in->l0.n = d.n;
        in->l0.nnz = d.nnz;
        in->l0.xadj = const_cast<int64_t *>(d.xadj);
        in->l0.adj = const_cast<int32_t *>(d.adj);
        in->l0.ew = const_cast<uint32_t *>(d.ew);
        in->l0.vw = const_cast<uint32_t *>(d.vw);
        in->l0.mate = const_cast<int32_t *>(mate);
        in->l0.cmap = cmap;
        in->l0.phase = PH_CONTRACT;
        launch_init_levels(c.ctrl, c.lv, 2, in->ctrl, in->l0, s);
        launch_level_contract(c, 0, d.n, d.n, s);
        struct RB {
            Control ctrl;
            LevelDesc l1;
        };
        RB *rb = (RB *)pinned(sizeof(RB), PIN_LEVELS);
        HIPCHK(hipMemcpyAsync(&rb->ctrl, c.ctrl, sizeof(Control), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&rb->l1, c.lv + 1, sizeof(LevelDesc), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (rb->ctrl.flags & CF_HUBS) continue;
        if (rb->ctrl.flags & CF_ARENA || rb->ctrl.nlevels != 2) return KAPPA_E_NOMEM;
        int32_t nc = rb->l1.n;
        int64_t nnzc = rb->l1.nnz;
        coarse->n = nc;
        coarse->nnz = nnzc;
        if (nc > coarse->cap_n || nnzc > coarse->cap_nnz) return KAPPA_E_CAPACITY;
        if (nnzc > 0 && (!coarse->adj || !coarse->ew)) return KAPPA_E_ARG;
        HIPCHK(hipMemcpyAsync(coarse->xadj, rb->l1.xadj, ((size_t)nc + 1) * sizeof(int64_t),
                              hipMemcpyDeviceToDevice, s));
        if (nc > 0)
            HIPCHK(hipMemcpyAsync(coarse->vw, rb->l1.vw, (size_t)nc * sizeof(uint32_t),
                                  hipMemcpyDeviceToDevice, s));
        if (nnzc > 0) {
            HIPCHK(hipMemcpyAsync(coarse->adj, rb->l1.adj, (size_t)nnzc * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(coarse->ew, rb->l1.ew, (size_t)nnzc * sizeof(uint32_t),
                                  hipMemcpyDeviceToDevice, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        return KAPPA_OK;
    }
    return KAPPA_E_NOMEM;
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
        info->grid_rounds = L.grid_rounds;
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

extern "C" int32_t kappa_hierarchy_rescan_stats(const kappa_hierarchy *h, int32_t l,
                                                int64_t *rows, int64_t *degsum, int32_t cap) {
    if (!h || l < 0 || l >= (int32_t)h->levels.size() || cap < 0) return KAPPA_E_ARG;
    const kappa_level &L = h->levels[l];
    int32_t k = std::min<int32_t>(cap, (int32_t)L.rescan.size());
    for (int32_t i = 0; i < k; ++i) {
        if (rows) rows[i] = L.rescan[i];
        if (degsum) degsum[i] = L.rescan_deg[i];
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
    uint32_t *flag = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) { flag = cv.get<uint32_t>(1); }))
        return KAPPA_E_NOMEM;
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
    UpAcc a;
    kappa_cut_result *rd = nullptr;
    int32_t *tr = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) {
            a.bw = cv.get<uint64_t>((int64_t)BW_SHARDS * k);
            a.acc = cv.get<uint64_t>(3 * NSHARD);
            a.arrive = cv.get<unsigned>(ARRIVE_WORDS);
            a.flag = cv.get<uint32_t>(1);
            rd = cv.get<kappa_cut_result>(1);
            tr = cv.get<int32_t>(tile_rows_needed(d.nnz));
        }))
        return KAPPA_E_NOMEM;
    launch_up_clear(a, k, s);
    launch_up_level(d, UP_GIVEN, nullptr, 0, nullptr, 0, const_cast<int32_t *>(part), k, eps_num,
                    eps_den, tr, a, block_w, rd, s);
    struct RB {
        kappa_cut_result r;
        uint32_t f;
    };
    RB *rb = (RB *)pinned(sizeof(RB));
    HIPCHK(hipMemcpyAsync(&rb->r, rd, sizeof(kappa_cut_result), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&rb->f, a.flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (rb->f) return KAPPA_E_RANGE;
    *out = rb->r;
    return KAPPA_OK;
}

// ---------------------------------------------------------------------------
// Cut and balance without allocation, for callers that cannot allocate (code
// under HIP graph capture, serving loops, harnesses that forbid it).  Its
// scratch (block-weight shards, accumulators, arrival counters, the result
// and the entry tiles' rows) lives in one file-scope device array per GPU,
// which every call on that GPU shares: calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr size_t NO_ALLOC_SCRATCH_BYTES = (size_t)2 << 20;
static __device__ __align__(256) unsigned char scratch[NO_ALLOC_SCRATCH_BYTES];

namespace {
constexpr int NO_ALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NO_ALLOC_MAX_DEVICES] = {};

// This GPU's scratch array by its device address (the array's name in host
// code is not one): looked up once per device, with that device current.
void *scratch_ptr() {
    int devid = 0;
    if (hipGetDevice(&devid) != hipSuccess || devid < 0 || devid >= NO_ALLOC_MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[devid]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[devid] = p;
    }
    return g_scratch_ptr[devid];
}

// The scratch layout of one cut/balance call (base == nullptr: sizes only).
struct CutScratch {
    UpAcc a;
    kappa_cut_result *rd = nullptr;
    int32_t *tr = nullptr;
    size_t bytes = 0;
    CutScratch(char *base, int32_t k, int64_t nnz) {
        Carve cv;
        cv.base = base;
        a.bw = cv.get<uint64_t>((int64_t)BW_SHARDS * k);
        a.acc = cv.get<uint64_t>(3 * NSHARD);
        a.arrive = cv.get<unsigned>(ARRIVE_WORDS);
        a.flag = cv.get<uint32_t>(1);
        rd = cv.get<kappa_cut_result>(1);
        tr = cv.get<int32_t>(tile_rows_needed(nnz));
        bytes = cv.off;
    }
};
struct NoAllocScope {
    NoAllocScope() { g_no_alloc_call = true; }
    ~NoAllocScope() { g_no_alloc_call = false; }
};
}  // namespace

extern "C" kappa_status kappa_cut_balance_noalloc(const kappa_graph *g, const int32_t *part,
                                                  int32_t k, uint32_t eps_num, uint32_t eps_den,
                                                  uint64_t *block_w, kappa_cut_result *out,
                                                  kappa_stream_t stream) {
    if (!graph_args_ok(g) || !out || !cut_args_ok(k, eps_num, eps_den)) return KAPPA_E_ARG;
    if (g->n > 0 && !part) return KAPPA_E_ARG;
    if (CutScratch(nullptr, k, g->nnz).bytes > NO_ALLOC_SCRATCH_BYTES) return KAPPA_E_CAPACITY;
    char *base = (char *)scratch_ptr();
    if (!base) return KAPPA_E_HIP;
    NoAllocScope scope;
    hipStream_t s = S(stream);
    const DevGraph d = dev(g);
    const CutScratch cs(base, k, d.nnz);
    launch_up_clear(cs.a, k, s);   // a fill kernel: the scratch keeps the last call's contents
    launch_up_level(d, UP_GIVEN, nullptr, 0, nullptr, 0, const_cast<int32_t *>(part), k, eps_num,
                    eps_den, cs.tr, cs.a, block_w, cs.rd, s);
    kappa_cut_result r;
    uint32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&r, cs.rd, sizeof r, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&flag, cs.a.flag, sizeof flag, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag) return KAPPA_E_RANGE;
    *out = r;
    return KAPPA_OK;
}

extern "C" kappa_status kappa_uncoarsen(const kappa_hierarchy *h, int32_t k, uint64_t part_seed,
                                        uint32_t eps_num, uint32_t eps_den, int32_t *part0,
                                        kappa_cut_result *results, kappa_stream_t stream) {
    if (!h || h->levels.empty() || !cut_args_ok(k, eps_num, eps_den)) return KAPPA_E_ARG;
    if (h->levels[0].n > 0 && !part0) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    const int32_t nl = (int32_t)h->levels.size();
    std::vector<int32_t *> part(nl, nullptr);
    kappa_cut_result *rd = nullptr;
    UpAcc a;
    int32_t *tr = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) {
            for (int32_t l = 1; l < nl; ++l) part[l] = cv.get<int32_t>(h->levels[l].n);
            rd = cv.get<kappa_cut_result>(nl);
            a.bw = cv.get<uint64_t>((int64_t)BW_SHARDS * k);
            a.acc = cv.get<uint64_t>(3 * NSHARD);
            a.arrive = cv.get<unsigned>(ARRIVE_WORDS);
            a.flag = cv.get<uint32_t>(1);
            tr = cv.get<int32_t>(tile_rows_needed(h->levels[0].nnz));
        }))
        return KAPPA_E_NOMEM;
    part[0] = part0;
    const int32_t L = nl - 1;
    std::vector<uint64_t> key = {2, pkey(w->base), (uint64_t)nl, (uint64_t)k, part_seed,
                                 (uint64_t)eps_num, (uint64_t)eps_den, pkey(part0)};
    for (const kappa_level &lv : h->levels) {
        key.push_back((uint64_t)lv.n);
        key.push_back((uint64_t)lv.nnz);
        key.push_back(pkey(lv.xadj));
        key.push_back(pkey(lv.adj));
        key.push_back(pkey(lv.ew));
        key.push_back(pkey(lv.vw));
        key.push_back(pkey(lv.cmap));
    }
    HIPCHK(run_seq(w->c, s, key, [&](hipStream_t q) {
        launch_up_clear(a, k, q);
        for (int32_t l = L; l >= 0; --l) {
            const kappa_level &lv = h->levels[l];
            DevGraph d;
            d.n = lv.n; d.nnz = lv.nnz; d.xadj = lv.xadj; d.adj = lv.adj; d.ew = lv.ew; d.vw = lv.vw;
            if (l == L)
                launch_up_level(d, UP_INITIAL, nullptr, 0, nullptr, part_seed, part[l], k, eps_num,
                                eps_den, tr, a, nullptr, rd + l, q);
            else
                launch_up_level(d, UP_PROJECT, lv.cmap, h->levels[l + 1].n, part[l + 1], 0, part[l],
                                k, eps_num, eps_den, tr, a, nullptr, rd + l, q);
        }
    }));
    uint32_t *hf = (uint32_t *)pinned(sizeof(kappa_cut_result) * nl + 8, PIN_RESULTS);
    if (!hf) return KAPPA_E_ARG;
    kappa_cut_result *hr = (kappa_cut_result *)((char *)hf + 8);
    HIPCHK(hipMemcpyAsync(hf, a.flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hr, rd, sizeof(kappa_cut_result) * nl, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*hf) return KAPPA_E_RANGE;
    if (results) std::memcpy(results, hr, sizeof(kappa_cut_result) * nl);
    return KAPPA_OK;
}

namespace {

bool refine_args_ok(int32_t k, uint32_t eps_num, uint32_t eps_den, const kappa_refine_params *p) {
    return p && k >= 1 && k <= REFINE_K_MAX && cut_args_ok(k, eps_num, eps_den) &&
           p->alpha_den >= 1 && p->depth >= 0 && p->max_local >= 1 && p->max_global >= 0 &&
           p->stop_after >= 1;
}

kappa_status refine_impl(const DevGraph &d, int32_t *part, int32_t k, uint32_t eps_num,
                         uint32_t eps_den, const kappa_refine_params *p, kappa_refine_stats *out,
                         hipStream_t s) {
    const int64_t n = d.n, maxp = std::max<int64_t>(1, (int64_t)k * (k - 1) / 2);
    RefineLaunch R{};
    unsigned long long *qbits = nullptr;
    int32_t *tmp_pair = nullptr, *tmp_col = nullptr;
    // the control block and the colour offsets, read back together
    struct Head {
        RefineCtl ctl;
        int32_t col_off[REFINE_COLOURS + 1];
    };
    Head *head = nullptr;
    std::unique_ptr<Workspace> w;
    if (!carve_workspace(s, w, [&](Carve &cv) {
            head = cv.get<Head>(1);
            R.bw = cv.get<int64_t>(k);
            R.bc = cv.get<int32_t>(k);
            qbits = cv.get<unsigned long long>((int64_t)k * REFINE_QW);
            tmp_pair = cv.get<int32_t>(maxp);
            tmp_col = cv.get<int32_t>(maxp);
            R.cpairs = cv.get<int32_t>(maxp);
            R.fill = cv.get<int32_t>(maxp);
            R.poff = cv.get<int32_t>(maxp);
            R.region = cv.get<int32_t>(n);
            R.dist = cv.get<int32_t>(n);
            R.gain = cv.get<int64_t>(2 * n);
            R.status = cv.get<uint8_t>(2 * n);
            R.qlist = cv.get<int32_t>(2 * n);
            R.mlog = cv.get<int32_t>(2 * n);
            R.slot = cv.get<int32_t>(2 * n);
        }))
        return KAPPA_E_NOMEM;
    R.xadj = d.xadj; R.adj = d.adj; R.ew = d.ew; R.vw = d.vw; R.part = part;
    R.n = d.n; R.k = k; R.eps_num = eps_num; R.eps_den = eps_den; R.seed = p->seed;
    R.alpha_num = p->alpha_num; R.alpha_den = p->alpha_den; R.depth = p->depth;
    R.max_local = p->max_local;
    // KAPPA_REFINE_QCAP (tests): fewer on-chip queue entries, to exercise the
    // entries kept in memory
    const char *qc = getenv("KAPPA_REFINE_QCAP");
    R.qcap = qc ? atoi(qc) : -1;
    R.ctl = &head->ctl;
    R.col_off = head->col_off;
    {
        ZeroRanges z;
        z.add((uint32_t *)head, sizeof(Head) / 4);
        z.add((uint32_t *)R.bw, 2 * (int64_t)k);
        z.add((uint32_t *)R.bc, k);
        launch_zero(z, s);
    }
    launch_refine_weights(part, d.vw, d.n, k, R.bw, R.bc, R.ctl, s);
    Head *rb = (Head *)pinned(sizeof(Head));
    if (!rb) return KAPPA_E_NOMEM;
    kappa_refine_stats st{};
    unsigned long long adopted = 0;
    int32_t idle = 0;
    bool pending = false;   // launched searches whose outcome has not been read
    for (int32_t gi = 0;; ++gi) {
        // the colouring of the next global iteration is launched before it is
        // known whether that iteration runs: one read-back per iteration
        if (gi < p->max_global) {
            ZeroRanges z;
            z.add((uint32_t *)qbits, (int64_t)k * REFINE_QW * 2);
            launch_zero(z, s);
            launch_refine_colouring(d.xadj, d.adj, part, d.n, k, qbits, tmp_pair, tmp_col,
                                    R.cpairs, R.col_off, R.fill, R.ctl, s);
        }
        HIPCHK(hipMemcpyAsync(rb, head, sizeof(Head), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (gi == 0 && (rb->ctl.flags & 1u)) return KAPPA_E_RANGE;
        if (rb->ctl.flags & 2u) {
            if (debug_on()) fprintf(stderr, "kappa: refine: block counts disagree with part\n");
            return KAPPA_E_HIP;
        }
        if (pending) {
            idle = rb->ctl.stats[4] > adopted ? 0 : idle + 1;
            adopted = rb->ctl.stats[4];
            pending = false;
            if (idle >= p->stop_after) break;
        }
        if (gi >= p->max_global) break;
        const int32_t ncol = rb->ctl.ncol;
        st.global_iterations += 1;
        st.colours += ncol;
        for (int32_t c = 0; c < ncol; ++c)
            if (rb->col_off[c + 1] > rb->col_off[c])
                launch_refine_colour(R, gi, c, rb->col_off[c + 1] - rb->col_off[c], s);
        HIPCHK(hipGetLastError());
        pending = true;
    }
    st.searches = (int64_t)rb->ctl.stats[1];
    st.moves = (int64_t)rb->ctl.stats[2];
    st.kept = (int64_t)rb->ctl.stats[3];
    st.adoptions = (int64_t)rb->ctl.stats[4];
    st.bytes = (int64_t)rb->ctl.stats[5];
    st.init_ticks = (int64_t)rb->ctl.stats[6];
    st.move_ticks = (int64_t)rb->ctl.stats[7];
    if (out) *out = st;
    return KAPPA_OK;
}

}  // namespace

extern "C" kappa_status kappa_refine(const kappa_graph *g, int32_t *part, int32_t k,
                                     uint32_t eps_num, uint32_t eps_den,
                                     const kappa_refine_params *params, kappa_refine_stats *stats,
                                     kappa_stream_t stream) {
    if (!graph_args_ok(g) || !refine_args_ok(k, eps_num, eps_den, params)) return KAPPA_E_ARG;
    if (g->n > 0 && !part) return KAPPA_E_ARG;
    return refine_impl(dev(g), part, k, eps_num, eps_den, params, stats, S(stream));
}

extern "C" kappa_status kappa_uncoarsen_refined(const kappa_hierarchy *h, int32_t k,
                                                uint64_t part_seed, uint32_t eps_num,
                                                uint32_t eps_den,
                                                const kappa_refine_params *params,
                                                int32_t *part0, kappa_cut_result *results,
                                                kappa_refine_stats *stats, kappa_stream_t stream) {
    if (!h || h->levels.empty() || !refine_args_ok(k, eps_num, eps_den, params))
        return KAPPA_E_ARG;
    if (h->levels[0].n > 0 && !part0) return KAPPA_E_ARG;
    hipStream_t s = S(stream);
    const int32_t nl = (int32_t)h->levels.size(), L = nl - 1;
    // the coarse levels' partitions in one arena (the workspace is taken by
    // the calls below)
    std::vector<size_t> off(nl, 0);
    size_t bytes = 256;
    for (int32_t l = 1; l < nl; ++l) {
        off[l] = bytes;
        bytes += ((size_t)std::max(1, h->levels[l].n) * sizeof(int32_t) + 255) & ~(size_t)255;
    }
    size_t got = 0;
    Allocator al;
    char *arena = (char *)take_arena(s, bytes, &got, &al);
    if (!arena) return KAPPA_E_NOMEM;
    struct Give {
        hipStream_t s; void *p; size_t b; Allocator al;
        ~Give() { give_arena(s, p, b, al); }
    } give{s, arena, got, al};
    std::vector<int32_t *> part(nl, nullptr);
    part[0] = part0;
    for (int32_t l = 1; l < nl; ++l) part[l] = (int32_t *)(arena + off[l]);
    for (int32_t l = L; l >= 0; --l) {
        const kappa_level &lv = h->levels[l];
        kappa_graph g{};
        g.n = lv.n; g.nnz = lv.nnz; g.xadj = lv.xadj; g.adj = lv.adj; g.ew = lv.ew; g.vw = lv.vw;
        kappa_status st;
        if (l == L)
            st = kappa_initial_partition(lv.n, k, part_seed, part[l], stream);
        else
            st = kappa_project(lv.cmap, lv.n, h->levels[l + 1].n, part[l + 1], part[l], stream);
        if (st != KAPPA_OK) return st;
        kappa_refine_params pl = *params;
        pl.seed = mix64(params->seed + (uint64_t)l);
        st = refine_impl(dev(&g), part[l], k, eps_num, eps_den, &pl, stats ? stats + l : nullptr,
                         s);
        if (st != KAPPA_OK) return st;
        if (results) {
            st = kappa_cut_balance(&g, part[l], k, eps_num, eps_den, nullptr, results + l, stream);
            if (st != KAPPA_OK) return st;
        }
    }
    return KAPPA_OK;
}

// ===========================================================================
// Served form: level-granular continuous batching.  The server holds the
// requests of one rating on one stream.  A step advances every active request
// by one level in one batched pass over the union of their current levels
// (each graph with the tie-break seed of its own depth); requests admitted
// since the last step join it at their level 0, and a request leaves as soon
// as a stop rule ends its hierarchy.  Each request's levels stay on the device
// in the step arenas that produced them, shared by the requests of a step.
// ===========================================================================
namespace {
// One block of a request's levels (or of a step's union), released when the
// last level carved from it is.  Taken from the allocator directly, not from
// the stream's arena cache: a cached arena may be far larger than asked for,
// and these blocks live as long as the requests holding them.
struct SrvMem {
    hipStream_t s = nullptr;
    void *p = nullptr;
    size_t bytes = 0;
    Allocator al;
    ~SrvMem() { dev_free(p, bytes, s, al); }
};
std::shared_ptr<SrvMem> srv_mem(hipStream_t s, size_t bytes) {
    auto m = std::make_shared<SrvMem>();
    m->s = s;
    m->al = current_allocator();
    m->bytes = std::max<size_t>(bytes, 256);
    m->p = dev_alloc(m->bytes, s, m->al, "served level");
    if (!m->p) return nullptr;
    return m;
}
struct SrvLevel {
    kappa_level lv;
    std::vector<std::shared_ptr<void>> holds;
};
struct SrvReq {
    int64_t id = 0;
    int32_t stop_n = 0;
    int32_t depth = 0;   // levels built below level 0
    std::vector<SrvLevel> levels;   // the last one is the current level
};
}  // namespace

struct kappa_server {
    hipStream_t s = nullptr;
    kappa_coarsen_params p{};
    std::vector<std::unique_ptr<SrvReq>> active, done;
    int64_t next_id = 0;
    uint32_t *interrupt = nullptr;       // host memory, coherent with the device
    const uint32_t *interrupt_dev = nullptr;
    ~kappa_server() {
        if (interrupt) (void)hipHostFree(interrupt);
    }
};

extern "C" kappa_status kappa_server_create(const kappa_coarsen_params *p, kappa_server **out,
                                            kappa_stream_t stream) {
    if (!out) return KAPPA_E_ARG;
    *out = nullptr;
    if (!params_ok(p, false)) return KAPPA_E_ARG;
    std::unique_ptr<kappa_server> v(new (std::nothrow) kappa_server());
    if (!v) return KAPPA_E_NOMEM;
    v->s = S(stream);
    v->p = *p;
    if (hipHostMalloc((void **)&v->interrupt, sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess)
        return KAPPA_E_NOMEM;
    __atomic_store_n(v->interrupt, 0u, __ATOMIC_RELEASE);
    void *dp = nullptr;
    HIPCHK(hipHostGetDevicePointer(&dp, v->interrupt, 0));
    v->interrupt_dev = (const uint32_t *)dp;
    *out = v.release();
    return KAPPA_OK;
}

extern "C" kappa_status kappa_server_interrupt(kappa_server *v, int32_t set) {
    if (!v) return KAPPA_E_ARG;
    __atomic_store_n(v->interrupt, set ? 1u : 0u, __ATOMIC_RELEASE);
    return KAPPA_OK;
}

extern "C" kappa_status kappa_server_admit(kappa_server *v, const kappa_graph *g, int32_t stop_n,
                                           int64_t *id) {
    if (!v || !id || !graph_args_ok(g)) return KAPPA_E_ARG;
    hipStream_t s = v->s;
    const DevGraph d = dev(g);
    int32_t maxdeg = 0;
    kappa_status st = validate_impl(d, s, &maxdeg, (v->p.flags & KAPPA_COARSEN_TRUSTED) != 0);
    if (st != KAPPA_OK) return st;
    // the request's level 0: a copy in the library's memory
    int64_t *xadj = nullptr;
    int32_t *adj = nullptr;
    uint32_t *ew = nullptr, *vw = nullptr;
    auto layout = [&](Carve &cv) {
        xadj = cv.get<int64_t>((int64_t)d.n + 1);
        adj = cv.get<int32_t>(d.nnz);
        ew = cv.get<uint32_t>(d.nnz);
        vw = cv.get<uint32_t>(d.n);
    };
    Carve lay;
    layout(lay);
    auto m = srv_mem(s, lay.off);
    if (!m) return KAPPA_E_NOMEM;
    Carve real;
    real.base = (char *)m->p;
    layout(real);
    HIPCHK(hipMemcpyAsync(xadj, d.xadj, 8 * ((size_t)d.n + 1), hipMemcpyDeviceToDevice, s));
    if (d.nnz > 0) {
        HIPCHK(hipMemcpyAsync(adj, d.adj, 4 * (size_t)d.nnz, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(ew, d.ew, 4 * (size_t)d.nnz, hipMemcpyDeviceToDevice, s));
    }
    if (d.n > 0) HIPCHK(hipMemcpyAsync(vw, d.vw, 4 * (size_t)d.n, hipMemcpyDeviceToDevice, s));
    std::unique_ptr<SrvReq> r(new (std::nothrow) SrvReq());
    if (!r) return KAPPA_E_NOMEM;
    r->id = v->next_id++;
    r->stop_n = stop_n;
    SrvLevel l0;
    l0.lv.n = d.n;
    l0.lv.nnz = d.nnz;
    l0.lv.maxdeg = maxdeg;
    l0.lv.xadj = xadj;
    l0.lv.adj = adj;
    l0.lv.ew = ew;
    l0.lv.vw = vw;
    l0.holds.push_back(m);
    r->levels.push_back(std::move(l0));
    *id = r->id;
    v->active.push_back(std::move(r));
    return KAPPA_OK;
}

extern "C" int32_t kappa_server_active(const kappa_server *v) {
    return v ? (int32_t)v->active.size() : 0;
}

namespace {
// Levels the geometric shrink of 0.6 per level (the usual one on meshes)
// needs to take n nodes to stop_n, plus one.
int levels_to_stop(int64_t n, int32_t stop_n) {
    const double r = std::max(1.0, (double)n / std::max(1, stop_n));
    return (int)std::ceil(std::log(r) / std::log(1.0 / 0.6)) + 1;
}

// One step of the server (arguments checked).  Finished request ids go to
// fin (host), at most cap of them are reported; *nfin gets how many finished.
kappa_status server_step(kappa_server *v, int64_t *fin, int32_t cap, int32_t *nfin) {
    hipStream_t s = v->s;
    int32_t nf = 0;
    auto finish = [&](std::unique_ptr<SrvReq> r) {
        if (nf < cap && fin) fin[nf] = r->id;
        ++nf;
        v->done.push_back(std::move(r));
    };
    // requests at the last level allowed stop there (the size rule first, as
    // at every level start; after a step it has been checked already)
    {
        std::vector<std::unique_ptr<SrvReq>> keep;
        for (auto &r : v->active) {
            if (r->depth >= v->p.max_levels) {
                kappa_level &cur = r->levels.back().lv;
                cur.stop = cur.n <= r->stop_n ? KAPPA_STOP_SIZE : KAPPA_STOP_MAXLEVEL;
                finish(std::move(r));
            } else {
                keep.push_back(std::move(r));
            }
        }
        v->active.swap(keep);
    }
    const int32_t count = (int32_t)v->active.size();
    *nfin = nf;
    if (count == 0) return KAPPA_OK;
    // the union of the current levels
    std::vector<int64_t> off(2 * ((size_t)count + 1), 0);
    int64_t *noff = off.data(), *eoff = off.data() + count + 1;
    std::vector<UnionSrc> src(count);
    std::vector<int32_t> stop(count), lmax(count);
    std::vector<uint64_t> gbase(count);
    int32_t maxdeg = 0, maxl = 1, first = 64;
    for (int32_t g = 0; g < count; ++g) {
        const SrvReq &r = *v->active[g];
        const kappa_level &cur = r.levels.back().lv;
        noff[g + 1] = noff[g] + cur.n;
        eoff[g + 1] = eoff[g] + cur.nnz;
        src[g] = UnionSrc{cur.xadj, cur.adj, cur.ew, cur.vw};
        stop[g] = r.stop_n;
        gbase[g] = v->p.seed + (uint64_t)r.depth;
        lmax[g] = v->p.max_levels - r.depth;
        maxl = std::max(maxl, lmax[g]);
        first = std::min(first, std::min(lmax[g], levels_to_stop(cur.n, r.stop_n)));
        maxdeg = std::max(maxdeg, cur.maxdeg);
    }
    const int64_t n = noff[count], nnz = eoff[count];
    if (n > INT32_MAX) return KAPPA_E_ARG;
    std::vector<int32_t> node_off(count + 1);
    for (int32_t g = 0; g <= count; ++g) node_off[g] = (int32_t)noff[g];
    int64_t *uxadj = nullptr;
    int32_t *uadj = nullptr;
    uint32_t *uew = nullptr, *uvw = nullptr;
    auto ulayout = [&](Carve &cv) {
        uxadj = cv.get<int64_t>(n + 1);
        uadj = cv.get<int32_t>(nnz);
        uew = cv.get<uint32_t>(nnz);
        uvw = cv.get<uint32_t>(n);
    };
    Carve ulay;
    ulayout(ulay);
    auto um = srv_mem(s, ulay.off);
    if (!um) return KAPPA_E_NOMEM;
    Carve ureal;
    ureal.base = (char *)um->p;
    ulayout(ureal);
    {
        UnionSrc *dsrc = nullptr;
        int64_t *doff = nullptr;
        std::unique_ptr<Workspace> w;
        if (!carve_workspace(s, w, [&](Carve &cv) {
                dsrc = cv.get<UnionSrc>(count);
                doff = cv.get<int64_t>(2 * ((int64_t)count + 1));
            }))
            return KAPPA_E_NOMEM;
        HIPCHK(hipMemcpyAsync(dsrc, src.data(), sizeof(UnionSrc) * count, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice,
                              s));
        launch_union_build(dsrc, count, doff, doff + count + 1, n, nnz, uxadj, uadj, uew, uvw, s);
        HIPCHK(hipGetLastError());
    }
    // levels of the batched form over the union, each graph with its own
    // depth's seeds and level cap, up to the first level boundary at which a
    // graph stops or the host interrupts the step
    kappa_coarsen_params pp = v->p;
    pp.max_levels = maxl;
    pp.flags |= KAPPA_COARSEN_TRUSTED;   // every request was validated when it was admitted
    BatchIn bi{count, node_off.data(), stop.data()};
    bi.gbase = gbase.data();
    bi.lmax = lmax.data();
    bi.interrupt = v->interrupt_dev;
    bi.interrupt_host = v->interrupt;
    bi.first_batch = std::max(1, std::min(first, 3));
    kappa_hierarchy UH;
    UH.s = s;
    BatchOut bo;
    const DevGraph d0{(int32_t)n, nnz, uxadj, uadj, uew, uvw};
    const uint64_t lvl0 = (uint64_t)n * 28 + (uint64_t)nnz * 8 + (uint64_t)(count + 1) * 8 + 8192;
    uint64_t arena = (maxdeg > BIN_MID_MAX ? 8 : 3) * lvl0 + (1u << 20);
    bool hubs = 2 * (int64_t)maxdeg - 2 > ROW_MID_MAX / 8;
    kappa_status st = KAPPA_OK;
    for (int attempt = 0; attempt < 6; ++attempt) {
        uint32_t retry = 0;
        st = coarsen_attempt(d0, maxdeg, &pp, s, &arena, false, hubs, &bi, &UH, &bo, &retry);
        if (debug_on())
            fprintf(stderr, "kappa: served step of %d requests (n %lld) attempt %d arena %llu: "
                    "status %d, retry flags 0x%x, levels %zu\n", count, (long long)n, attempt,
                    (unsigned long long)arena, (int)st, retry, UH.levels.size());
        if (st == KAPPA_OK || !retry) break;
        if (retry & CF_ARENA) arena *= 4;
        if (retry & CF_HUBS) hubs = true;
    }
    if (st != KAPPA_OK) return st;
    // every union level built, per graph with local ids, in one step block:
    // level j's row offsets, entries, node weights, the cmap of level j - 1,
    // and per graph its first entry and largest degree on level j
    const int J = (int)UH.levels.size() - 1;
    struct XL {
        int64_t *xadj = nullptr;
        int32_t *adj = nullptr, *cmap = nullptr, *noff = nullptr;
        uint32_t *ew = nullptr, *vw = nullptr;
    };
    std::vector<XL> xl(J + 1);
    int64_t *info = nullptr;   // per level j >= 1: eoff[count + 1], then dmax[count] as int32
    const int64_t info_words = (int64_t)count + 1 + ((int64_t)count + 1) / 2;
    std::shared_ptr<SrvMem> xm;
    std::vector<int64_t> hinfo;
    if (J >= 1) {
        auto xlayout = [&](Carve &cv) {
            for (int j = 1; j <= J; ++j) {
                const kappa_level &U = UH.levels[j], &P = UH.levels[j - 1];
                xl[j].xadj = cv.get<int64_t>((int64_t)U.n + count);
                xl[j].adj = cv.get<int32_t>(U.nnz);
                xl[j].ew = cv.get<uint32_t>(U.nnz);
                xl[j].vw = cv.get<uint32_t>(U.n);
                xl[j - 1].cmap = cv.get<int32_t>(P.n);
                xl[j].noff = cv.get<int32_t>((int64_t)count + 1);
            }
            info = cv.get<int64_t>(info_words * J);
        };
        Carve xlay;
        xlayout(xlay);
        xm = srv_mem(s, xlay.off);
        if (!xm) return KAPPA_E_NOMEM;
        Carve xreal;
        xreal.base = (char *)xm->p;
        xlayout(xreal);
        ZeroRanges z;
        z.add(info, (size_t)(2 * info_words * J));
        launch_zero(z, s);
        for (int j = 1; j <= J; ++j) {
            const kappa_level &U = UH.levels[j], &P = UH.levels[j - 1];
            HIPCHK(hipMemcpyAsync(xl[j].noff, bo.noff[j].data(), 4 * ((size_t)count + 1),
                                  hipMemcpyHostToDevice, s));
            DevGraph u{U.n, U.nnz, U.xadj, U.adj, U.ew, U.vw};
            u.gid = U.gid;
            int64_t *ij = info + info_words * (j - 1);
            launch_serve_extract(u, xl[j].noff, count, P.cmap, P.gid, P.n, xl[j].xadj, xl[j].adj,
                                 xl[j].ew, xl[j].vw, xl[j - 1].cmap, ij, (int32_t *)(ij + count + 1),
                                 s);
            HIPCHK(hipGetLastError());
        }
        hinfo.resize((size_t)info_words * J);
        HIPCHK(hipMemcpyAsync(hinfo.data(), info, 8 * hinfo.size(), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int32_t g = 0; g < count; ++g) {   // every graph ended the step somewhere
        const int32_t c = bo.coarsest[g], why = bo.reason[g];
        if (c < 0 || c > J || (c == 0 && why == KAPPA_STOP_NONE)) return KAPPA_E_HIP;
    }
    std::vector<std::unique_ptr<SrvReq>> keep;
    for (int32_t g = 0; g < count; ++g) {
        std::unique_ptr<SrvReq> r = std::move(v->active[g]);
        const int32_t c = bo.coarsest[g], why = bo.reason[g];
        for (int j = 1; j <= c; ++j) {
            const int32_t a = bo.noff[j][g], b = bo.noff[j][g + 1];
            const int64_t *ij = hinfo.data() + (size_t)info_words * (j - 1);
            const int32_t *dmax = (const int32_t *)(ij + count + 1);
            SrvLevel &cur = r->levels.back();
            cur.lv.cmap = xl[j - 1].cmap + bo.noff[j - 1][g];
            cur.lv.matched = (int64_t)cur.lv.n - (b - a);
            cur.holds.push_back(xm);
            SrvLevel nx;
            nx.lv.n = b - a;
            nx.lv.nnz = ij[g + 1] - ij[g];
            nx.lv.maxdeg = dmax[g];
            nx.lv.xadj = xl[j].xadj + a + g;
            nx.lv.adj = xl[j].adj + ij[g];
            nx.lv.ew = xl[j].ew + ij[g];
            nx.lv.vw = xl[j].vw + a;
            nx.holds.push_back(xm);
            r->levels.push_back(std::move(nx));
        }
        r->depth += c;
        if (why == KAPPA_STOP_NONE) {   // the step ended before its hierarchy did
            keep.push_back(std::move(r));
        } else {
            r->levels.back().lv.stop = why;
            finish(std::move(r));
        }
    }
    v->active.swap(keep);
    *nfin = nf;
    return KAPPA_OK;
}
}  // namespace

extern "C" kappa_status kappa_server_step(kappa_server *v, int64_t *finished, int32_t cap,
                                          int32_t *nfinished) {
    if (!v || !nfinished || cap < 0 || (cap > 0 && !finished)) return KAPPA_E_ARG;
    *nfinished = 0;
    return server_step(v, finished, cap, nfinished);
}

extern "C" kappa_status kappa_server_take(kappa_server *v, int64_t id, kappa_hierarchy **out) {
    if (!v || !out) return KAPPA_E_ARG;
    *out = nullptr;
    for (size_t i = 0; i < v->done.size(); ++i) {
        if (v->done[i]->id != id) continue;
        std::unique_ptr<SrvReq> r = std::move(v->done[i]);
        v->done.erase(v->done.begin() + (ptrdiff_t)i);
        kappa_hierarchy *H = new (std::nothrow) kappa_hierarchy();
        if (!H) return KAPPA_E_NOMEM;
        H->s = v->s;
        for (auto &l : r->levels) {
            H->levels.push_back(l.lv);
            for (auto &h : l.holds) H->holds.push_back(h);
        }
        *out = H;
        return KAPPA_OK;
    }
    return KAPPA_E_ARG;   // not finished, or already taken
}

extern "C" void kappa_server_free(kappa_server *v) { delete v; }

extern "C" kappa_status kappa_cache_release(void) {
    HIPCHK(hipDeviceSynchronize());
    std::lock_guard<std::mutex> g(g_cache_mu);
    for (StreamCache *c : g_caches) {
        std::lock_guard<std::mutex> a(c->mu), b(c->amu);
        for (GraphEntry &e : c->graphs)
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
        c->graphs.clear();
        c->seen.clear();
        // the device is idle: blocks go back without stream order (the stream
        // a cache belongs to may no longer exist)
        dev_free(c->ws, c->ws_bytes, nullptr, c->ws_al, true);
        c->ws = nullptr;
        c->ws_bytes = 0;
        for (const CachedArena &ca : c->arenas) dev_free(ca.p, ca.bytes, nullptr, ca.al, true);
        c->arenas.clear();
    }
    return KAPPA_OK;
}

extern "C" kappa_status kappa_set_allocator(kappa_alloc_fn alloc, kappa_free_fn dealloc,
                                            void *ctx) {
    if ((alloc == nullptr) != (dealloc == nullptr)) return KAPPA_E_ARG;
    const kappa_status st = kappa_cache_release();
    if (st != KAPPA_OK) return st;
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.dealloc = dealloc;
    g_alloc.ctx = ctx;
    return KAPPA_OK;
}

extern "C" void kappa_graphs_enable(int32_t on) { g_graphs_on = on != 0; }

extern "C" void kappa_arena_first(uint64_t bytes) { g_arena_first.store(bytes); }

extern "C" void kappa_tail_enable(int32_t on) { g_tail_on = on != 0; }
extern "C" void kappa_persistent_enable(int32_t on) { g_persistent_on = on != 0; }

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

extern "C" const char *kappa_version(void) { return "kappa-mi355x 0.2 (gfx950)"; }
