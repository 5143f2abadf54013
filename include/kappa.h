/*
 * kappa.h -- C ABI of the MI355X (gfx950) coarsening-hierarchy library.
 *
 * Implements the contraction phase of the multilevel graph partitioner of
 * "Engineering a Scalable High Quality Graph Partitioner" (Holtgrewe, Sanders,
 * Schulz), together with the projection and cut/balance evaluation used on the
 * way back up:
 *   edge rating (Section 3.1) -> locally-heaviest-edge matching (Section 3.3)
 *   -> contraction into a weighted coarse graph (Section 2) -> repeat until
 *   small (Section 2, stop rule of Section 4) -> projection of a partition
 *   (uncontraction, Section 2) -> cut and balance (Section 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graph.  G = (V, E, c, w) of Section 2 as a symmetric CSR in device memory:
 *   xadj[n+1] int64   row offsets, xadj[0] = 0, non-decreasing, xadj[n] = nnz
 *   adj[nnz]  int32   neighbour ids, each row strictly ascending, no self loop
 *   ew[nnz]   uint32  edge weight w({v,u}), equal in both directions, w >= 1
 *   vw[n]     uint32  node weight c(v) >= 0
 *   nnz = 2|E|.  Sum of w over E and sum of c over V must stay <= 2^32 - 1;
 *   contraction never increases either sum, so every level keeps the bound and
 *   every weight of every level fits uint32.  (The paper allows real weights;
 *   integers make every comparison exact.)  Callers holding int32 tensors pass
 *   their bits: they are read as uint32.
 * Pointers.  Every array argument is a DEVICE pointer unless its comment says
 *   host.  The caller owns every array it passes; the library never frees
 *   them.  Arrays of length 0 may be NULL.
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Work is
 *   enqueued on it.  Calls that return a result on the host (status of a
 *   validation, round counts, cut values) synchronise that stream before they
 *   return.
 * Errors.  Every entry point returns a kappa_status; no exception crosses the
 *   ABI.  On an error nothing is guaranteed about the output arrays.
 * Ratings.  Ratings are exact rationals num/den with num, den < 2^64; edge e
 *   ranks above edge f iff num_e*den_f > num_f*den_e (128-bit), else
 *   h(e) > h(f), else eid(e) < eid(f), where eid = (min(u,v) << 32) | max(u,v)
 *   and h(e) = mix64(seed ^ eid), mix64 being the SplitMix64 output function.
 *   A zero denominator is +infinity.  This strict order makes the matching
 *   unique: it equals the Greedy matching of Section 3.2 under the same order.
 */
#ifndef KAPPA_H
#define KAPPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *kappa_stream_t; /* a hipStream_t */

typedef enum {
    KAPPA_OK = 0,
    KAPPA_E_ARG = -1,      /* bad size, NULL pointer, unknown enum, k or eps out of range */
    KAPPA_E_GRAPH = -2,    /* CSR not symmetric / not simple / rows not ascending / bad offsets */
    KAPPA_E_RANGE = -3,    /* w = 0, sum of w or c above 2^32-1, block id or map entry out of range */
    KAPPA_E_NOMEM = -4,    /* device allocation failed */
    KAPPA_E_CAPACITY = -5, /* an output buffer is smaller than the result */
    KAPPA_E_HIP = -6       /* a HIP runtime call failed */
} kappa_status;

/* Section 3.1 ratings of an edge {u,v} with weight w. */
typedef enum {
    KAPPA_EXPANSION_STAR2 = 0, /* w^2 / (c(u) c(v))                 (paper's default) */
    KAPPA_INNER_OUTER = 1,     /* w / (Out(u) + Out(v) - 2w), Out(v) = sum of w at v */
    KAPPA_WEIGHT = 2,          /* w                                                   */
    KAPPA_EXPANSION = 3,       /* w / (c(u) + c(v))                                   */
    KAPPA_EXPANSION_STAR = 4   /* w / (c(u) c(v))                                     */
} kappa_rating;

/* Why the level loop ended (recorded on the coarsest level). */
typedef enum {
    KAPPA_STOP_NONE = 0,
    KAPPA_STOP_SIZE = 1,     /* n <= stop_n before matching                     */
    KAPPA_STOP_EMPTY = 2,    /* the matching of the last level was empty        */
    KAPPA_STOP_STALL = 3,    /* the last contraction removed < stall of nodes   */
    KAPPA_STOP_MAXLEVEL = 4  /* max_levels contractions done                    */
} kappa_stop;

typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t *xadj;
    const int32_t *adj;
    const uint32_t *ew;
    const uint32_t *vw;
} kappa_graph;

/* Caller-allocated output graph.  cap_n / cap_nnz are the capacities of the
   arrays (vw and xadj need cap_n and cap_n + 1 entries); n / nnz receive the
   sizes.  Capacities equal to the fine graph's n and nnz always suffice. */
typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t cap_n;
    int64_t cap_nnz;
    int64_t *xadj;
    int32_t *adj;
    uint32_t *ew;
    uint32_t *vw;
} kappa_graph_out;

typedef struct {
    int32_t rating;       /* kappa_rating */
    uint64_t seed;        /* level l matches with seed_l = mix64(seed + l) */
    int32_t stop_n;       /* stop once n <= stop_n */
    uint32_t stall_num;   /* stop after a level with (n_l - n_{l+1}) * stall_den */
    uint32_t stall_den;   /*   < stall_num * n_l; stall_num = 0 disables the rule */
    int32_t max_levels;   /* at most this many contractions (<= 256) */
    uint32_t flags;       /* 0, or KAPPA_COARSEN_TRUSTED and/or KAPPA_COARSEN_TWO_PHASE */
    int32_t block_bits;   /* KAPPA_COARSEN_TWO_PHASE: blocks of 2^block_bits ids, 0..11 */
} kappa_coarsen_params;

/* The caller has checked the graph with kappa_validate (and not changed it
   since): only the row offsets and the node-weight sum are checked again.
   A graph that would fail kappa_validate is undefined behaviour (kernels
   may read outside its arrays). */
#define KAPPA_COARSEN_TRUSTED 1u

/* Every level is matched by the two-phase matcher (kappa_match_two_phase)
   with blocks of 2^block_bits consecutive ids of that level, instead of the
   local-max rounds on the whole graph.  Single-graph form only
   (kappa_coarsen); the batched forms return KAPPA_E_ARG.  A level's
   `rounds` and round statistics then describe its gap rounds. */
#define KAPPA_COARSEN_TWO_PHASE 2u

/* Exact cut/balance of a k-way partition (Section 2; imbalance as in
   Section 5.2).  L_max = (1 + eps) c(V)/k + max_v c(v) = lmax_num / lmax_den
   with lmax_den = k * eps_den. */
typedef struct {
    uint64_t cut;        /* sum of w over edges whose ends lie in different blocks */
    uint64_t total;      /* c(V) */
    uint64_t max_block;  /* max_i c(V_i) */
    uint64_t max_node;   /* max_v c(v) on this graph */
    uint64_t lmax_num;
    uint64_t lmax_den;
    uint64_t imb_num;    /* max(0, max_block - L_max) * lmax_den */
    uint64_t bal_num;    /* balance = k * max_block / c(V) = bal_num / bal_den */
    uint64_t bal_den;
    int64_t feasible;    /* 1 iff max_block <= L_max */
} kappa_cut_result;

typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t rounds;      /* matching rounds spent on this level (0 on the coarsest) */
    int64_t matched;     /* |M| of this level's matching */
    int32_t stop_reason; /* kappa_stop; nonzero only on the coarsest level */
    int32_t grid_rounds; /* of those rounds, how many ran as grid-wide kernel launches (the
                            rest ran in one workgroup once few nodes were pending); 0 in a
                            hierarchy taken out of a batch */
} kappa_level_info;

typedef struct kappa_hierarchy kappa_hierarchy; /* opaque, library-owned */

/* Checks that g is a graph in the form above (Section 2: simple, undirected,
   w > 0, c >= 0) and that the weight sums fit.  Returns KAPPA_OK,
   KAPPA_E_ARG (sizes/NULL), KAPPA_E_GRAPH (structure) or KAPPA_E_RANGE
   (weights), checked in that priority.  Synchronous. */
kappa_status kappa_validate(const kappa_graph *g, kappa_stream_t stream);

/* Section 3.1: writes the rating of every CSR entry j (edge {v, adj[j]})
   as num[j] / den[j] (both uint64, nnz entries each).  g must be valid. */
kappa_status kappa_rate(const kappa_graph *g, int32_t rating, uint64_t *num, uint64_t *den,
                        kappa_stream_t stream);

/* Section 3.3: parallel locally-heaviest-edge matching.  In every round each
   free node with a free neighbour points at its best edge to a free
   neighbour; edges that are best at both ends are matched; rounds repeat
   until no edge can be added.  mate[n] (device, out): partner or -1.
   rounds_out, matched_out (host, may be NULL): round count and |M|.
   level_seed is the tie-break seed used in h(e) directly.  Synchronous. */
kappa_status kappa_match(const kappa_graph *g, int32_t rating, uint64_t level_seed,
                         int32_t *mate, int32_t *rounds_out, int64_t *matched_out,
                         kappa_stream_t stream);

/* Section 3.3, the two-phase scheme: a preliminary partition into blocks
   (here by the node numbering: block(v) = v >> block_bits, 0 <= block_bits
   <= 11, so that a locality order such as recursive coordinate bisection
   makes them geometric blocks); Greedy inside every block (one workgroup
   per block); then the gap graph -- edges between two blocks that are above
   the block edge matched at each of their ends -- matched by the parallel
   local-max rounds.  A gap edge replaces the block edges at its ends; a node
   whose block partner is taken that way stays unmatched.  mate[n] (device,
   out): the result; block_mate[n] (device, out, may be NULL): the block
   phase's matching; matched_out (host, may be NULL): |M|.  The order of
   edges, seeds and the rest as for kappa_match.  Returns KAPPA_E_ARG for
   block_bits outside [0, 11].  Synchronous. */
kappa_status kappa_match_two_phase(const kappa_graph *g, int32_t rating, uint64_t level_seed,
                                   int32_t block_bits, int32_t *mate, int32_t *block_mate,
                                   int64_t *matched_out, kappa_stream_t stream);

/* Section 3.3 (the preliminary partition from 2D coordinates): the recursive
   coordinate bisection order of n points.  xy (device, 2n doubles, x and y
   of point i at 2i and 2i+1).  Every box of more than `leaf` points (leaf >=
   1) is sorted stably by x at even depths and by y at odd depths, then cut
   after its first half (its first len/2 points, rounded down), the lower half
   first; a box of at most `leaf` points keeps its order.  order[n] (device,
   out): order[x] = the point at position x.  -0.0 sorts as +0.0.  Returns
   KAPPA_E_ARG for n < 0, leaf < 1 or a missing array.  Synchronous. */
kappa_status kappa_rcb_order(const double *xy, int32_t n, int32_t leaf, int32_t *order,
                             kappa_stream_t stream);

/* Renumbers g by an order of its nodes (for instance kappa_rcb_order's):
   node x of `out` is node order[x] of g, with its node weight, its edges
   renamed through the inverse and its row sorted again.  out (host struct,
   device arrays, caller-owned, capacities cap_n >= n and cap_nnz >= nnz)
   receives n, nnz, xadj, adj, ew and vw.  Returns KAPPA_E_ARG if order is not
   a permutation of 0..n-1 (nothing else is written then) or nnz > 2^31 - 1,
   KAPPA_E_CAPACITY if out is too small.  g must be valid.  Synchronous. */
kappa_status kappa_relabel(const kappa_graph *g, const int32_t *order, kappa_graph_out *out,
                           kappa_stream_t stream);

/* Section 2: contracts the matching `mate` (as written by kappa_match, or any
   valid matching of g).  Coarse ids: a node is a representative if it is
   unmatched or the smaller end of its matched edge; representatives are
   numbered in ascending fine id.  cmap[n] (device, out): coarse id of each
   fine node.  coarse (host struct, device arrays): the coarse graph, rows
   ascending, parallel edges merged with summed weight.  Returns
   KAPPA_E_CAPACITY if coarse's capacities are too small.  Synchronous. */
kappa_status kappa_contract(const kappa_graph *g, const int32_t *mate, int32_t *cmap,
                            kappa_graph_out *coarse, kappa_stream_t stream);

/* The whole contraction phase: validate g, then match and contract level
   after level (level l uses seed_l = mix64(seed + l)) until a stop rule
   fires.  *out receives a library-owned hierarchy; level 0 refers to the
   caller's arrays of g, which must stay alive and unchanged while the
   hierarchy is used.  Synchronous. */
kappa_status kappa_coarsen(const kappa_graph *g, const kappa_coarsen_params *params,
                           kappa_hierarchy **out, kappa_stream_t stream);

int32_t kappa_hierarchy_levels(const kappa_hierarchy *h);

/* Level l of h (0 = input): its graph (device arrays owned by h), its fine ->
   coarse map (NULL on the coarsest level) and its statistics.  Any output
   pointer may be NULL. */
kappa_status kappa_hierarchy_level(const kappa_hierarchy *h, int32_t l, kappa_graph *g,
                                   const int32_t **cmap, kappa_level_info *info);

/* Round statistics of level l's matching (Section 3.3 rounds): for round r
   (0-based), pointing[r] = number of free nodes that had a free neighbour and
   degsum[r] = the sum of their degrees.  Copies min(rounds, cap) entries to
   the host arrays and returns the level's round count (at most 64 rounds are
   kept per level; a negative kappa_status on a bad argument). */
int32_t kappa_hierarchy_round_stats(const kappa_hierarchy *h, int32_t l, int64_t *pointing,
                                    int64_t *degsum, int32_t cap);

/* Rescan statistics of level l's matching, for the same rounds: rows[r] =
   the nodes whose row the pick scanned again in round r (0-based) and
   degsum[r] = the sum of their degrees.  Without chunked rows every pending
   node of a later round is scanned again; where long rows are scanned in
   chunks (a power-law graph), a pending node whose choice is still free
   keeps it and is not counted, and only the rounds run as grid launches are
   counted.  Either way the nodes counted pointed in the round before.  Index
   0 (the first round, which scans every row) holds zeros.  Recorded only
   while the per-launch profiler is on (kappa_profile_enable) when the
   hierarchy is built, since gathering them costs time; zeros otherwise.
   Copies min(rounds, cap) entries and returns the round count, as
   kappa_hierarchy_round_stats. */
int32_t kappa_hierarchy_rescan_stats(const kappa_hierarchy *h, int32_t l, int64_t *rows,
                                     int64_t *degsum, int32_t cap);

/* Frees h (stream-ordered on the stream it was built on). NULL is a no-op. */
void kappa_hierarchy_free(kappa_hierarchy *h);

/* Batched form.  `count` independent graphs laid out as ONE block-diagonal
   CSR `u` (device arrays, global ids): graph g owns nodes
   [node_off[g], node_off[g+1]) and only edges among them.  node_off (host,
   count + 1 entries, node_off[0] = 0, non-decreasing, node_off[count] =
   u->n) and stop_n (host, count entries, or NULL for p->stop_n everywhere)
   stay with the caller.  All graphs are coarsened together, level by level,
   every kernel launch covering every graph still coarsening; each graph's
   hierarchy equals what kappa_coarsen gives for that graph alone with the
   same parameters (tie hashes use graph-local ids; the size, empty-matching
   and stall rules and max_levels apply per graph).  Returns KAPPA_E_GRAPH if
   an edge joins two graphs, else as kappa_coarsen; the 32-bit limits of
   kappa_validate on the total edge weight and the total node weight apply to
   the union as a whole (a caller batches graphs whose sums fit).
   Synchronous; the batch is library-owned (kappa_batch_free). */
typedef struct kappa_batch kappa_batch;
kappa_status kappa_coarsen_batch(const kappa_graph *u, int32_t count, const int32_t *node_off,
                                 const int32_t *stop_n, const kappa_coarsen_params *p,
                                 kappa_batch **out, kappa_stream_t stream);
/* The batched form over separate graphs: graphs[0 .. count) (host array of
   descriptors of device graphs, each valid as for kappa_coarsen) are laid out
   as one block-diagonal union on the device by the library (graph g's nodes
   follow those of graphs 0 .. g-1), which it owns with the batch; then as
   kappa_coarsen_batch.  The input graphs need to stay alive only during the
   call.  KAPPA_E_ARG if the union would exceed 2^31 - 1 nodes. */
kappa_status kappa_coarsen_graphs(const kappa_graph *graphs, int32_t count, const int32_t *stop_n,
                                  const kappa_coarsen_params *p, kappa_batch **out,
                                  kappa_stream_t stream);

int32_t kappa_batch_count(const kappa_batch *b);
/* levels (host, may be NULL): graph g's level count; stop_reason: its kappa_stop. */
kappa_status kappa_batch_graph_info(const kappa_batch *b, int32_t g, int32_t *levels,
                                    int32_t *stop_reason);
/* Graph g's hierarchy as a standalone, library-owned kappa_hierarchy (ids
   local to g; level info has rounds = 0, since rounds are shared by the
   batch), for every hierarchy call (kappa_hierarchy_level,
   kappa_uncoarsen, ...).  Free it with kappa_hierarchy_free.  Synchronous. */
kappa_status kappa_batch_hierarchy(const kappa_batch *b, int32_t g, kappa_hierarchy **out,
                                   kappa_stream_t stream);
void kappa_batch_free(kappa_batch *b);

/* Served form: level-granular continuous batching of coarsening requests.
   A server holds the requests of one rating (p->rating, seed, stall rule and
   max_levels apply to every request; p->stop_n is unused) on one stream.
   kappa_server_step advances every active request in one batched pass over
   the union of their current levels (the work of the batched form; each
   graph with the tie-break seeds mix64(seed + level) of its own levels, so
   that its hierarchy is the one kappa_coarsen gives it alone).  A step runs
   level after level on the device and ends at the first level boundary at
   which some request's hierarchy has ended (by a stop rule of Section 2 / 4)
   or kappa_server_interrupt has been raised: requests join and leave the
   active set at level boundaries, between steps.  Requests admitted since
   the last step join it at their level 0.  Each request's levels stay on the
   device (library memory) until its hierarchy is taken and freed.  All calls
   but kappa_server_interrupt are synchronous on the server's stream and must
   come from one thread at a time. */
typedef struct kappa_server kappa_server;
kappa_status kappa_server_create(const kappa_coarsen_params *p, kappa_server **out,
                                 kappa_stream_t stream);
/* Validates g (as kappa_validate, unless p->flags has KAPPA_COARSEN_TRUSTED),
   copies it into library memory (the caller may free g afterwards) and adds
   it to the active set with its own stop size; *id (host) names it. */
kappa_status kappa_server_admit(kappa_server *v, const kappa_graph *g, int32_t stop_n,
                                int64_t *id);
int32_t kappa_server_active(const kappa_server *v);
/* set != 0: the running step (or the next one) ends at its next level
   boundary, e.g. because a request waits to be admitted; set = 0 clears the
   request.  The flag stays as set until changed.  May be called from any
   thread, also while a step runs. */
kappa_status kappa_server_interrupt(kappa_server *v, int32_t set);
/* One step for every active request (at least one level each, unless it
   stops before its first).  finished (host, cap entries, may be NULL when cap
   is 0) receives the ids of the requests whose hierarchy ended in this step;
   *nfinished (host) their count (ids beyond cap are not listed but are
   finished all the same). */
kappa_status kappa_server_step(kappa_server *v, int64_t *finished, int32_t cap,
                               int32_t *nfinished);
/* The hierarchy of finished request id, as a library-owned kappa_hierarchy
   (for kappa_hierarchy_level, kappa_uncoarsen, ...; per-level round counts
   are 0: rounds are shared by a step).  KAPPA_E_ARG if id has not finished or
   was taken already. */
kappa_status kappa_server_take(kappa_server *v, int64_t id, kappa_hierarchy **out);
void kappa_server_free(kappa_server *v);

/* Stand-in for the initial partitioning of Section 4 (which runs external
   partitioners): part[x] = mix64(seed + x) mod k for x < n.  k in [1, 4096]. */
kappa_status kappa_initial_partition(int32_t n, int32_t k, uint64_t seed, int32_t *part,
                                     kappa_stream_t stream);

/* Uncontraction as projection (Section 2): part_fine[v] =
   part_coarse[cmap[v]] for v < n_fine.  Every cmap entry must lie in
   [0, n_coarse), else KAPPA_E_RANGE.  Synchronous. */
kappa_status kappa_project(const int32_t *cmap, int32_t n_fine, int32_t n_coarse,
                           const int32_t *part_coarse, int32_t *part_fine,
                           kappa_stream_t stream);

/* Cut and balance of the k-way partition part[n] of g (Section 2).
   k in [1, 4096]; eps = eps_num / eps_den with eps_den in [1, 10^6] and
   eps_num <= 16 * 10^6.  block_w (device, k entries, out, may be NULL):
   c(V_i).  out (host): the exact results.  KAPPA_E_RANGE if a block id is
   outside [0, k).  Synchronous. */
kappa_status kappa_cut_balance(const kappa_graph *g, const int32_t *part, int32_t k,
                               uint32_t eps_num, uint32_t eps_den, uint64_t *block_w,
                               kappa_cut_result *out, kappa_stream_t stream);

/* Allocation-free variant of kappa_cut_balance, for callers that cannot
   allocate (code under HIP graph capture, tight serving loops, harnesses that
   forbid allocation): the same arguments, results and errors, but no device
   or pinned host allocation of any kind.  Its scratch is one file-scope
   device array of 2 MiB per GPU, held until the process ends: the block-weight
   shards (64 * k bytes), small accumulators and one int32 per 2048 CSR entries
   (the entry tiles' first rows).  A graph whose scratch would not fit (about
   8.8 * 10^8 entries and more) is rejected with KAPPA_E_CAPACITY before any
   device work.  Every call on a GPU shares that GPU's array (it keeps the last
   call's contents and is cleared by each call with a fill kernel, not a
   memset), so calls that overlap on one GPU race: serialise them.  out
   (host) is written through a stream-ordered copy.  Synchronous. */
kappa_status kappa_cut_balance_noalloc(const kappa_graph *g, const int32_t *part, int32_t k,
                                       uint32_t eps_num, uint32_t eps_den, uint64_t *block_w,
                                       kappa_cut_result *out, kappa_stream_t stream);

/* The way back up in one call: partitions the coarsest level of h with
   kappa_initial_partition(part_seed), projects level by level down to
   level 0 and evaluates cut/balance on every level.  part0 (device, n_0
   entries, out): the level-0 partition.  results (host, one entry per level,
   may be NULL): results[l] for level l.  Synchronous. */
kappa_status kappa_uncoarsen(const kappa_hierarchy *h, int32_t k, uint64_t part_seed,
                             uint32_t eps_num, uint32_t eps_den, int32_t *part0,
                             kappa_cut_result *results, kappa_stream_t stream);

/* Parameters of the pairwise refinement (Section 5; Table 2 names the
   presets minimal / fast / strong). */
typedef struct {
    uint64_t seed;        /* tie-break seed of the local searches */
    uint32_t alpha_num;   /* FM patience alpha = alpha_num / alpha_den (>= 1): a search */
    uint32_t alpha_den;   /*   stops after more than alpha * min(|A|, |B|) moves without gain */
    int32_t depth;        /* BFS search depth (>= 0) around the boundary of each block */
    int32_t max_local;    /* local iterations per pair (>= 1) */
    int32_t max_global;   /* max. global iterations (>= 0) */
    int32_t stop_after;   /* global iterations in a row without change that end it (>= 1) */
} kappa_refine_params;

typedef struct {
    int64_t global_iterations; /* global iterations run */
    int64_t searches;          /* two-block local searches run (two per local iteration) */
    int64_t moves;             /* node moves made by them */
    int64_t kept;              /* moves kept after the rollbacks of adopted searches */
    int64_t adoptions;         /* local iterations whose better search improved the pair */
    int64_t colours;           /* colours of Q summed over the global iterations */
    int64_t bytes;             /* memory the local searches touch, by a fixed model (for
                                  measurement): per search 40 B per node of the two blocks
                                  + 12 B per entry of their rows; per move 17 B per queued
                                  node scanned + 25 B per entry of the moved node's row;
                                  12 B per kept move of an adopted search */
    int64_t init_ticks;        /* device wall-clock ticks (100 MHz) that the pair workgroups spent
                                  preparing searches (gains, boundary, BFS), summed over them */
    int64_t move_ticks;        /* the same for the moves, rollbacks and adoptions */
} kappa_refine_stats;

/* Pairwise refinement of the k-way partition part (Section 5), in place.
   Each global iteration colours the quotient graph Q greedily (Section 5.1:
   Q's edges in ascending (a, b) order, each taking the smallest colour free
   at both ends) and walks the colours in order; the pairs of one colour run
   side by side.  A pair runs local iterations: two two-block FM searches
   (Section 5.2) with the run seeds
     mix64(mix64(mix64(seed + g) ^ ((a << 32) | b)) + 2 t + r),  r = 0, 1,
   for global iteration g and local iteration t; each queue orders nodes by
   gain (w to the other block - w to the own block, neighbours of the two
   blocks only), then by mix64(run seed ^ v), then by the smaller id; queues
   start with the boundary nodes and admit nodes within `depth` same-block
   hops of it; TopGain picks the queue with the larger top, except that the
   heavier block gives when a block is overloaded (c > L_max) and the two
   weights differ; the search stops when both queues are empty or after
   more than alpha * min(|A|, |B|) moves without improvement, and rolls back
   to the first state with the smallest (imbalance, cut), imbalance =
   max(0, c(A) - L_max, c(B) - L_max).  The better search (r = 0 on a tie)
   is adopted if it improves on the start; otherwise the pair is done.
   Global iterations stop after stop_after in a row without an adoption or
   after max_global.  k in [1, 256]; eps as in kappa_cut_balance.  part
   (device, n entries, in/out); stats (host, may be NULL).
   KAPPA_E_RANGE (part unchanged) if a block id lies outside [0, k).
   Synchronous. */
kappa_status kappa_refine(const kappa_graph *g, int32_t *part, int32_t k, uint32_t eps_num,
                          uint32_t eps_den, const kappa_refine_params *params,
                          kappa_refine_stats *stats, kappa_stream_t stream);

/* The way back up with refinement: the coarsest level of h is partitioned
   by kappa_initial_partition(part_seed); then from the coarsest level down,
   each level is projected from the one above (not the coarsest), refined
   by kappa_refine with the seed mix64(params->seed + l), and evaluated.
   part0 (device, n_0 entries, out): the level-0 partition.  results and
   stats (host, one entry per level, may be NULL).  Synchronous. */
kappa_status kappa_uncoarsen_refined(const kappa_hierarchy *h, int32_t k, uint64_t part_seed,
                                     uint32_t eps_num, uint32_t eps_den,
                                     const kappa_refine_params *params, int32_t *part0,
                                     kappa_cut_result *results, kappa_refine_stats *stats,
                                     kappa_stream_t stream);

/* Per-kernel timing with HIP events on the launch stream.  While enabled,
   every kernel launch of the library is bracketed by two events; read the
   totals with kappa_profile_read.  Not thread-safe. */
void kappa_profile_enable(int32_t on);
void kappa_profile_reset(void);
/* Copies up to `cap` entries: name (host, static strings), launches and
   summed milliseconds per kernel.  Returns the number of kernels recorded.
   Synchronises the device. */
int32_t kappa_profile_read(const char **names, int64_t *launches, double *ms, int32_t cap);

/* Device allocator for all memory the library allocates (workspaces,
   hierarchy arenas, batch unions).  alloc(bytes, stream, ctx) returns a
   device pointer usable in stream order on `stream` (NULL: out of memory);
   dealloc(ptr, bytes, stream, ctx) returns it once the work enqueued on
   `stream` before the call no longer needs it (stream NULL: the device is
   idle).  Both NULL restores the default, the device's stream-ordered pool
   (hipMallocAsync / hipFreeAsync).  The call first releases the memory cache
   (as kappa_cache_release: no call may be running); hierarchies and batches
   that are still alive return their memory to the allocator they came from.
   KAPPA_E_ARG if exactly one of alloc and dealloc is NULL. */
typedef void *(*kappa_alloc_fn)(size_t bytes, kappa_stream_t stream, void *ctx);
typedef void (*kappa_free_fn)(void *ptr, size_t bytes, kappa_stream_t stream, void *ctx);
kappa_status kappa_set_allocator(kappa_alloc_fn alloc, kappa_free_fn dealloc, void *ctx);

/* Device memory kept between calls: per stream, one workspace for call-local
   buffers (grown on demand, reused by the next call on that stream) and up
   to four arenas of freed hierarchies (reused by kappa_coarsen on that
   stream).  kappa_cache_release synchronises the device and frees all of it;
   no call may be running on any stream.  Later calls allocate again. */
kappa_status kappa_cache_release(void);

/* on = 1: launch sequences that repeat with the same sizes and buffers (a
   batch of levels of kappa_coarsen, the whole of kappa_uncoarsen) are
   captured as HIP graphs on their second occurrence and replayed from then
   on, on a side stream of the caller's stream ordered by events both ways.
   on = 0 (the default, measured faster on gfx950) launches every kernel
   directly.  Results do not depend on it. */
void kappa_graphs_enable(int32_t on);

/* Arena size of the first attempt of kappa_coarsen and kappa_coarsen_batch,
   in bytes, for every later call in the process (0, the default: sized from
   level 0, about three times its arrays).  When nonzero, the levels of the
   first attempt must fit in exactly that many bytes (raised to what level 0
   itself needs); a call whose levels do not fit starts again with four times
   the arena, up to five times.  Results do not depend on it: it exists to
   exercise the arena-overflow path at chosen levels. */
void kappa_arena_first(uint64_t bytes);

/* on = 1: in kappa_coarsen, once a level has at most 16384 nodes and
   131072 entries, that level and every later one run in a single workgroup
   in one launch instead of a sequence of grid-wide launches per level.
   on = 0 (the default, measured faster on gfx950: one workgroup cannot hide
   the latency of a level's dependent loads) runs every level with the grid
   kernels.  Results do not depend on it. */
void kappa_tail_enable(int32_t on);

/* on = 1: the matching rounds after the first of a level run in one
   cooperative launch (every workgroup resident; the pick and mate phases of
   a round separated by grid-wide barriers whose waits are bounded, so a
   broken state fails the call with KAPPA_E_HIP rather than hang), on levels
   whose long rows are not scanned in chunks; the others, and every level
   when the device cannot launch it, keep one launch per phase and round.
   on = 0 (the default, measured faster: 8.7 against 21.2 ms per step on the
   random geometric graph of 2^20 nodes, 86.9 against 99.3 ms on the batch of
   4096 graphs) launches every round's kernels.  Results do not depend on it.
   A cooperative launch needs the device to itself: with kernels of other
   streams running beside it, some of its workgroups may not be resident,
   its barrier waits time out and the call fails with KAPPA_E_HIP.  HIP-graph
   replay is not used while it is on. */
void kappa_persistent_enable(int32_t on);

/* Tunable thresholds of the level kernels.  None changes a result (every
   hierarchy and partition is the same under any valid table); they move
   work between kernels.  Valid ranges in brackets; the compiled defaults in
   parentheses.  At load the library reads the table at $KAPPA_TUNING (a
   path; "none" keeps the defaults) or else kappa_tuning.txt beside the
   library, if present (paper_0910_2004_amd/autotune.py measures and writes
   it).  A table applies to calls started after it is set; setting it while
   calls run on other threads is allowed but those calls may use either. */
typedef struct {
    int32_t bin_small_max;      /* matching: rows of at most this many entries take the 4-lane
                                   path, longer ones a wave [1, 16] (16) */
    int32_t tail_max;           /* matching: a level goes to the one-workgroup finisher once at
                                   most this many nodes still point somewhere [0, 4096] (128) */
    int32_t finish_max;         /* the finisher takes a level whose grid rounds ran out only with
                                   at most this many nodes pending [0, 2^20] (4096) */
    int32_t finish_max_big;     /*   and at most this many of them with rows above 1024
                                   entries [0, 2^16] (64); else the level gets more grid rounds */
    int32_t row_small_max;      /* contraction: coarse rows whose entry bound is at most this
                                   are merged by 16 lanes, longer ones by a wave [2, 64] (64) */
    int32_t scan_one_block_max; /* prefix sums of at most this many items run in one
                                   workgroup, longer ones in two grid launches [0, 2^22] (16384) */
    int32_t rounds_base;        /* grid matching rounds launched per level: rounds_base for a
                                   level of at most rounds_n0 nodes [1, 16] (3), */
    int32_t rounds_n0;          /*   [1, 2^24] (2048), */
    int32_t rounds_growth;      /*   one more per factor rounds_growth in nodes [2, 1024] (8), */
    int32_t rounds_cap;         /*   at most rounds_cap [rounds_base, 32] (8) */
} kappa_tuning;
/* The current table (host). */
kappa_status kappa_tuning_get(kappa_tuning *out);
/* Replaces the table; KAPPA_E_RANGE (table unchanged) if a field is out of
   range. */
kappa_status kappa_tuning_set(const kappa_tuning *t);
/* Reads "name value" lines (names as the fields above, '#' starts a comment;
   fields not named keep their current values) from path and sets the table:
   KAPPA_E_ARG if the file cannot be read or holds an unknown name or a
   malformed line, KAPPA_E_RANGE if a value is out of range (table
   unchanged in both cases). */
kappa_status kappa_tuning_load(const char *path);

const char *kappa_status_str(kappa_status st);
const char *kappa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KAPPA_H */
