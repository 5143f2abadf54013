/*
 * kappa_oracle.c -- sequential CPU oracle for the coarsening hierarchy of the
 * multilevel partitioner in "Engineering a Scalable High Quality Graph
 * Partitioner" (Holtgrewe, Sanders, Schulz), and for the pairwise refinement
 * of its uncoarsening phase (Section 5).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this file; only the test suite, the smoke check and the CPU baseline of
 * the benchmark load it.  It is plain, single-threaded C99 (plus the compiler's
 * unsigned __int128), written for a reader who checks it against the paper by
 * eye, not for speed.
 *
 * Conventions (readings of the paper, shared with the GPU library only through
 * the paper and the design notes, never through code):
 *   - G = (V, E, c, w) as in Section 2 ("Preliminaries"), stored as a symmetric
 *     CSR: xadj[n+1] (int64), adj[nnz] (int32), ew[nnz] (uint32 = w),
 *     vw[n] (uint32 = c).  nnz = 2|E|.
 *   - weights are integers: w >= 1, c >= 0, sum w(E) <= 2^32-1 and
 *     sum c(V) <= 2^32-1 (Section 2 allows reals; integers make every
 *     comparison exact).
 *   - a rating is an exact rational num/den with num, den < 2^64; ratings are
 *     compared by 128-bit cross products (Section 3.1 defines the ratings).
 *   - the strict order on edges: e > f iff num_e*den_f > num_f*den_e, else
 *     h(e) > h(f), else eid(e) < eid(f), with eid = (min << 32) | max and
 *     h(e) = mix64(seed ^ eid).  The paper leaves ties open; this order makes
 *     the matching unique.
 *   - mix64 is the output function ("finaliser") of SplitMix64 (Steele, Lea,
 *     Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Status codes.  Same numbers as the library's, fixed by the design notes. */
#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_GRAPH (-2)
#define ORC_E_RANGE (-3)

/* Rating selector (Section 3.1). */
#define ORC_EXPANSION_STAR2 0
#define ORC_INNER_OUTER 1
#define ORC_WEIGHT 2
#define ORC_EXPANSION 3
#define ORC_EXPANSION_STAR 4

/* ------------------------------------------------------------------------ */
/* SplitMix64 output function, from its published definition.              */
/* ------------------------------------------------------------------------ */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* SplitMix64 stream: state += golden gamma, then the output function. */
uint64_t orc_splitmix64_next(uint64_t *state)
{
    *state += 0x9e3779b97f4a7c15ULL;
    return orc_mix64(*state);
}

/* ------------------------------------------------------------------------ */
/* Validation: the input must be the graph of Section 2 in CSR form.        */
/* Checks are grouped in three classes with a fixed priority:               */
/*   ARG   (sizes / pointers) > GRAPH (structure) > RANGE (weights).        */
/* ------------------------------------------------------------------------ */
static int row_contains(const int64_t *xadj, const int32_t *adj, const uint32_t *ew,
                        int32_t row, int32_t target, uint32_t *w_out)
{
    for (int64_t j = xadj[row]; j < xadj[row + 1]; ++j)
        if (adj[j] == target) { *w_out = ew[j]; return 1; }
    return 0;
}

int orc_validate(int32_t n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                 const uint32_t *ew, const uint32_t *vw)
{
    if (n < 0 || nnz < 0) return ORC_E_ARG;
    if (xadj == NULL) return ORC_E_ARG;
    if (n > 0 && vw == NULL) return ORC_E_ARG;
    if (nnz > 0 && (adj == NULL || ew == NULL)) return ORC_E_ARG;

    /* structure: offsets */
    if (xadj[0] != 0 || xadj[n] != nnz) return ORC_E_GRAPH;
    for (int32_t v = 0; v < n; ++v)
        if (xadj[v + 1] < xadj[v]) return ORC_E_GRAPH;
    /* structure: targets in range, no self loop, rows strictly ascending
       (no parallel edges: the graph is simple), and symmetric with equal
       weights (the graph is undirected). */
    for (int32_t v = 0; v < n; ++v) {
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t u = adj[j];
            if (u < 0 || u >= n || u == v) return ORC_E_GRAPH;
            if (j > xadj[v] && adj[j - 1] >= u) return ORC_E_GRAPH;
        }
    }
    for (int32_t v = 0; v < n; ++v) {
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            uint32_t back;
            if (!row_contains(xadj, adj, ew, adj[j], v, &back)) return ORC_E_GRAPH;
            if (back != ew[j]) return ORC_E_GRAPH;
        }
    }
    /* range: w >= 1 (Section 2 asks w > 0), sums below 2^32 */
    uint64_t sw = 0, sc = 0;
    for (int32_t v = 0; v < n; ++v) {
        sc += vw[v];
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            if (ew[j] == 0) return ORC_E_RANGE;
            if (adj[j] > v) sw += ew[j];
        }
    }
    if (sw > 0xffffffffULL || sc > 0xffffffffULL) return ORC_E_RANGE;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Out(v) = sum of w over the edges at v (Section 3.1, definition under the  */
/* innerOuter rating).                                                      */
/* ------------------------------------------------------------------------ */
void orc_out(int32_t n, const int64_t *xadj, const uint32_t *ew, uint64_t *out)
{
    for (int32_t v = 0; v < n; ++v) {
        uint64_t s = 0;
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) s += ew[j];
        out[v] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Ratings of Section 3.1 as exact rationals num/den for the edge {u,v}.     */
/* ------------------------------------------------------------------------ */
static void rating(int kind, uint64_t w, uint64_t cu, uint64_t cv,
                   uint64_t out_u, uint64_t out_v, uint64_t *num, uint64_t *den)
{
    switch (kind) {
    case ORC_WEIGHT:          /* w(e) */
        *num = w; *den = 1; break;
    case ORC_EXPANSION:       /* w / (c(u) + c(v)) */
        *num = w; *den = cu + cv; break;
    case ORC_EXPANSION_STAR:  /* w / (c(u) c(v)) */
        *num = w; *den = cu * cv; break;
    case ORC_INNER_OUTER:     /* w / (Out(v) + Out(u) - 2 w) */
        *num = w; *den = out_u + out_v - 2 * w; break;
    case ORC_EXPANSION_STAR2: /* w^2 / (c(u) c(v)) */
    default:
        *num = w * w; *den = cu * cv; break;
    }
}

/* Rating of every CSR entry (both directions of each edge get the same value). */
int orc_rate(int32_t n, const int64_t *xadj, const int32_t *adj, const uint32_t *ew,
             const uint32_t *vw, int kind, uint64_t *num, uint64_t *den)
{
    if (kind < 0 || kind > 4) return ORC_E_ARG;
    uint64_t *out = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    orc_out(n, xadj, ew, out);
    for (int32_t v = 0; v < n; ++v)
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t u = adj[j];
            rating(kind, ew[j], vw[u], vw[v], out[u], out[v], &num[j], &den[j]);
        }
    free(out);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The strict order on edges.                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t a, b;        /* endpoints, a < b */
    uint64_t num, den;   /* rating */
    uint64_t h;          /* tie-break hash */
} orc_edge;

static uint64_t edge_id(int32_t x, int32_t y)
{
    uint64_t lo = (uint64_t)(x < y ? x : y), hi = (uint64_t)(x < y ? y : x);
    return (lo << 32) | hi;
}

/* +1 if e is above f in the order, -1 if below, 0 only if e and f are the
   same edge. */
static int edge_cmp(const orc_edge *e, const orc_edge *f)
{
    u128 l = (u128)e->num * f->den;
    u128 r = (u128)f->num * e->den;
    if (l != r) return l > r ? 1 : -1;
    if (e->h != f->h) return e->h > f->h ? 1 : -1;
    uint64_t ie = edge_id(e->a, e->b), jf = edge_id(f->a, f->b);
    if (ie != jf) return ie < jf ? 1 : -1;
    return 0;
}

static int edge_cmp_desc(const void *p, const void *q)
{
    return -edge_cmp((const orc_edge *)p, (const orc_edge *)q);
}

/* Fill the list of undirected edges {a,b}, a < b, with their ratings. */
static int64_t collect_edges(int32_t n, const int64_t *xadj, const int32_t *adj,
                             const uint32_t *ew, const uint32_t *vw, int kind,
                             uint64_t seed, orc_edge *edges)
{
    uint64_t *out = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    orc_out(n, xadj, ew, out);
    int64_t m = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t u = adj[j];
            if (u <= v) continue;
            orc_edge *e = &edges[m++];
            e->a = v; e->b = u;
            rating(kind, ew[j], vw[v], vw[u], out[v], out[u], &e->num, &e->den);
            e->h = orc_mix64(seed ^ edge_id(v, u));
        }
    free(out);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Matching, formulation A: Greedy (Section 3.2).  Edges are scanned in     */
/* descending order; an edge enters the matching if both ends are free.     */
/* Returns |M|; mate[v] = partner or -1.                                    */
/* ------------------------------------------------------------------------ */
int64_t orc_match_greedy(int32_t n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                         const uint32_t *ew, const uint32_t *vw, int kind, uint64_t seed,
                         int32_t *mate)
{
    orc_edge *edges = (orc_edge *)malloc((size_t)(nnz / 2 + 1) * sizeof(orc_edge));
    int64_t m = collect_edges(n, xadj, adj, ew, vw, kind, seed, edges);
    qsort(edges, (size_t)m, sizeof(orc_edge), edge_cmp_desc);
    for (int32_t v = 0; v < n; ++v) mate[v] = -1;
    int64_t matched = 0;
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = edges[i].a, b = edges[i].b;
        if (mate[a] < 0 && mate[b] < 0) { mate[a] = b; mate[b] = a; ++matched; }
    }
    free(edges);
    return matched;
}

/* ------------------------------------------------------------------------ */
/* Matching, formulation B: the parallel scheme of Section 3.3 run in       */
/* synchronous rounds.  In each round every free node that still has a free */
/* neighbour points at its best incident edge to a free neighbour; edges    */
/* that are best at both ends are matched; repeat until no free node has a  */
/* free neighbour.  round_active[r] / round_degree[r] (optional, capacity   */
/* max_rounds) receive the number of pointing nodes in round r and the sum  */
/* of their degrees.  Returns the number of rounds; *matched_out = |M|.     */
/* ------------------------------------------------------------------------ */
int32_t orc_match_rounds(int32_t n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                         const uint32_t *ew, const uint32_t *vw, int kind, uint64_t seed,
                         int32_t *mate, int64_t *matched_out,
                         int64_t *round_active, int64_t *round_degree, int32_t max_rounds)
{
    (void)nnz;
    uint64_t *out = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    orc_out(n, xadj, ew, out);
    int32_t *best = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v) mate[v] = -1;
    int32_t rounds = 0;
    int64_t matched = 0;
    for (;;) {
        int64_t active = 0, degsum = 0;
        for (int32_t v = 0; v < n; ++v) {
            best[v] = -1;
            if (mate[v] >= 0) continue;
            orc_edge cur, cand;
            int have = 0;
            for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
                int32_t u = adj[j];
                if (mate[u] >= 0) continue;
                cand.a = v < u ? v : u; cand.b = v < u ? u : v;
                rating(kind, ew[j], vw[v], vw[u], out[v], out[u], &cand.num, &cand.den);
                cand.h = orc_mix64(seed ^ edge_id(v, u));
                if (!have || edge_cmp(&cand, &cur) > 0) { cur = cand; best[v] = u; have = 1; }
            }
            if (have) { ++active; degsum += xadj[v + 1] - xadj[v]; }
        }
        if (active == 0) break;
        if (round_active && rounds < max_rounds) {
            round_active[rounds] = active;
            round_degree[rounds] = degsum;
        }
        ++rounds;
        for (int32_t v = 0; v < n; ++v) {
            int32_t u = best[v];
            if (u >= 0 && best[u] == v && v < u) { mate[v] = u; mate[u] = v; ++matched; }
        }
    }
    free(best);
    free(out);
    *matched_out = matched;
    return rounds;
}

/* ------------------------------------------------------------------------ */
/* Matching, formulation C: the two-phase scheme of Section 3.3.            */
/*   1. A preliminary partition of the nodes into blocks; here the initial  */
/*      numbering: block(v) = v >> block_bits.                              */
/*   2. A sequential matcher inside every block: Greedy (Section 3.2) over  */
/*      the edges whose two ends share a block.                             */
/*   3. The gap graph: the edges {u,v} between two blocks that are above,   */
/*      in the strict order, the edge matched in step 2 at u (if any) and   */
/*      the one at v (if any).                                              */
/*   4. The parallel matcher on the gap graph: local-max rounds, which      */
/*      under the strict order equal Greedy on the gap graph.               */
/*   5. A gap edge replaces the block edges at its ends; a node whose       */
/*      block partner is taken this way stays unmatched (the paper says no  */
/*      more about it).                                                     */
/* mate[v] = partner or -1; loc_out (optional) receives step 2's matching,  */
/* *gap_out (optional) the number of gap-graph edges and *gap_matched_out   */
/* (optional) the number matched in step 4.  Returns |M|.                   */
/* ------------------------------------------------------------------------ */
int64_t orc_match_two_phase(int32_t n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                            const uint32_t *ew, const uint32_t *vw, int kind, uint64_t seed,
                            int32_t block_bits, int32_t *mate, int32_t *loc_out,
                            int64_t *gap_out, int64_t *gap_matched_out)
{
    size_t n1 = (size_t)(n > 0 ? n : 1);
    orc_edge *all = (orc_edge *)malloc((size_t)(nnz / 2 + 1) * sizeof(orc_edge));
    orc_edge *list = (orc_edge *)malloc((size_t)(nnz / 2 + 1) * sizeof(orc_edge));
    int64_t m = collect_edges(n, xadj, adj, ew, vw, kind, seed, all);
    int32_t *loc = (int32_t *)malloc(n1 * sizeof(int32_t));
    int64_t *loc_edge = (int64_t *)malloc(n1 * sizeof(int64_t));   /* index into list */
    int32_t *gap = (int32_t *)malloc(n1 * sizeof(int32_t));
#define BLOCK_OF(x) ((int64_t)(x) >> block_bits)

    /* step 2: Greedy over the block-internal edges */
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i)
        if (BLOCK_OF(all[i].a) == BLOCK_OF(all[i].b)) list[k++] = all[i];
    qsort(list, (size_t)k, sizeof(orc_edge), edge_cmp_desc);
    for (int32_t v = 0; v < n; ++v) { loc[v] = -1; loc_edge[v] = -1; }
    for (int64_t i = 0; i < k; ++i) {
        int32_t a = list[i].a, b = list[i].b;
        if (loc[a] < 0 && loc[b] < 0) {
            loc[a] = b; loc[b] = a;
            loc_edge[a] = i; loc_edge[b] = i;
        }
    }

    /* step 3: the gap graph (kept in `all`, compacted in place) */
    int64_t g = 0;
    for (int64_t i = 0; i < m; ++i) {
        orc_edge e = all[i];
        if (BLOCK_OF(e.a) == BLOCK_OF(e.b)) continue;
        if (loc_edge[e.a] >= 0 && edge_cmp(&e, &list[loc_edge[e.a]]) < 0) continue;
        if (loc_edge[e.b] >= 0 && edge_cmp(&e, &list[loc_edge[e.b]]) < 0) continue;
        all[g++] = e;
    }

    /* step 4: Greedy on the gap graph */
    qsort(all, (size_t)g, sizeof(orc_edge), edge_cmp_desc);
    for (int32_t v = 0; v < n; ++v) gap[v] = -1;
    int64_t gm = 0;
    for (int64_t i = 0; i < g; ++i) {
        int32_t a = all[i].a, b = all[i].b;
        if (gap[a] < 0 && gap[b] < 0) { gap[a] = b; gap[b] = a; ++gm; }
    }

    /* step 5: gap edges first, then the block edges whose two ends are untouched */
    int64_t matched = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (gap[v] >= 0) mate[v] = gap[v];
        else if (loc[v] >= 0 && gap[loc[v]] < 0) mate[v] = loc[v];
        else mate[v] = -1;
        if (mate[v] > v) ++matched;
    }
#undef BLOCK_OF
    if (loc_out) memcpy(loc_out, loc, (size_t)(n > 0 ? n : 0) * sizeof(int32_t));
    if (gap_out) *gap_out = g;
    if (gap_matched_out) *gap_matched_out = gm;
    free(gap); free(loc_edge); free(loc); free(list); free(all);
    return matched;
}

/* ------------------------------------------------------------------------ */
/* Contraction (Section 2): each matched pair {u,v} becomes one node x with */
/* c(x) = c(u) + c(v); the edges of u and v move to x; parallel edges are   */
/* merged with summed weight; the contracted edge itself disappears.        */
/* Coarse numbering (the paper leaves it open): a node is a representative  */
/* if it is unmatched or the smaller end of its matched edge; coarse ids    */
/* are the representatives' ranks in ascending fine id; rows ascend.        */
/* Outputs: cmap[n], cvw[n'], cxadj[n'+1], cadj/cew[nnz'].  Capacities are  */
/* those of the fine graph.  Returns n'; *cnnz_out = nnz'.                  */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; uint32_t w; } orc_entry;

static int entry_cmp(const void *p, const void *q)
{
    uint64_t a = ((const orc_entry *)p)->key, b = ((const orc_entry *)q)->key;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int32_t orc_contract(int32_t n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                     const uint32_t *ew, const uint32_t *vw, const int32_t *mate,
                     int32_t *cmap, uint32_t *cvw, int64_t *cxadj, int32_t *cadj,
                     uint32_t *cew, int64_t *cnnz_out)
{
    /* coarse ids */
    int32_t nc = 0;
    for (int32_t v = 0; v < n; ++v)
        if (mate[v] < 0 || v < mate[v]) cmap[v] = nc++;
    for (int32_t v = 0; v < n; ++v)
        if (mate[v] >= 0 && v > mate[v]) cmap[v] = cmap[mate[v]];
    /* coarse node weights */
    for (int32_t x = 0; x < nc; ++x) cvw[x] = 0;
    for (int32_t v = 0; v < n; ++v) cvw[cmap[v]] += vw[v];
    /* every fine entry (v,u) that is not the contracted edge becomes a
       coarse entry (cmap v, cmap u); sort and merge equal pairs */
    orc_entry *ent = (orc_entry *)malloc((size_t)(nnz + 1) * sizeof(orc_entry));
    int64_t k = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t a = cmap[v], b = cmap[adj[j]];
            if (a == b) continue;
            ent[k].key = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
            ent[k].w = ew[j];
            ++k;
        }
    qsort(ent, (size_t)k, sizeof(orc_entry), entry_cmp);
    for (int32_t x = 0; x <= nc; ++x) cxadj[x] = 0;
    int64_t out = 0;
    for (int64_t i = 0; i < k; ) {
        uint64_t key = ent[i].key;
        uint64_t s = 0;
        while (i < k && ent[i].key == key) s += ent[i++].w;
        int32_t a = (int32_t)(key >> 32), b = (int32_t)(key & 0xffffffffu);
        cadj[out] = b;
        cew[out] = (uint32_t)s;
        ++out;
        cxadj[a + 1] += 1;
    }
    for (int32_t x = 0; x < nc; ++x) cxadj[x + 1] += cxadj[x];
    free(ent);
    *cnnz_out = out;
    return nc;
}

/* ------------------------------------------------------------------------ */
/* Stand-in for initial partitioning of the coarsest graph: block of x is    */
/* mix64(seed + x) mod k.  (The paper runs Scotch or pMetis here, Section 4; */
/* those systems are not part of this hierarchy.)                           */
/* ------------------------------------------------------------------------ */
void orc_initial_partition(int32_t n, int32_t k, uint64_t seed, int32_t *part)
{
    for (int32_t x = 0; x < n; ++x)
        part[x] = (int32_t)(orc_mix64(seed + (uint64_t)x) % (uint64_t)k);
}

/* Uncontraction seen as projection: a fine node takes the block of the
   coarse node it was contracted into (Section 2, "uncontracting"). */
void orc_project(int32_t n_fine, const int32_t *cmap, const int32_t *part_coarse,
                 int32_t *part_fine)
{
    for (int32_t v = 0; v < n_fine; ++v) part_fine[v] = part_coarse[cmap[v]];
}

/* ------------------------------------------------------------------------ */
/* Cut and balance (Section 2, and the imbalance of Section 5.2).           */
/*   cut      = sum over edges {u,v} with different blocks of w({u,v})      */
/*   W_i      = c(V_i)                                                      */
/*   L_max    = (1+eps) c(V)/k + max_v c(v), eps = eps_num/eps_den, kept as */
/*              the exact rational lmax_num / lmax_den                      */
/*   imbalance= max(0, max_i W_i - L_max)  (numerator over lmax_den)        */
/*   balance  = k max_i W_i / c(V)          (bal_num / bal_den)             */
/* res[] layout: cut, total, max_block, max_node, lmax_num, lmax_den,        */
/*               imb_num, bal_num, bal_den, feasible                         */
/* ------------------------------------------------------------------------ */
int orc_cut_balance(int32_t n, const int64_t *xadj, const int32_t *adj, const uint32_t *ew,
                    const uint32_t *vw, const int32_t *part, int32_t k,
                    uint32_t eps_num, uint32_t eps_den, uint64_t *block_w, uint64_t *res)
{
    /* k in [1, 4096], eps = eps_num/eps_den with eps_den in [1, 10^6] and
       eps_num <= 16 eps_den: every result below then fits 64 bits. */
    if (k < 1 || k > 4096 || eps_den == 0 || eps_den > 1000000u ||
        eps_num > 16000000u)
        return ORC_E_ARG;
    for (int32_t v = 0; v < n; ++v)
        if (part[v] < 0 || part[v] >= k) return ORC_E_RANGE;
    uint64_t cut = 0, total = 0, maxc = 0, maxw = 0;
    for (int32_t i = 0; i < k; ++i) block_w[i] = 0;
    for (int32_t v = 0; v < n; ++v) {
        block_w[part[v]] += vw[v];
        total += vw[v];
        if (vw[v] > maxc) maxc = vw[v];
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j)
            if (adj[j] > v && part[adj[j]] != part[v]) cut += ew[j];
    }
    for (int32_t i = 0; i < k; ++i) if (block_w[i] > maxw) maxw = block_w[i];
    u128 lnum = (u128)((uint64_t)eps_den + eps_num) * total + (u128)k * eps_den * maxc;
    u128 lden = (u128)k * eps_den;
    u128 lhs = lden * maxw;
    res[0] = cut;
    res[1] = total;
    res[2] = maxw;
    res[3] = maxc;
    res[4] = (uint64_t)lnum;
    res[5] = (uint64_t)lden;
    res[6] = lhs > lnum ? (uint64_t)(lhs - lnum) : 0;
    res[7] = (uint64_t)k * maxw;
    res[8] = total;
    res[9] = lhs <= lnum ? 1 : 0;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Greedy certificate, used to check a matching at sizes where re-running    */
/* Greedy is too slow.  A matching M equals the Greedy matching of the      */
/* strict order iff every edge outside M touches an edge of M that is above */
/* it (by induction over the descending scan).  Returns the number of edges */
/* that break this, plus the number of broken mate entries; 0 means M is    */
/* exactly the Greedy matching.                                             */
/* ------------------------------------------------------------------------ */
int64_t orc_greedy_certificate(int32_t n, const int64_t *xadj, const int32_t *adj,
                               const uint32_t *ew, const uint32_t *vw, int kind,
                               uint64_t seed, const int32_t *mate)
{
    uint64_t *out = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    orc_out(n, xadj, ew, out);
    int64_t bad = 0;
    /* M must be a matching made of graph edges */
    uint32_t *mw = (uint32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    for (int32_t v = 0; v < n; ++v) {
        int32_t u = mate[v];
        if (u < 0) continue;
        if (u >= n || u == v || mate[u] != v) { ++bad; continue; }
        uint32_t w;
        if (!row_contains(xadj, adj, ew, v, u, &w)) { ++bad; continue; }
        mw[v] = w;
    }
    if (bad) { free(mw); free(out); return bad; }
    for (int32_t v = 0; v < n; ++v)
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t u = adj[j];
            if (u <= v || mate[v] == u) continue;
            orc_edge f;
            f.a = v; f.b = u;
            rating(kind, ew[j], vw[v], vw[u], out[v], out[u], &f.num, &f.den);
            f.h = orc_mix64(seed ^ edge_id(v, u));
            int blocked = 0;
            int32_t ends[2] = {v, u};
            for (int t = 0; t < 2 && !blocked; ++t) {
                int32_t x = ends[t], y = mate[x];
                if (y < 0) continue;
                orc_edge g;
                g.a = x < y ? x : y; g.b = x < y ? y : x;
                rating(kind, mw[x], vw[x], vw[y], out[x], out[y], &g.num, &g.den);
                g.h = orc_mix64(seed ^ edge_id(x, y));
                if (edge_cmp(&g, &f) > 0) blocked = 1;
            }
            if (!blocked) ++bad;
        }
    free(mw);
    free(out);
    return bad;
}

/* ======================================================================== */
/* Refinement between pairs of blocks (Section 5).                          */
/*                                                                          */
/* Readings (the paper leaves these open; the GPU library follows the same  */
/* readings, written down in the design notes):                            */
/*   - Q has an edge {a, b} (a < b) iff some edge of G joins blocks a and b.  */
/*     Q's edges are coloured by the sequential greedy edge colouring that  */
/*     Section 5.1 parallelises: edges in ascending (a, b) order, each     */
/*     taking the smallest colour unused at both ends.  Pairs of one colour */
/*     share no block, so their local searches are independent.             */
/*   - gain(v) = w(v, other block) - w(v, own block), counting only the    */
/*     neighbours inside the two blocks (Section 5.2).                      */
/*   - the queue order is: larger gain, then larger mix64(run_seed ^ v),    */
/*     then smaller v (the paper breaks ties at random).                    */
/*   - the search area is the bounded BFS of Section 5.2: inside each block,*/
/*     the nodes within `depth` same-block hops of a node adjacent to the   */
/*     other block.  Queues start with the boundary nodes (distance 0); a  */
/*     node of the area enters its queue when a neighbour moves.             */
/*   - queue selection TopGain: the larger top under the queue order; when  */
/*     one block is overloaded (c > L_max) and the weights differ, MaxLoad: */
/*     the heavier block gives (the other queue if the heavier one is      */
/*     empty).  Moves are never refused; the rollback keeps balance.        */
/*   - the search stops when both queues are empty or when more than        */
/*     alpha * min(|A|, |B|) moves (node counts at the start) followed the  */
/*     last improvement; it is rolled back to the first state with the      */
/*     lexicographically smallest (imbalance, cut), where imbalance =      */
/*     max(0, c(A) - L_max, c(B) - L_max), scaled by k * eps_den.           */
/*   - each local search runs twice, with run seeds r = 0 and 1 (the two    */
/*     PEs of Section 5); the better end state is adopted (r = 0 on a tie). */
/*     A pair repeats local searches (local iterations) until one brings   */
/*     no strict improvement or max_local were run; a global iteration     */
/*     walks all colours in ascending order; global iterations repeat until */
/*     stop_after of them in a row improved nothing (Table 2: "no change"  */
/*     is 1, "2x no change" is 2) or max_global were run.                   */
/*   - run seed = mix64(mix64(mix64(seed + g) ^ ((a << 32) | b)) + 2 t + r) */
/*     for global iteration g, pair (a, b), local iteration t, run r.       */
/* ======================================================================== */

/* Q and its greedy edge colouring.  Writes the pairs in ascending (a, b)
   order with their colours; returns the number of colours (at most 2k - 3
   for k >= 2: greedy needs at most 2 * maxdeg(Q) - 1). */
int32_t orc_quotient_colouring(int32_t n, const int64_t *xadj, const int32_t *adj,
                               const int32_t *part, int32_t k, int32_t *pair_a,
                               int32_t *pair_b, int32_t *colour, int32_t *npairs)
{
    uint8_t *q = (uint8_t *)calloc((size_t)k * k, 1);
    for (int32_t v = 0; v < n; ++v)
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t a = part[v], b = part[adj[j]];
            if (a < b) q[(size_t)a * k + b] = 1;
        }
    int32_t ncol_cap = 2 * k;
    uint8_t *used = (uint8_t *)calloc((size_t)k * ncol_cap, 1);
    int32_t m = 0, ncol = 0;
    for (int32_t a = 0; a < k; ++a)
        for (int32_t b = a + 1; b < k; ++b) {
            if (!q[(size_t)a * k + b]) continue;
            int32_t c = 0;
            while (used[(size_t)a * ncol_cap + c] || used[(size_t)b * ncol_cap + c]) ++c;
            used[(size_t)a * ncol_cap + c] = used[(size_t)b * ncol_cap + c] = 1;
            pair_a[m] = a;
            pair_b[m] = b;
            colour[m] = c;
            ++m;
            if (c + 1 > ncol) ncol = c + 1;
        }
    free(used);
    free(q);
    *npairs = m;
    return ncol;
}

/* (imbalance, cut) order: is (i1, c1) strictly below (i2, c2)? */
static int state_below(int64_t i1, int64_t c1, int64_t i2, int64_t c2)
{
    return i1 < i2 || (i1 == i2 && c1 < c2);
}

/* scaled imbalance of a pair: max(0, S c(A) - L, S c(B) - L) with
   S = k eps_den and L = (eps_den + eps_num) c(V) + S max_v c(v) */
static int64_t pair_imbalance(int64_t wa, int64_t wb, int64_t s, int64_t l)
{
    int64_t x = s * (wa > wb ? wa : wb) - l;
    return x > 0 ? x : 0;
}

/* is queue entry (g1, h1, v1) above (g2, h2, v2)? */
static int entry_above(int64_t g1, uint64_t h1, int32_t v1, int64_t g2, uint64_t h2, int32_t v2)
{
    if (g1 != g2) return g1 > g2;
    if (h1 != h2) return h1 > h2;
    return v1 < v2;
}

/* Work arrays of the local searches, indexed by node id and allocated once
   per refinement call: side[] is -1 and status[], gain[], dist[] are zero /
   zero / -1 for every node outside a running search (each search resets the
   nodes of its two blocks when it ends). */
typedef struct {
    int64_t g;
    uint64_t h;
    int32_t v;
} fm_entry;
typedef struct {
    fm_entry *e;
    int64_t n, cap;
} fm_heap;
typedef struct {
    int8_t *side, *status; /* status: 0 idle, 1 queued, 2 moved */
    int64_t *gain;
    int32_t *dist, *bfs;
    fm_heap q[2];
} fm_work;

static void fm_work_init(fm_work *w, int32_t n)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    w->side = (int8_t *)malloc(nn);
    w->status = (int8_t *)calloc(nn, 1);
    w->gain = (int64_t *)calloc(nn, sizeof(int64_t));
    w->dist = (int32_t *)malloc(nn * sizeof(int32_t));
    w->bfs = (int32_t *)malloc(nn * sizeof(int32_t));
    for (size_t v = 0; v < nn; ++v) { w->side[v] = -1; w->dist[v] = -1; }
    for (int i = 0; i < 2; ++i) {
        w->q[i].cap = 1024;
        w->q[i].n = 0;
        w->q[i].e = (fm_entry *)malloc((size_t)w->q[i].cap * sizeof(fm_entry));
    }
}

static void fm_work_free(fm_work *w)
{
    free(w->side); free(w->status); free(w->gain); free(w->dist); free(w->bfs);
    free(w->q[0].e); free(w->q[1].e);
}

/* Binary max-heap under the queue order (entry_above); a node whose gain
   changes while queued gets a new entry, and entries whose node moved or
   whose gain is no longer current are dropped when they reach the top. */
static void heap_push(fm_heap *q, int64_t g, uint64_t h, int32_t v)
{
    if (q->n == q->cap) {
        q->cap *= 2;
        q->e = (fm_entry *)realloc(q->e, (size_t)q->cap * sizeof(fm_entry));
    }
    int64_t i = q->n++;
    fm_entry x = {g, h, v};
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!entry_above(x.g, x.h, x.v, q->e[p].g, q->e[p].h, q->e[p].v)) break;
        q->e[i] = q->e[p];
        i = p;
    }
    q->e[i] = x;
}

static void heap_pop(fm_heap *q)
{
    fm_entry x = q->e[--q->n];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= q->n) break;
        if (c + 1 < q->n && entry_above(q->e[c + 1].g, q->e[c + 1].h, q->e[c + 1].v, q->e[c].g,
                                        q->e[c].h, q->e[c].v))
            ++c;
        if (!entry_above(q->e[c].g, q->e[c].h, q->e[c].v, x.g, x.h, x.v)) break;
        q->e[i] = q->e[c];
        i = c;
    }
    if (q->n > 0) q->e[i] = x;
}

/* The queued node with the largest (gain, hash, smaller id), or -1. */
static int32_t heap_top(fm_heap *q, const int8_t *status, const int64_t *gain)
{
    while (q->n > 0) {
        fm_entry t = q->e[0];
        if (status[t.v] == 1 && gain[t.v] == t.g) return t.v;
        heap_pop(q);
    }
    return -1;
}

/* One two-block local search on blocks a and b of part (part is not
   changed); nodes[0 .. nn) are the nodes of the two blocks.  moves (capacity
   nn) receives the moved nodes in order.  res: start imbalance, start cut,
   end imbalance, end cut, moves made, moves kept (the rolled-back prefix),
   with imbalances scaled by s. */
static void fm_pair(fm_work *W, const int64_t *xadj, const int32_t *adj, const uint32_t *ew,
                    const uint32_t *vw, const int32_t *part, const int32_t *nodes, int64_t nn,
                    int32_t a, int32_t b, int64_t wa, int64_t wb, int64_t s, int64_t l,
                    uint64_t run_seed, uint32_t alpha_num, uint32_t alpha_den, int32_t depth,
                    int32_t *moves, int64_t *res)
{
    (void)b;   // side 1 is every listed node not in block a
    int8_t *side = W->side, *status = W->status;
    int64_t *gain = W->gain;
    int32_t *dist = W->dist, *bfs = W->bfs;
    int64_t cnt[2] = {0, 0}, cut = 0;
    for (int64_t i = 0; i < nn; ++i) {
        int32_t v = nodes[i];
        side[v] = part[v] == a ? 0 : 1;
        ++cnt[side[v]];
    }
    /* gains, boundary, cut */
    int32_t head = 0, tail = 0;
    for (int64_t i = 0; i < nn; ++i) {
        int32_t v = nodes[i];
        int boundary = 0;
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t u = adj[j];
            if (side[u] < 0) continue;
            if (side[u] != side[v]) {
                gain[v] += ew[j];
                boundary = 1;
                if (side[v] == 0) cut += ew[j];
            } else {
                gain[v] -= ew[j];
            }
        }
        if (boundary) { dist[v] = 0; bfs[tail++] = v; }
    }
    /* bounded BFS inside each block from its boundary */
    while (head < tail) {
        int32_t v = bfs[head++];
        if (dist[v] >= depth) continue;
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t u = adj[j];
            if (side[u] == side[v] && dist[u] < 0) { dist[u] = dist[v] + 1; bfs[tail++] = u; }
        }
    }
    /* the queues start with the boundary */
    W->q[0].n = W->q[1].n = 0;
    for (int64_t i = 0; i < nn; ++i) {
        int32_t v = nodes[i];
        if (dist[v] == 0) {
            status[v] = 1;
            heap_push(&W->q[side[v]], gain[v], orc_mix64(run_seed ^ (uint64_t)v), v);
        }
    }

    int64_t w[2] = {wa, wb};
    int64_t best_imb = pair_imbalance(w[0], w[1], s, l), best_cut = cut;
    res[0] = best_imb;
    res[1] = best_cut;
    int32_t m = 0, kept = 0;
    int64_t since = 0, smaller = cnt[0] < cnt[1] ? cnt[0] : cnt[1];
    for (;;) {
        /* the top of each queue */
        int32_t top[2] = {heap_top(&W->q[0], status, gain), heap_top(&W->q[1], status, gain)};
        if (top[0] < 0 && top[1] < 0) break;
        int from;
        int overloaded = s * w[0] > l || s * w[1] > l;
        if (overloaded && w[0] != w[1]) {
            from = w[0] > w[1] ? 0 : 1;                 /* MaxLoad */
            if (top[from] < 0) from = 1 - from;
        } else if (top[0] < 0 || top[1] < 0) {
            from = top[0] < 0 ? 1 : 0;
        } else {                                         /* TopGain */
            uint64_t h0 = orc_mix64(run_seed ^ (uint64_t)top[0]);
            uint64_t h1 = orc_mix64(run_seed ^ (uint64_t)top[1]);
            from = entry_above(gain[top[0]], h0, top[0], gain[top[1]], h1, top[1]) ? 0 : 1;
        }
        int32_t v = top[from];
        int to = 1 - from;
        status[v] = 2;
        side[v] = (int8_t)to;
        w[from] -= vw[v];
        w[to] += vw[v];
        cut -= gain[v];
        moves[m++] = v;
        for (int64_t j = xadj[v]; j < xadj[v + 1]; ++j) {
            int32_t u = adj[j];
            if (side[u] < 0 || status[u] == 2) continue;
            if (side[u] == to) gain[u] -= 2 * (int64_t)ew[j];
            else gain[u] += 2 * (int64_t)ew[j];
            if (status[u] == 0 && dist[u] >= 0) status[u] = 1;
            if (status[u] == 1)
                heap_push(&W->q[side[u]], gain[u], orc_mix64(run_seed ^ (uint64_t)u), u);
        }
        int64_t imb = pair_imbalance(w[0], w[1], s, l);
        if (state_below(imb, cut, best_imb, best_cut)) {
            best_imb = imb;
            best_cut = cut;
            kept = m;
            since = 0;
        } else {
            ++since;
        }
        if (since * (int64_t)alpha_den > (int64_t)alpha_num * smaller) break;
    }
    res[2] = best_imb;
    res[3] = best_cut;
    res[4] = m;
    res[5] = kept;
    for (int64_t i = 0; i < nn; ++i) {   /* leave the work arrays clean */
        int32_t v = nodes[i];
        side[v] = -1;
        status[v] = 0;
        gain[v] = 0;
        dist[v] = -1;
    }
}

static int refine_args_ok(int32_t k, uint32_t eps_num, uint32_t eps_den, uint32_t alpha_den,
                          int32_t depth)
{
    return k >= 1 && k <= 256 && eps_den >= 1 && eps_den <= 1000000u &&
           eps_num <= 16000000u && alpha_den >= 1 && depth >= 0;
}

/* S = k eps_den and L = (eps_den + eps_num) c(V) + S max_v c(v), and the
   block weights */
static void refine_scale(int32_t n, const uint32_t *vw, const int32_t *part, int32_t k,
                         uint32_t eps_num, uint32_t eps_den, int64_t *bw, int64_t *s, int64_t *l)
{
    int64_t total = 0, maxc = 0;
    for (int32_t i = 0; i < k; ++i) bw[i] = 0;
    for (int32_t v = 0; v < n; ++v) {
        bw[part[v]] += vw[v];
        total += vw[v];
        if ((int64_t)vw[v] > maxc) maxc = vw[v];
    }
    *s = (int64_t)k * eps_den;
    *l = ((int64_t)eps_den + eps_num) * total + *s * maxc;
}

/* One local search on blocks a < b with the given run seed (for tests). */
int orc_fm_pair(int32_t n, const int64_t *xadj, const int32_t *adj, const uint32_t *ew,
                const uint32_t *vw, const int32_t *part, int32_t k, int32_t a, int32_t b,
                uint32_t eps_num, uint32_t eps_den, uint64_t run_seed, uint32_t alpha_num,
                uint32_t alpha_den, int32_t depth, int32_t *moves, int64_t *res)
{
    if (!refine_args_ok(k, eps_num, eps_den, alpha_den, depth) || a < 0 || b <= a || b >= k)
        return ORC_E_ARG;
    for (int32_t v = 0; v < n; ++v)
        if (part[v] < 0 || part[v] >= k) return ORC_E_RANGE;
    int64_t *bw = (int64_t *)malloc((size_t)k * sizeof(int64_t)), s, l;
    refine_scale(n, vw, part, k, eps_num, eps_den, bw, &s, &l);
    int32_t *nodes = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t nn = 0;
    for (int32_t v = 0; v < n; ++v)
        if (part[v] == a || part[v] == b) nodes[nn++] = v;
    fm_work W;
    fm_work_init(&W, n);
    fm_pair(&W, xadj, adj, ew, vw, part, nodes, nn, a, b, bw[a], bw[b], s, l, run_seed, alpha_num,
            alpha_den, depth, moves, res);
    fm_work_free(&W);
    free(nodes);
    free(bw);
    return ORC_OK;
}

uint64_t orc_run_seed(uint64_t seed, int32_t g, int32_t a, int32_t b, int32_t t, int32_t r)
{
    uint64_t h = orc_mix64(seed + (uint64_t)g);
    h = orc_mix64(h ^ (((uint64_t)(uint32_t)a << 32) | (uint32_t)b));
    return orc_mix64(h + 2 * (uint64_t)t + (uint64_t)r);
}

/* Pairwise refinement of one level, in place on part.  stats: global
   iterations run, local searches run, moves made, moves kept, adoptions
   (local iterations that improved), colours summed over global iterations. */
int orc_refine(int32_t n, const int64_t *xadj, const int32_t *adj, const uint32_t *ew,
               const uint32_t *vw, int32_t *part, int32_t k, uint32_t eps_num, uint32_t eps_den,
               uint64_t seed, uint32_t alpha_num, uint32_t alpha_den, int32_t depth,
               int32_t max_local, int32_t max_global, int32_t stop_after, int64_t *stats)
{
    if (!refine_args_ok(k, eps_num, eps_den, alpha_den, depth) || max_local < 1 ||
        max_global < 0 || stop_after < 1)
        return ORC_E_ARG;
    for (int32_t v = 0; v < n; ++v)
        if (part[v] < 0 || part[v] >= k) return ORC_E_RANGE;
    for (int i = 0; i < 6; ++i) stats[i] = 0;
    int64_t *bw = (int64_t *)malloc((size_t)k * sizeof(int64_t)), s, l;
    refine_scale(n, vw, part, k, eps_num, eps_den, bw, &s, &l);
    size_t kk = (size_t)k * k / 2 + 1, nn = (size_t)(n > 0 ? n : 1);
    int32_t *pa = (int32_t *)malloc(kk * sizeof(int32_t));
    int32_t *pb = (int32_t *)malloc(kk * sizeof(int32_t));
    int32_t *pc = (int32_t *)malloc(kk * sizeof(int32_t));
    int32_t *mv[2] = {(int32_t *)malloc(nn * sizeof(int32_t)), (int32_t *)malloc(nn * sizeof(int32_t))};
    /* the nodes of every block, ascending (blocks a and b change together,
       after an adoption in their pair) */
    int32_t **bl = (int32_t **)calloc((size_t)k, sizeof(int32_t *));
    int64_t *bn = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int32_t *pnodes = (int32_t *)malloc(nn * sizeof(int32_t));
    fm_work W;
    fm_work_init(&W, n);
    int32_t idle = 0;
    for (int32_t g = 0; g < max_global; ++g) {
        int32_t np;
        int32_t ncol = orc_quotient_colouring(n, xadj, adj, part, k, pa, pb, pc, &np);
        stats[0] += 1;
        stats[5] += ncol;
        for (int32_t i = 0; i < k; ++i) bn[i] = 0;
        for (int32_t v = 0; v < n; ++v) ++bn[part[v]];
        for (int32_t i = 0; i < k; ++i) {
            bl[i] = (int32_t *)realloc(bl[i], (size_t)(bn[i] > 0 ? bn[i] : 1) * sizeof(int32_t));
            bn[i] = 0;
        }
        for (int32_t v = 0; v < n; ++v) bl[part[v]][bn[part[v]]++] = v;
        int improved = 0;
        for (int32_t c = 0; c < ncol; ++c)
            for (int32_t p = 0; p < np; ++p) {
                if (pc[p] != c) continue;
                int32_t a = pa[p], b = pb[p];
                for (int32_t t = 0; t < max_local; ++t) {
                    /* the nodes of blocks a and b, in ascending id order */
                    int64_t na = bn[a], nb = bn[b], nab = 0;
                    {
                        int64_t i = 0, j = 0;
                        const int32_t *la = bl[a], *lb = bl[b];
                        while (i < na || j < nb)
                            pnodes[nab++] = (j >= nb || (i < na && la[i] < lb[j])) ? la[i++] : lb[j++];
                    }
                    int64_t res[2][6];
                    for (int r = 0; r < 2; ++r)
                        fm_pair(&W, xadj, adj, ew, vw, part, pnodes, nab, a, b, bw[a], bw[b], s,
                                l, orc_run_seed(seed, g, a, b, t, r), alpha_num, alpha_den, depth,
                                mv[r], res[r]);
                    stats[1] += 2;
                    stats[2] += res[0][4] + res[1][4];
                    int r = state_below(res[1][2], res[1][3], res[0][2], res[0][3]) ? 1 : 0;
                    if (!state_below(res[r][2], res[r][3], res[r][0], res[r][1])) break;
                    for (int64_t i = 0; i < res[r][5]; ++i) {
                        int32_t v = mv[r][i];
                        int32_t to = part[v] == a ? b : a;
                        bw[part[v]] -= vw[v];
                        bw[to] += vw[v];
                        part[v] = to;
                    }
                    /* the two blocks' node lists after the moves */
                    bl[a] = (int32_t *)realloc(bl[a], (size_t)(nab > 0 ? nab : 1) * sizeof(int32_t));
                    bl[b] = (int32_t *)realloc(bl[b], (size_t)(nab > 0 ? nab : 1) * sizeof(int32_t));
                    bn[a] = bn[b] = 0;
                    for (int64_t i = 0; i < nab; ++i) {
                        int32_t v = pnodes[i];
                        if (part[v] == a) bl[a][bn[a]++] = v; else bl[b][bn[b]++] = v;
                    }
                    stats[3] += res[r][5];
                    stats[4] += 1;
                    improved = 1;
                }
            }
        idle = improved ? 0 : idle + 1;
        if (idle >= stop_after) break;
    }
    fm_work_free(&W);
    for (int32_t i = 0; i < k; ++i) free(bl[i]);
    free(bl); free(bn); free(pnodes);
    free(pa); free(pb); free(pc); free(mv[0]); free(mv[1]); free(bw);
    return ORC_OK;
}
