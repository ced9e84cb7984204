/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU statement of the speculative greedy coloring of
 * Tas, Kaya and Saule, "Greed is Good: Optimistic Algorithms for
 * Bipartite-Graph Partial Coloring on Multicore Architectures" (2017),
 * run with fixed round semantics so that every round has one exact result.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file; the coloring library never links, calls or includes it,
 * and it shares no code, header or table with the device implementation.
 *
 * Problem (Section II): color the V_A side of a bipartite graph so that any
 * two vertices sharing a V_B net differ; colors are non-negative, -1 marks an
 * uncolored vertex.  nets(u) lists the nets of vertex u, vtxs(v) the vertices
 * of net v.  For distance-2 coloring (Section IV) the nets are the closed
 * neighbourhoods N[v] = {v} u nbor(v) of a symmetric graph.
 *
 * Round semantics fixed here where the paper's threads race:
 *   - every round reads a snapshot s of the previous round's colors and
 *     writes a tentative array t (Algorithm 1's loop run Jacobi-style);
 *   - removal is global: u loses iff some x sharing a net with u has
 *     t[x] == t[u] and a lower rank (the rule of Algorithm 3); a loser is
 *     reset to -1 (as Algorithms 7 and 10 do);
 *   - a net-based round (Algorithm 8 / 9) writes vertex x only from its
 *     owner net: the largest net containing x, ties to the lowest net id;
 *   - the balancing state of Algorithms 11 and 12 lives per chunk of `chunk`
 *     consecutive worklist entries and restarts every round.
 * Ranks are vertex ids; a caller-supplied order is applied by relabelling the
 * graph before the call (oracle/__init__.py).
 *
 * Every parallel loop below runs items that do not read each other's output
 * within the round, so the OpenMP schedule cannot change any result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

enum { OR_OK = 0, OR_E_INVALID = -1, OR_E_NOT_CONVERGED = -6, OR_E_INTERNAL = -8 };
enum { POL_FF = 0, POL_B1 = 1, POL_B2 = 2, POL_B1G = 3 };

typedef struct {
    int32_t n_a, n_b, d2;
    const int64_t *a_off; const int32_t *a_idx;   /* nets(u)  (d2: nbor(u)) */
    const int64_t *b_off; const int32_t *b_idx;   /* vtxs(v)  (d2: nbor(v)) */
} graph_t;

/* nets(u); in distance-2 mode N[u] = {u} followed by nbor(u) */
static int64_t nets_count(const graph_t *g, int32_t u)
{
    int64_t k = g->a_off[u + 1] - g->a_off[u];
    return g->d2 ? k + 1 : k;
}
static int32_t net_at(const graph_t *g, int32_t u, int64_t k)
{
    if (g->d2) {
        if (k == 0) return u;
        k -= 1;
    }
    return g->a_idx[g->a_off[u] + k];
}
/* vtxs(v); in distance-2 mode the center v comes first (Algorithm 9), then nbor(v) */
static int64_t vtxs_count(const graph_t *g, int32_t v)
{
    int64_t k = g->b_off[v + 1] - g->b_off[v];
    return g->d2 ? k + 1 : k;
}
static int32_t vtx_at(const graph_t *g, int32_t v, int64_t k)
{
    if (g->d2) {
        if (k == 0) return v;
        k -= 1;
    }
    return g->b_idx[g->b_off[v] + k];
}

/* A forbidden-color set F kept as a marker array that is never cleared:
 * color col is in F iff mark[col] == cur (the marker trick of the paper's
 * implementation notes at the end of Section III). */
typedef struct {
    int64_t *mark;
    int32_t *holder;
    int64_t cap;
    int64_t cur;
} fset_t;

static int fset_init(fset_t *f, int64_t cap)
{
    f->cap = cap;
    f->cur = 0;
    f->mark = (int64_t *)calloc((size_t)cap, sizeof(int64_t));
    f->holder = (int32_t *)calloc((size_t)cap, sizeof(int32_t));
    return (f->mark && f->holder) ? 0 : -1;
}
static void fset_free(fset_t *f)
{
    free(f->mark);
    free(f->holder);
}
static void fset_clear(fset_t *f) { f->cur++; }
static int fset_has(const fset_t *f, int64_t col)
{
    return col >= 0 && col < f->cap && f->mark[col] == f->cur;
}
static void fset_add(fset_t *f, int64_t col) { f->mark[col] = f->cur; }

typedef struct { int64_t col_max, col_next; } chunk_state_t;

/* smallest color >= from that is not in F */
static int64_t free_at_or_above(const fset_t *F, int64_t from)
{
    int64_t c = from;
    while (fset_has(F, c)) c++;
    return c;
}

/* largest color <= from that is not in F, or -1 when [0, from] is all in F */
static int64_t free_at_or_below(const fset_t *F, int64_t from)
{
    int64_t c = from;
    while (c >= 0 && fset_has(F, c)) c--;
    return c;
}

/* The color policies, each stated as the color it picks for a forbidden set F.
 *   First-fit (Algorithm 2): the smallest free color.
 *   B1 (Algorithm 11): an even rank takes the largest free color not above
 *     col_max, or, when [0, col_max] is all forbidden, the smallest free color
 *     above col_max; an odd rank takes first-fit.  col_max then grows to the
 *     pick.
 *   B1G: B1's pick with col_max fixed for the whole round to the largest
 *     color of the round's snapshot (-1 before any color); no state passes
 *     between vertices.
 *   B2 (Algorithm 12): the smallest free color at or above col_next if it does
 *     not exceed col_max, else first-fit.  col_max grows to the pick and
 *     col_next becomes the pick + 1 capped at col_max / 3 + 1 (integer floor). */
static int64_t policy_pick(int policy, const fset_t *F, chunk_state_t *st, int32_t rank)
{
    int64_t col;
    switch (policy) {
    case POL_B1:
    case POL_B1G:
        if (rank % 2 == 0) {
            col = free_at_or_below(F, st->col_max);
            if (col < 0) col = free_at_or_above(F, st->col_max + 1);
        } else {
            col = free_at_or_above(F, 0);
        }
        if (policy == POL_B1 && col > st->col_max) st->col_max = col;
        return col;
    case POL_B2: {
        col = free_at_or_above(F, st->col_next);
        if (col > st->col_max) col = free_at_or_above(F, 0);
        if (col > st->col_max) st->col_max = col;
        const int64_t cap = st->col_max / 3 + 1;
        st->col_next = col + 1 < cap ? col + 1 : cap;
        return col;
    }
    default:
        return free_at_or_above(F, 0);
    }
}

/* owner(u): the net of u with the most vertices, ties to the lowest net id. */
static void compute_owner(const graph_t *g, int32_t *owner)
{
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t u = 0; u < g->n_a; u++) {
        int32_t best = -1;
        int64_t best_size = -1;
        int64_t k = nets_count(g, u);
        for (int64_t j = 0; j < k; j++) {
            int32_t v = net_at(g, u, j);
            int64_t sz = vtxs_count(g, v);
            if (sz > best_size || (sz == best_size && v < best)) {
                best = v;
                best_size = sz;
            }
        }
        owner[u] = best;
    }
}

static int64_t max_net_size(const graph_t *g)
{
    int64_t m = 0;
    for (int32_t v = 0; v < g->n_b; v++) {
        int64_t k = vtxs_count(g, v);
        if (k > m) m = k;
    }
    return m;
}

/*
 * Vertex-based coloring of the worklist (Algorithm 4 gathering F, Algorithm 2
 * first-fit or Algorithms 11 / 12 choosing the color).  F(w) is every color
 * found in the snapshot among the vertices sharing a net with w.
 */
static int color_vertex_round(const graph_t *g, const int32_t *s, int32_t *t,
                              const int32_t *W, int64_t nw, int policy, int32_t chunk,
                              int64_t color_cap)
{
    int err = 0;
    int64_t nchunks = (nw + chunk - 1) / chunk;
    int64_t snap_max = -1;   /* largest color of the snapshot (B1G) */
    for (int32_t x = 0; x < g->n_a; x++)
        if (s[x] > snap_max) snap_max = s[x];
    #pragma omp parallel reduction(| : err)
    {
        fset_t F;
        if (fset_init(&F, color_cap)) {
            err |= 1;
        } else {
            #pragma omp for schedule(dynamic, 1)
            for (int64_t ch = 0; ch < nchunks; ch++) {
                chunk_state_t st = {policy == POL_B1G ? snap_max : 0, 0};
                int64_t lo = ch * chunk, hi = lo + chunk < nw ? lo + chunk : nw;
                for (int64_t i = lo; i < hi; i++) {
                    int32_t w = W[i];
                    fset_clear(&F);
                    int64_t kn = nets_count(g, w);
                    for (int64_t a = 0; a < kn; a++) {
                        int32_t v = net_at(g, w, a);
                        int64_t kv = vtxs_count(g, v);
                        for (int64_t b = 0; b < kv; b++) {
                            int32_t x = vtx_at(g, v, b);
                            if (x != w && s[x] != -1) fset_add(&F, s[x]);
                        }
                    }
                    int64_t col = policy_pick(policy, &F, &st, w);
                    if (col + 1 >= color_cap) err |= 2;
                    t[w] = (int32_t)col;
                }
            }
            fset_free(&F);
        }
    }
    return err ? OR_E_INTERNAL : OR_OK;
}

/* ascending int comparison for qsort */
static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* is col in the ascending array a[0..n)? */
static int sorted_has(const int32_t *a, int64_t n, int32_t col)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (a[mid] == col) return 1;
        if (a[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return 0;
}

/*
 * Vertex-based first-fit through per-net color sets (same result as
 * color_vertex_round with first-fit, for graphs whose neighbourhoods are too
 * large to gather vertex by vertex).  F(w) is the union over v in nets(w) of
 * C_v, the snapshot colors of v's colored members (w itself is uncolored, so
 * excluding it changes nothing).  First-fit is the smallest color in no C_v.
 * Every color below ff_v (the smallest color missing from C_v) lies in C_v and
 * hence in F(w), so the search starts at the largest ff_v over w's nets; each
 * candidate is then tested against every C_v (kept sorted).
 */
static int color_vertex_round_sets(const graph_t *g, const int32_t *s, int32_t *t,
                                   const int32_t *W, int64_t nw)
{
    int err = 0;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)g->n_b + 1));
    int32_t *ff = (int32_t *)malloc(sizeof(int32_t) * ((size_t)g->n_b + 1));
    if (!off || !ff) { free(off); free(ff); return OR_E_INTERNAL; }
    off[0] = 0;
    for (int32_t v = 0; v < g->n_b; v++) off[v + 1] = off[v] + vtxs_count(g, v);
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * ((size_t)off[g->n_b] + 1));
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * ((size_t)g->n_b + 1));
    if (!col || !cnt) { free(off); free(ff); free(col); free(cnt); return OR_E_INTERNAL; }
    /* C_v, sorted, and ff_v, for the nets of worklist vertices (no other
     * net is looked at this round) */
    uint8_t *need = (uint8_t *)calloc((size_t)g->n_b + 1, 1);
    if (!need) { free(off); free(ff); free(col); free(cnt); return OR_E_INTERNAL; }
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nw; i++) {
        int64_t kn = nets_count(g, W[i]);
        for (int64_t a = 0; a < kn; a++) need[net_at(g, W[i], a)] = 1;
    }
    #pragma omp parallel for schedule(dynamic, 256) reduction(| : err)
    for (int32_t v = 0; v < g->n_b; v++) {
        cnt[v] = 0;
        ff[v] = 0;
        if (!need[v]) continue;
        int32_t *c = col + off[v];
        int64_t k = 0, kv = vtxs_count(g, v);
        for (int64_t b = 0; b < kv; b++) {
            int32_t x = vtx_at(g, v, b);
            if (s[x] != -1) c[k++] = s[x];
        }
        qsort(c, (size_t)k, sizeof(int32_t), cmp_int);
        int32_t f = 0;
        for (int64_t i = 0; i < k; i++) {
            if (i > 0 && c[i] == c[i - 1]) err |= 4;   /* colored members of a net differ */
            if (c[i] == f) f++;
        }
        cnt[v] = k;
        ff[v] = f;
    }
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nw; i++) {
        int32_t w = W[i];
        int64_t kn = nets_count(g, w);
        int32_t c = 0;
        for (int64_t a = 0; a < kn; a++) {
            int32_t v = net_at(g, w, a);
            if (ff[v] > c) c = ff[v];
        }
        for (;;) {
            int used = 0;
            for (int64_t a = 0; a < kn && !used; a++) {
                int32_t v = net_at(g, w, a);
                used = sorted_has(col + off[v], cnt[v], c);
            }
            if (!used) break;
            c++;
        }
        t[w] = c;
    }
    free(off); free(ff); free(col); free(cnt); free(need);
    return err ? OR_E_INTERNAL : OR_OK;
}

/*
 * Explicit neighbour lists nbor(u) (Section II: the vertices other than u
 * sharing a net with u), built once per call when they are small (dense
 * graphs, where walking the nets of every worklist vertex every round repeats
 * the same vertices many times).  off[n_a + 1], idx: ascending per vertex.
 */
typedef struct { int64_t *off; int32_t *idx; } nbor_t;

static int build_nbor(const graph_t *g, nbor_t *nb)
{
    int err = 0;
    int64_t *cnt = (int64_t *)calloc((size_t)g->n_a + 1, sizeof(int64_t));
    nb->off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)g->n_a + 1));
    nb->idx = NULL;
    if (!cnt || !nb->off) { free(cnt); return -1; }
    for (int pass = 0; pass < 2 && !err; pass++) {
        #pragma omp parallel reduction(| : err)
        {
            int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * ((size_t)g->n_a + 1));
            if (!mark) err |= 1;
            else {
                for (int32_t i = 0; i <= g->n_a; i++) mark[i] = -1;
                #pragma omp for schedule(dynamic, 64)
                for (int32_t u = 0; u < g->n_a; u++) {
                    int64_t k = 0, base = pass ? nb->off[u] : 0;
                    int64_t kn = nets_count(g, u);
                    for (int64_t a = 0; a < kn; a++) {
                        int32_t v = net_at(g, u, a);
                        int64_t kv = vtxs_count(g, v);
                        for (int64_t b = 0; b < kv; b++) {
                            int32_t x = vtx_at(g, v, b);
                            if (x == u || mark[x] == u) continue;
                            mark[x] = u;
                            if (pass) nb->idx[base + k] = x;
                            k++;
                        }
                    }
                    if (pass) qsort(nb->idx + base, (size_t)k, sizeof(int32_t), cmp_int);
                    else cnt[u] = k;
                }
                free(mark);
            }
        }
        if (pass == 0 && !err) {
            nb->off[0] = 0;
            for (int32_t u = 0; u < g->n_a; u++) nb->off[u + 1] = nb->off[u] + cnt[u];
            nb->idx = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nb->off[g->n_a] + 1));
            if (!nb->idx) err |= 1;
        }
    }
    free(cnt);
    if (err) { free(nb->off); free(nb->idx); nb->off = NULL; nb->idx = NULL; return -1; }
    return 0;
}

/* first-fit over F(w) = colors of the colored vertices of nbor(w) (Algorithm 2) */
static int color_vertex_round_nbor(const graph_t *g, const nbor_t *nb, const int32_t *s, int32_t *t,
                                   const int32_t *W, int64_t nw)
{
    int err = 0;
    #pragma omp parallel reduction(| : err)
    {
        fset_t F;
        if (fset_init(&F, (int64_t)g->n_a + 2)) err |= 1;
        else {
            #pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < nw; i++) {
                int32_t w = W[i];
                fset_clear(&F);
                for (int64_t k = nb->off[w]; k < nb->off[w + 1]; k++) {
                    int32_t x = nb->idx[k];
                    if (s[x] != -1 && s[x] <= g->n_a) fset_add(&F, s[x]);
                }
                int64_t col = 0;
                while (fset_has(&F, col)) col++;
                t[w] = (int32_t)col;
            }
            fset_free(&F);
        }
    }
    return err ? OR_E_INTERNAL : OR_OK;
}

/*
 * Net-based coloring (Sections III and IV).  Every net with an uncolored
 * member hands colors to its uncolored members in adjacency order
 * (distance-2: the center first, Algorithm 9); only the owner net's proposal
 * is written.  Worklist vertices without any net take the policy's color for
 * an empty F.  The variants:
 *   NET_ALG8    Algorithm 8: F = the colors of the colored members (a first
 *               pass), then reverse first-fit from |vtxs(v)| - 1 (distance-2:
 *               |nbor(v)|), each handed color joining F.
 *   NET_ALG6    Algorithm 6 (first-fit inside the net, no first pass): the
 *               members are visited once, in order; a colored member adds its
 *               color to F, an uncolored one takes the smallest color not in
 *               F at or above the previous pick, which then joins F.  A colored
 *               member whose color an earlier member was just given keeps it
 *               in this round (snapshot colors are fixed); the removal step
 *               evicts it, since the earlier member has the lower rank.
 *   NET_ALG6R   Algorithm 6 with the reverse start: the same single pass, the
 *               pick being the largest color not in F at or below the
 *               previous one, starting from |vtxs(v)| - 1.
 * With net_balance (Section V: the balancing heuristics apply to nets as to
 * vertices), Algorithm 8's first pass is kept and each uncolored member takes
 * policy_pick(F) instead of the reverse first-fit color, the net id taking
 * the place of the vertex id in B1's parity; the policy state runs through
 * `chunk` consecutive net ids (a virtual thread) and restarts every round.
 */
enum { NET_ALG8 = 0, NET_ALG6 = 1, NET_ALG6R = 2 };

static int color_net_round(const graph_t *g, const int32_t *s, int32_t *t,
                           const int32_t *owner, const int32_t *W, int64_t nw,
                           int policy, int net_alg, int net_balance, int32_t chunk,
                           int64_t snap_max, int64_t color_cap, int64_t max_size)
{
    int err = 0;
    const int32_t span = net_balance ? chunk : 1;   /* nets sharing one policy state */
    const int64_t nchunks = ((int64_t)g->n_b + span - 1) / span;
    #pragma omp parallel reduction(| : err)
    {
        fset_t F;
        int32_t *L = (int32_t *)malloc((size_t)(max_size + 1) * sizeof(int32_t));
        if (fset_init(&F, color_cap) || !L) {
            err |= 1;
        } else {
            #pragma omp for schedule(dynamic, 64)
            for (int64_t ch = 0; ch < nchunks; ch++) {
                chunk_state_t state = {policy == POL_B1G ? snap_max : 0, 0};
                const int64_t lo = ch * span;
                const int64_t hi = lo + span < g->n_b ? lo + span : g->n_b;
                for (int32_t v = (int32_t)lo; v < hi; v++) {
                    int64_t kv = vtxs_count(g, v);
                    int any_uncolored = 0;
                    for (int64_t b = 0; b < kv; b++)
                        if (s[vtx_at(g, v, b)] == -1) any_uncolored = 1;
                    if (!any_uncolored) continue;
                    fset_clear(&F);
                    if (net_alg == NET_ALG8) {
                        int64_t nl = 0;
                        for (int64_t b = 0; b < kv; b++) {
                            int32_t x = vtx_at(g, v, b);
                            if (s[x] != -1 && !fset_has(&F, s[x])) {
                                fset_add(&F, s[x]);
                            } else {
                                /* a colored x whose color is already in F would mean
                                 * two colored members of one net share a color,
                                 * which the removal step never leaves behind */
                                if (s[x] != -1) err |= 4;
                                L[nl++] = x;
                            }
                        }
                        int64_t col = kv - 1;   /* |vtxs(v)| - 1; distance-2: |nbor(v)| */
                        for (int64_t i = 0; i < nl; i++) {
                            if (net_balance) {
                                col = policy_pick(policy, &F, &state, v);
                            } else {
                                col = free_at_or_below(&F, col);
                                if (col < 0) err |= 8;
                            }
                            if (col + 1 >= color_cap) { err |= 2; break; }
                            if (owner[L[i]] == v) t[L[i]] = (int32_t)col;
                            fset_add(&F, col);
                        }
                    } else {
                        const int forward = net_alg == NET_ALG6;
                        int64_t col = forward ? 0 : kv - 1;
                        for (int64_t b = 0; b < kv; b++) {
                            int32_t x = vtx_at(g, v, b);
                            if (s[x] != -1) {
                                fset_add(&F, s[x]);
                                continue;
                            }
                            col = forward ? free_at_or_above(&F, col) : free_at_or_below(&F, col);
                            if (col < 0) err |= 8;
                            if (col < 0 || col + 1 >= color_cap) { err |= 2; break; }
                            if (owner[x] == v) t[x] = (int32_t)col;
                            fset_add(&F, col);
                        }
                    }
                }
            }
            #pragma omp for schedule(static)
            for (int64_t i = 0; i < nw; i++) {
                int32_t w = W[i];
                if (owner[w] == -1) {
                    const fset_t empty = {NULL, NULL, 0, 0};
                    chunk_state_t st = {0, 0};
                    t[w] = (int32_t)policy_pick(policy, &empty, &st, w);
                }
            }
            fset_free(&F);
        }
        free(L);
    }
    return err ? OR_E_INTERNAL : OR_OK;
}

/*
 * Removal: u loses iff t[u] != -1 and a vertex x sharing a net with u has
 * t[x] == t[u] and x < u (the lower rank keeps its color, Algorithm 3's
 * rule, applied to every colored vertex).  Per net, the lowest-ranked holder
 * of each color is found first; every other holder of that color loses.
 */
static int remove_conflicts(const graph_t *g, const int32_t *t, uint8_t *lose, int64_t color_cap)
{
    int err = 0;
    memset(lose, 0, (size_t)g->n_a);
    #pragma omp parallel reduction(| : err)
    {
        fset_t F;
        if (fset_init(&F, color_cap)) {
            err |= 1;
        } else {
            #pragma omp for schedule(dynamic, 256)
            for (int32_t v = 0; v < g->n_b; v++) {
                int64_t kv = vtxs_count(g, v);
                fset_clear(&F);
                for (int64_t b = 0; b < kv; b++) {
                    int32_t x = vtx_at(g, v, b);
                    int32_t col = t[x];
                    if (col == -1) continue;
                    if (!fset_has(&F, col) || x < F.holder[col]) {
                        fset_add(&F, col);
                        F.holder[col] = x;
                    }
                }
                for (int64_t b = 0; b < kv; b++) {
                    int32_t x = vtx_at(g, v, b);
                    int32_t col = t[x];
                    if (col != -1 && F.holder[col] != x) {
                        #pragma omp atomic write
                        lose[x] = 1;
                    }
                }
            }
            fset_free(&F);
        }
    }
    return err ? OR_E_INTERNAL : OR_OK;
}

/*
 * Removal in the vertex form (Algorithm 5 with Algorithm 3's test): only the
 * worklist is checked; w loses iff a vertex x sharing a net with w has
 * t[x] == t[w] and x < w.  Equal to the net form whenever every vertex that
 * was colored before the round keeps a color no worklist vertex proposes:
 * after a vertex-based round (a proposal avoids every colored neighbour's
 * color) and after a net-based round that started with nothing colored.
 */
static int remove_conflicts_vertex(const graph_t *g, const int32_t *t, const int32_t *W, int64_t nw,
                                   uint8_t *lose)
{
    memset(lose, 0, (size_t)g->n_a);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nw; i++) {
        int32_t w = W[i];
        if (t[w] == -1) continue;
        int lost = 0;
        int64_t kn = nets_count(g, w);
        for (int64_t a = 0; a < kn && !lost; a++) {
            int32_t v = net_at(g, w, a);
            int64_t kv = vtxs_count(g, v);
            for (int64_t b = 0; b < kv && !lost; b++) {
                int32_t x = vtx_at(g, v, b);
                if (x < w && t[x] == t[w]) lost = 1;
            }
        }
        lose[w] = (uint8_t)lost;
    }
    return OR_OK;
}

/* FNV-1a, 64-bit, over the little-endian bytes of a[0..n) */
static uint64_t fnv1a_i32(const int32_t *a, int64_t n)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (int64_t i = 0; i < n; i++) {
        uint32_t v = (uint32_t)a[i];
        for (int k = 0; k < 4; k++) {
            h ^= (v >> (8 * k)) & 0xffu;
            h *= 0x100000001b3ull;
        }
    }
    return h;
}

/*
 * The speculative loop of Algorithm 1 on V_color = V_A.
 *   colors     in: starting coloring (all -1, or a conflict-free partial one
 *              to resume from); out: the coloring reached.
 *   start_round  index of the first round (selects the net_color_mask bit).
 *   literal_ff   first-fit rounds gather F(w) member by member (Algorithm 4
 *              as printed) instead of through the per-net color sets.
 *   max_rounds   rounds to run at most (0: n_a + 65); status -6 when the
 *              worklist is still non-empty after them.
 *   net_alg    net-based rounds: NET_ALG8, NET_ALG6 or NET_ALG6R (see
 *              color_net_round); net_balance: net-based rounds choose by the
 *              policy (Algorithm 8's first pass, then policy_pick per member).
 *   vertex_removal_mask  bit r (r < 64; rounds past 63 follow bit 63): round
 *              r checks conflicts in the vertex form, when that form is exact
 *              (a vertex-based round, or a net-based round that started with
 *              nothing colored); otherwise, and for clear bits, the net form.
 *   log_*      optional per-round records (mode, |W_r|, losers, evicted
 *              colored vertices, max color after the round, FNV-1a-64 of the
 *              tentative colors t after the coloring step and of the colors
 *              after the round), log_cap entries.
 */
int oracle_color(int32_t n_a, int32_t n_b,
                 const int64_t *a_off, const int32_t *a_idx,
                 const int64_t *b_off, const int32_t *b_idx,
                 int32_t d2, uint64_t net_color_mask, int32_t policy, int32_t chunk,
                 int32_t max_rounds, int32_t start_round, int32_t literal_ff,
                 int32_t net_alg, int32_t net_balance, uint64_t vertex_removal_mask,
                 int32_t *colors, int32_t *rounds_out,
                 int32_t log_cap, int32_t *log_mode, int64_t *log_w, int64_t *log_losers,
                 int64_t *log_evicted, int32_t *log_maxc, uint64_t *log_hash_t, uint64_t *log_hash_c)
{
    if (n_a < 0 || n_b < 0 || chunk <= 0 || policy < 0 || policy > 3) return OR_E_INVALID;
    if (net_alg < NET_ALG8 || net_alg > NET_ALG6R || (net_balance && net_alg != NET_ALG8)) return OR_E_INVALID;
    if (d2 && n_a != n_b) return OR_E_INVALID;
    graph_t g = {n_a, n_b, d2, a_off, a_idx, b_off, b_idx};
    if (max_rounds <= 0) max_rounds = n_a + 65;

    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_a + 1));
    int32_t *t = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_a + 1));
    int32_t *W = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_a + 1));
    int32_t *owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_a + 1));
    uint8_t *lose = (uint8_t *)malloc((size_t)(n_a + 1));
    nbor_t nb = {NULL, NULL};
    int status = OR_OK;
    if (!s || !t || !W || !owner || !lose) { status = OR_E_INTERNAL; goto done; }

    compute_owner(&g, owner);
    int64_t max_size = max_net_size(&g);
    /* dense graphs: walking nets would revisit the same vertices many times;
     * use explicit neighbour lists (at most n_a^2 entries) for first-fit */
    if (policy == POL_FF && !literal_ff && (int64_t)n_a * n_a <= (int64_t)1 << 28) {
        double walk = 0.0;
        for (int32_t v = 0; v < n_b; v++) {
            double k = (double)vtxs_count(&g, v);
            walk += k * k;
        }
        if (walk > 4.0 * (double)n_a * (double)n_a && build_nbor(&g, &nb)) {
            status = OR_E_INTERNAL;
            goto done;
        }
    }
    int32_t r = 0;
    for (;;) {
        /* snapshot and worklist of the uncolored vertices, ascending rank */
        memcpy(s, colors, sizeof(int32_t) * (size_t)n_a);
        int64_t nw = 0, maxc = -1;
        for (int32_t u = 0; u < n_a; u++) {
            if (s[u] == -1) W[nw++] = u;
            else if (s[u] > maxc) maxc = s[u];
        }
        if (nw == 0) break;
        if (r >= max_rounds) { status = OR_E_NOT_CONVERGED; break; }
        int32_t round_id = start_round + r;
        int net_mode = round_id < 64 && ((net_color_mask >> round_id) & 1u);
        /* every color a round can produce stays below this bound */
        int64_t cap = maxc + 2 + (int64_t)chunk + 2;
        if (max_size + 2 > cap) cap = max_size + 2;
        /* balanced net rounds: a pick exceeds the chunk's col_max by at most the
         * net's size, and col_max starts at 0 (B1G: the snapshot's largest color) */
        if (net_mode && net_balance) cap = (maxc > 0 ? maxc : 0) + (int64_t)chunk * (max_size + 1) + 4;

        memcpy(t, s, sizeof(int32_t) * (size_t)n_a);
        int e;
        if (net_mode) e = color_net_round(&g, s, t, owner, W, nw, policy, net_alg, net_balance, chunk, maxc, cap,
                                          max_size);
        else if (policy == POL_FF && !literal_ff && nb.off) e = color_vertex_round_nbor(&g, &nb, s, t, W, nw);
        else if (policy == POL_FF && !literal_ff) e = color_vertex_round_sets(&g, s, t, W, nw);
        else e = color_vertex_round(&g, s, t, W, nw, policy, chunk, cap);
        if (e) { status = e; break; }
        if (r < log_cap && log_hash_t) log_hash_t[r] = fnv1a_i32(t, n_a);
        int64_t tmax = -1;
        for (int32_t u = 0; u < n_a; u++)
            if (t[u] > tmax) tmax = t[u];
        if (tmax + 2 > cap) cap = tmax + 2;
        const int vbit = round_id < 64 ? round_id : 63;
        const int vertex_form = ((vertex_removal_mask >> vbit) & 1u) && (!net_mode || maxc < 0);
        if (vertex_form) e = remove_conflicts_vertex(&g, t, W, nw, lose);
        else e = remove_conflicts(&g, t, lose, cap);
        if (e) { status = e; break; }
        int64_t losers = 0, evicted = 0, nmax = -1;
        for (int32_t u = 0; u < n_a; u++) {
            if (lose[u]) {
                losers++;
                if (s[u] != -1) evicted++;
                colors[u] = -1;
            } else {
                colors[u] = t[u];
                if (t[u] > nmax) nmax = t[u];
            }
        }
        if (r < log_cap) {
            if (log_mode) log_mode[r] = net_mode;
            if (log_w) log_w[r] = nw;
            if (log_losers) log_losers[r] = losers;
            if (log_evicted) log_evicted[r] = evicted;
            if (log_maxc) log_maxc[r] = (int32_t)nmax;
            if (log_hash_c) log_hash_c[r] = fnv1a_i32(colors, n_a);
        }
        r++;
    }
    if (rounds_out) *rounds_out = r;
done:
    free(s); free(t); free(W); free(owner); free(lose);
    free(nb.off); free(nb.idx);
    return status;
}

/*
 * Sequential greedy coloring: vertices in rank order, each taking the
 * smallest color not used by an already colored vertex sharing a net with it
 * (the sequential V-V of the experiments, which needs no conflict phase).
 */
int oracle_seq_greedy(int32_t n_a, int32_t n_b,
                      const int64_t *a_off, const int32_t *a_idx,
                      const int64_t *b_off, const int32_t *b_idx,
                      int32_t d2, int32_t *colors)
{
    graph_t g = {n_a, n_b, d2, a_off, a_idx, b_off, b_idx};
    fset_t F;
    if (fset_init(&F, (int64_t)n_a + 2)) return OR_E_INTERNAL;
    for (int32_t u = 0; u < n_a; u++) colors[u] = -1;
    for (int32_t u = 0; u < n_a; u++) {
        fset_clear(&F);
        int64_t kn = nets_count(&g, u);
        for (int64_t a = 0; a < kn; a++) {
            int32_t v = net_at(&g, u, a);
            int64_t kv = vtxs_count(&g, v);
            for (int64_t b = 0; b < kv; b++) {
                int32_t x = vtx_at(&g, v, b);
                if (x != u && colors[x] != -1) fset_add(&F, colors[x]);
            }
        }
        int64_t col = 0;
        while (fset_has(&F, col)) col++;
        colors[u] = (int32_t)col;
    }
    fset_free(&F);
    return OR_OK;
}

/* Number of (net, pair) violations: two members of one net with one color, or
 * a member left uncolored (counted once per member). */
int64_t oracle_count_violations(int32_t n_a, int32_t n_b,
                                const int64_t *b_off, const int32_t *b_idx,
                                int32_t d2, const int32_t *colors)
{
    graph_t g = {n_a, n_b, d2, NULL, NULL, b_off, b_idx};
    int64_t bad = 0;
    int64_t cap = 2;
    for (int32_t u = 0; u < n_a; u++) {
        if (colors[u] < 0) bad++;
        else if (colors[u] + 2 > cap) cap = colors[u] + 2;
    }
    #pragma omp parallel reduction(+ : bad)
    {
        fset_t F;
        if (fset_init(&F, cap) == 0) {
            #pragma omp for schedule(dynamic, 256)
            for (int32_t v = 0; v < n_b; v++) {
                fset_clear(&F);
                int64_t kv = vtxs_count(&g, v);
                for (int64_t b = 0; b < kv; b++) {
                    int32_t col = colors[vtx_at(&g, v, b)];
                    if (col < 0) continue;
                    if (fset_has(&F, col)) bad++;
                    else fset_add(&F, col);
                }
            }
            fset_free(&F);
        } else {
            bad += 1;
        }
    }
    return bad;
}

/*
 * Color-set statistics (the quantities of the balancing experiments): the
 * number of non-empty color sets, the largest color, the min / max / mean /
 * population standard deviation of the non-empty set cardinalities, and the
 * number of empty sets below the largest color.  Uncolored entries are
 * ignored.
 */
int oracle_color_stats(const int32_t *colors, int64_t n, int64_t *out_i, double *out_d)
{
    int64_t maxc = -1;
    for (int64_t i = 0; i < n; i++)
        if (colors[i] > maxc) maxc = colors[i];
    int64_t *card = (int64_t *)calloc((size_t)(maxc + 2), sizeof(int64_t));
    if (!card) return OR_E_INTERNAL;
    for (int64_t i = 0; i < n; i++)
        if (colors[i] >= 0) card[colors[i]]++;
    int64_t ndist = 0, cmin = 0, cmax = 0, total = 0;
    for (int64_t c = 0; c <= maxc; c++) {
        if (card[c] == 0) continue;
        if (ndist == 0 || card[c] < cmin) cmin = card[c];
        if (card[c] > cmax) cmax = card[c];
        ndist++;
        total += card[c];
    }
    double mean = ndist ? (double)total / (double)ndist : 0.0;
    double var = 0.0;
    for (int64_t c = 0; c <= maxc; c++) {
        if (card[c] == 0) continue;
        double d = (double)card[c] - mean;
        var += d * d;
    }
    var = ndist ? var / (double)ndist : 0.0;
    double sd = sqrt(var);
    out_i[0] = ndist;
    out_i[1] = maxc;
    out_i[2] = cmin;
    out_i[3] = cmax;
    out_i[4] = (maxc + 1) - ndist;
    out_d[0] = mean;
    out_d[1] = sd;
    free(card);
    return OR_OK;
}

/*
 * Smallest-last processing orders (Section VI compares the natural order with
 * ColPack's smallest-last order).  The degree of a vertex u is counted as in
 * the largest-first order: key(u) = the number of (net, other member) pairs
 * of u among the vertices not yet removed, sum over v in nets(u) of
 * (|vtxs(v) still present| - 1), an upper bound of its distance-2 degree
 * (distance-2: the nets are the closed neighbourhoods).  Vertices are removed
 * smallest key first; the processing order is the reverse of the removal
 * sequence (the last vertex removed gets rank 0).
 *   batched = 0  one vertex per step: the smallest key, ties to the lowest id
 *                (ColPack's peeling with a fixed tie rule; cost quadratic in
 *                |V_A|, for small graphs)
 *   batched = 1  every vertex whose key equals the current minimum is removed
 *                in the same step; a step's vertices take consecutive ranks in
 *                ascending id, steps in reverse order of removal (the form
 *                the device computes in parallel)
 * order_out[k] = the vertex of rank k.  Returns the number of steps.
 */
int64_t oracle_order_smallest_last(int32_t n_a, int32_t n_b, const int64_t *a_off, const int32_t *a_idx,
                                   const int64_t *b_off, const int32_t *b_idx, int32_t d2, int32_t batched,
                                   int32_t slack_shift, int32_t *order_out)
{
    graph_t g = {n_a, n_b, d2, a_off, a_idx, b_off, b_idx};
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n_a + 1));
    uint8_t *gone = (uint8_t *)calloc((size_t)n_a + 1, 1);
    int32_t *seq = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n_a + 1));   /* removal sequence */
    int64_t *step_end = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n_a + 1));
    int32_t *batch = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n_a + 1));
    if (!key || !gone || !seq || !step_end || !batch) {
        free(key); free(gone); free(seq); free(step_end); free(batch);
        return -1;
    }
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t u = 0; u < n_a; u++) {
        int64_t k = 0, kn = nets_count(&g, u);
        for (int64_t a = 0; a < kn; a++) k += vtxs_count(&g, net_at(&g, u, a)) - 1;
        key[u] = k;
    }
    int64_t removed = 0, steps = 0;
    while (removed < n_a) {
        int64_t d = INT64_MAX;
        int32_t first = -1;
        for (int32_t u = 0; u < n_a; u++)
            if (!gone[u] && key[u] < d) { d = key[u]; first = u; }
        int64_t nb = 0;
        if (batched) {
            const int64_t thr = slack_shift >= 63 ? d : d + (d >> slack_shift);
            for (int32_t u = 0; u < n_a; u++)
                if (!gone[u] && key[u] <= thr) batch[nb++] = u;
        } else {
            batch[nb++] = first;
        }
        for (int64_t i = 0; i < nb; i++) {
            gone[batch[i]] = 1;
            seq[removed + i] = batch[i];
        }
        /* every (net, removed member) pair leaves the keys of the members
         * still present */
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < nb; i++) {
            int32_t u = batch[i];
            int64_t kn = nets_count(&g, u);
            for (int64_t a = 0; a < kn; a++) {
                int32_t v = net_at(&g, u, a);
                int64_t kv = vtxs_count(&g, v);
                for (int64_t b = 0; b < kv; b++) {
                    int32_t x = vtx_at(&g, v, b);
                    if (!gone[x]) {
                        #pragma omp atomic
                        key[x] -= 1;
                    }
                }
            }
        }
        removed += nb;
        step_end[steps++] = removed;
    }
    /* ranks: steps in reverse, each step's vertices in ascending id (a step's
     * vertices were collected in ascending id) */
    int64_t k = 0;
    for (int64_t st = steps - 1; st >= 0; st--) {
        int64_t lo = st ? step_end[st - 1] : 0, hi = step_end[st];
        for (int64_t i = lo; i < hi; i++) order_out[k++] = seq[i];
    }
    free(key); free(gone); free(seq); free(step_end); free(batch);
    return steps;
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

/* threads of the parallel loops from now on (the CPU-baseline timings) */
void oracle_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}
