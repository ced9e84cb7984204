/*
 * bgpc.h -- C ABI of the MI355X (gfx950) speculative greedy coloring library.
 *
 * Method: Tas, Kaya and Saule, "Greed is Good: Optimistic Algorithms for
 * Bipartite-Graph Partial Coloring on Multicore Architectures" (2017).
 *
 * Problem (Section II): given a bipartite graph G = (V_A u V_B, E), give every
 * vertex of V_A a non-negative color so that two vertices adjacent to a common
 * V_B vertex ("net") differ.  -1 marks an uncolored vertex.  Distance-2
 * coloring (Section IV) colors every vertex of a symmetric graph differently
 * from all vertices within distance two; the library runs it as the bipartite
 * problem whose nets are the closed neighbourhoods N[v] = {v} u nbor(v).
 *
 * The colors come from the speculative loop of Algorithm 1 with fixed round
 * semantics so that the result of every round is unique:
 *   - a round reads the colors left by the previous round (a snapshot) and
 *     proposes tentative colors for the uncolored vertices, in rank order;
 *   - a vertex loses its tentative or current color iff a vertex sharing a
 *     net with it holds the same color and has a lower rank (Algorithm 3's
 *     rule); losers become uncolored and form the next round's worklist;
 *   - vertex-based rounds choose by first-fit (Algorithms 2 and 4) or by the
 *     balancing policies B1 / B2 (Algorithms 11 and 12), whose state restarts
 *     every `chunk` consecutive worklist entries (or by B1 with one bound for
 *     the whole round, BGPC_B1_GLOBAL);
 *   - net-based rounds (Algorithms 8 and 9) run reverse first-fit inside each
 *     net holding an uncolored vertex, starting at |vtxs(v)| - 1; a vertex
 *     takes the proposal of its owner net only: the largest net containing
 *     it, ties to the lowest net id.  Net-based rounds run where bit r of
 *     net_color_mask is set; every other round is vertex-based.
 * Ranks are vertex ids, or positions in `order` when one is given.
 *
 * Conventions for every entry point:
 *   - graph arrays and colors_out are DEVICE pointers (hipMalloc / torch
 *     tensors on the GPU); option, log and stats structs are host memory;
 *   - the caller owns every buffer it passes; inputs are never modified;
 *   - the library allocates its own stream-ordered workspace per call and
 *     releases it before returning;
 *   - calls are ordered on opts->stream (NULL: the default stream) and return
 *     after the result is complete;
 *   - a negative return value is a bgpc_status error; colors_out is then
 *     undefined, except for BGPC_E_NOT_CONVERGED, where it holds the state
 *     reached after max_rounds rounds (uncolored vertices are -1).
 *   - calls on distinct streams may run concurrently from distinct threads.
 */
#ifndef BGPC_H
#define BGPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BGPC_API __attribute__((visibility("default")))

typedef enum {
    BGPC_OK = 0,
    BGPC_E_INVALID = -1,         /* bad sizes, NULL pointers, bad option values */
    BGPC_E_UNSORTED = -2,        /* (BGPC_STRICT) a member list not strictly ascending */
    BGPC_E_NOT_TRANSPOSE = -3,   /* (BGPC_STRICT) csr_A is not the transpose of csr_B */
    BGPC_E_NOT_SYMMETRIC = -4,   /* (BGPC_STRICT) adjacency not symmetric, or a self loop */
    BGPC_E_OOM = -5,             /* device workspace allocation failed */
    BGPC_E_NOT_CONVERGED = -6,   /* worklist non-empty after max_rounds rounds */
    BGPC_E_HIP = -7,             /* a HIP runtime call failed */
    BGPC_E_UNSUPPORTED = -8,     /* a size beyond the library's limits (see below) */
    BGPC_E_INTERNAL = -9         /* a device-side invariant check failed */
} bgpc_status;

/*
 * Compressed sparse rows.  offsets[n_rows + 1] and indices[nnz] are device
 * arrays of int32; row i lists its columns in indices[offsets[i] ..
 * offsets[i + 1]), strictly ascending.  nnz must equal offsets[n_rows].
 */
typedef struct {
    int32_t n_rows;
    int32_t n_cols;
    int64_t nnz;
    const int32_t *offsets;
    const int32_t *indices;
} bgpc_csr;

/* color policies of vertex-based rounds */
enum {
    BGPC_FIRST_FIT = 0,   /* Algorithm 2: smallest color not forbidden */
    BGPC_B1 = 1,          /* Algorithm 11: alternate reverse / forward search around col_max */
    BGPC_B2 = 2,          /* Algorithm 12: forward search from col_next, capped at col_max / 3 + 1 */
    BGPC_B1_GLOBAL = 3    /* Algorithm 11's choice with col_max fixed for the whole round to the
                             largest color of the round's snapshot (-1 before any color): no state
                             passes between vertices, so `chunk` does not matter */
};

/* opts->flags */
enum {
    BGPC_STRICT = 1u,      /* validate sortedness, transpose / symmetry before coloring */
    BGPC_RESUME = 2u,      /* colors_out holds a conflict-free partial coloring to continue from */
    BGPC_INCREMENTAL = 4u, /* first-fit vertex rounds recompute only the vertices whose neighbourhood
                              changed (same results; pays off when few proposals change per round) */
    BGPC_NET_BALANCE = 8u  /* net-based rounds choose by opts->policy (Section V: the balancing
                              heuristics "are also similar" for nets): Algorithm 8's first pass
                              gathers F from the colored members, then every uncolored member in
                              adjacency order takes the policy's pick from F (B1's parity is the
                              net id's), each pick joining F; the policy state runs through `chunk`
                              consecutive net ids and restarts every round.  Requires
                              net_alg == BGPC_NET_ALG8.  Colors of such rounds can exceed the
                              largest net; BGPC_E_UNSUPPORTED when a net's picks pass the LDS
                              bitmap (about 440,000 colors) */
};

/* net-based coloring variants (opts->net_alg), Section III */
enum {
    BGPC_NET_ALG8 = 0,          /* Algorithm 8: first pass over the net gathers the colored members'
                                   colors, then reverse first-fit from |vtxs(v)| - 1 (distance-2:
                                   |nbor(v)|, Algorithm 9) for the uncolored members */
    BGPC_NET_ALG6 = 1,          /* Algorithm 6: one pass in adjacency order; a colored member adds its
                                   color to F, an uncolored one takes the smallest color at or above
                                   the previous pick not in F.  A colored member whose color an earlier
                                   member was just given keeps it this round (snapshot colors) and is
                                   evicted by the removal step (the earlier member ranks lower) */
    BGPC_NET_ALG6_REVERSE = 2   /* Algorithm 6 with the reverse start: the same single pass, picks
                                   going down from |vtxs(v)| - 1 */
};

/*
 * Optional per-round record, host arrays of `cap` entries each (any may be
 * NULL).  Round r (counted from the call's first round) stores: mode (0
 * vertex-based, 1 net-based), |W_r| (vertices the round started uncolored),
 * the losers of its removal step, how many of them were colored before the
 * round ("evicted"; only net-based rounds after the first can evict), and the
 * largest color present after the round.  `n` receives the rounds recorded.
 * hash_t / hash_c: FNV-1a-64 over the little-endian bytes of the int32 array
 * of tentative colors t (every vertex's color after the round's coloring
 * step: its proposal, its color, or -1) and of the colors after the round,
 * both indexed by rank; asking for either makes every round wait for the host
 * (diagnostics, not for timing).  round_ms: device time of each round,
 * from HIP events recorded between rounds on opts->stream.
 */
typedef struct {
    int32_t cap;
    int32_t n;
    int32_t *mode;
    int64_t *w_size;
    int64_t *losers;
    int64_t *evicted;
    int32_t *max_color;
    uint64_t *hash_t;
    uint64_t *hash_c;
    float *round_ms;
} bgpc_round_log;

/*
 * Optional kernel timing: when opts->prof is set, the driver records a HIP
 * event pair on opts->stream around every launch of the kernel named by
 * `kernel` and returns the summed event time, the number of launches and the
 * algorithmic bytes those launches had to move, compulsory streams only,
 * never cache re-reads.  Removal (net form, Algorithm 7): per net of the
 * round -- a net with a member uncolored or proposing -- 8 bytes (its two
 * offsets) plus 8 per member (its id and its state).  Coloring: per worklist
 * entry 16 bytes (id, two row offsets, proposal), 4 per incidence (net id),
 * 8 per distinct net mask.
 */
enum {
    BGPC_PROF_CONFLICT = 0,   /* net-side removal scan of small nets */
    BGPC_PROF_COLOR = 1       /* vertex-based first-fit coloring of the worklist */
};

typedef struct {
    int32_t kernel;           /* BGPC_PROF_* */
    int32_t launches;         /* out */
    double ms;                /* out: summed event time of those launches */
    double bytes;             /* out: summed algorithmic bytes of those launches */
    double bytes_scanned;     /* out: the same figure over the nets the removal scan actually read
                                 (vertex-based rounds re-scan only nets whose members changed their
                                 proposals; equal to bytes for the coloring kernel) */
    double bytes_states;      /* out: removal counted with one offset and the member ids per net and
                                 every member state read once per round (at most |V_A| states);
                                 equal to bytes for the coloring kernel */
} bgpc_profile;

/*
 * Launch and data-structure choices of bgpc_color / d2gc_color that do not
 * change any result (every value gives the same colors and rounds): picked
 * by the library from the graph's shape, by bgpc_autotune, or by the caller.
 * -1 (0 for the grids): the library's choice.
 */
typedef struct {
    int32_t front;         /* front-driven first-fit rounds (only vertices whose nets hold color 0 are
                              recolored; removal over the nets whose members changed; winners from the
                              vertices whose loss count dropped to 0): 0 off, 1 on where the schedule
                              allows it (vertex-based first-fit, nets of at most 64 members, needs
                              standing proposals) */
    int32_t standing;      /* standing proposals in vertex-based rounds (a loser keeps its proposal and
                              only nets with a changed member are scanned again): 0 off, 1 on */
    int32_t planes;        /* per-net 64-bit color words past color 63: 0 off (per-vertex LDS bitmaps
                              from the distance-2 walk), 1 on */
    int32_t color_grid;    /* workgroups per CU of the first-fit launch (a wave each) */
    int32_t removal_grid;  /* workgroups per CU of the removal launches */
    int32_t apply_grid;    /* workgroups per CU of the apply / compaction launches */
} bgpc_tuning;

typedef struct {
    uint64_t net_color_mask;  /* bit r (r < 64): round r is net-based */
    int32_t policy;           /* BGPC_FIRST_FIT, BGPC_B1 or BGPC_B2 */
    int32_t chunk;            /* worklist entries per balancing state, >= 1 (default 64) */
    int32_t max_rounds;       /* rounds to run at most; 0: n + 65 */
    int32_t start_round;      /* index of the first round (selects mask bits); with BGPC_RESUME */
    uint32_t flags;           /* BGPC_STRICT | BGPC_RESUME | BGPC_INCREMENTAL */
    int32_t reserved;
    void *stream;             /* hipStream_t; NULL = default stream */
    bgpc_round_log *log;      /* optional */
    int32_t *rounds_out;      /* optional, host: rounds run */
    bgpc_profile *prof;       /* optional kernel timing */
    uint64_t net_conflict_mask;  /* bit r (r < 64; later rounds follow bit 63) set: round r finds its
                                    losers net by net (Algorithm 7's form); clear: vertex by vertex
                                    over the worklist (Algorithm 5's form: each worklist vertex walks
                                    its distance-2 neighbourhood for a lower-ranked holder of its
                                    color).  Speed only: both forms give the same losers wherever the
                                    vertex form is used, which is a vertex-based round or a net-based
                                    first round without BGPC_RESUME; elsewhere the net form runs
                                    whatever the bit.  Default all ones */
    int32_t net_alg;          /* BGPC_NET_ALG8 (default), BGPC_NET_ALG6, BGPC_NET_ALG6_REVERSE */
    int32_t reserved2;
    const bgpc_tuning *tuning;  /* NULL: the choices bgpc_autotune cached for graphs of this shape, else the
                                   library's rules */
} bgpc_opts;

/* Fills *opts with the defaults: vertex-based first-fit rounds, chunk 64,
 * net-side removal, Algorithm 8 in net-based rounds. */
BGPC_API void bgpc_opts_default(bgpc_opts *opts);

/*
 * Bipartite-graph partial coloring of V_A (Sections II-III, V).
 *   csr_A    vertices -> nets: n_rows = |V_A|, n_cols = |V_B| (nets(u))
 *   csr_B    nets -> vertices: n_rows = |V_B|, n_cols = |V_A| (vtxs(v)),
 *            the transpose of csr_A
 *   order    NULL for the natural order, else a device int32[|V_A|]
 *            permutation: order[k] is the vertex of rank k (Section II:
 *            the order in which vertices are visited).  The library copies
 *            the graph relabelled to ranks into its own workspace (about
 *            4 |V_A| + 3 nnz int32 more) and maps the colors back; the
 *            caller's arrays are not modified.  BGPC_E_INVALID when it is
 *            not a permutation of [0, |V_A|)
 *   colors_out  device int32[|V_A|], indexed by vertex id; with
 *            BGPC_RESUME it is read first
 * Limits: |V_A|, |V_B| < 2^30; nnz < 2^31; when net-based rounds run, no
 * net above 220,000 vertices; colors below 440,000 (BGPC_E_UNSUPPORTED).
 */
BGPC_API int bgpc_color(const bgpc_csr *csr_A, const bgpc_csr *csr_B, const int32_t *order,
                        const bgpc_opts *opts, int32_t *colors_out);

/*
 * Distance-2 coloring (Section IV) of a symmetric graph without self loops:
 * adj is its CSR (n_rows = n_cols = n).  Nets are the closed neighbourhoods;
 * in net-based rounds the center of N[v] is queued before nbor(v)
 * (Algorithm 9) and colors start at |nbor(v)|.
 * `order` as for bgpc_color (a permutation of the n vertices).
 */
BGPC_API int d2gc_color(const bgpc_csr *adj, const int32_t *order, const bgpc_opts *opts,
                        int32_t *colors_out);

/*
 * Autotuner: times bgpc_color (csr_B non-NULL) or d2gc_color (csr_B NULL: the
 * symmetric adjacency csr_A) on the caller's graph under `opts` for each
 * candidate choice of bgpc_tuning, one field at a time (coordinate descent
 * from the library's choices; front, standing, planes, then the three grids),
 * keeping a candidate only when it is faster over `trials` calls (the
 * fastest of them).  Every candidate's colors and rounds must equal the
 * library's default choices' (else BGPC_E_INTERNAL: a tuning changed a
 * result).  The best choice is written to *best and cached for graphs of the
 * same shape (distance-2 or not, schedule and policy class, log2 of |V_A|,
 * |V_B| and nnz / |V_A|): later calls whose opts->tuning is NULL use it.
 * Allocates two color arrays; colors_scratch may be NULL.  *ms_default and
 * *ms_best (optional) receive the default and the tuned call times.
 */
BGPC_API int bgpc_autotune(const bgpc_csr *csr_A, const bgpc_csr *csr_B, const bgpc_opts *opts, int32_t trials,
                           bgpc_tuning *best, double *ms_default, double *ms_best);

/*
 * Largest-first processing order (the paper's experiments compare processing
 * orders, Section VI; this is the cheap degree-based one, computed on the
 * device): vertices by decreasing key(u) = sum over the nets v of u of
 * (|vtxs(v)| - 1) -- the number of (net, other member) pairs of u, an upper
 * bound of its distance-2 degree -- ties by increasing id.  For distance-2
 * coloring the nets are the closed neighbourhoods: key(u) = sum over x in
 * N[u] of |nbor(x)|.
 *   csr_A, csr_B / adj  as for bgpc_color / d2gc_color (trusted: no
 *                       validation beyond the sizes)
 *   stream              hipStream_t or NULL; the call returns once the order
 *                       is complete
 *   order_out           device int32[|V_A|] (resp. [n]), written with the
 *                       vertex of each rank; pass it as `order` above
 * Allocates its own workspace (two uint64 and one int32 per vertex plus the
 * sort's scratch).  BGPC_E_INVALID for inconsistent sizes or a NULL output.
 */
BGPC_API int bgpc_order_largest_first(const bgpc_csr *csr_A, const bgpc_csr *csr_B, void *stream,
                                      int32_t *order_out);
BGPC_API int d2gc_order_largest_first(const bgpc_csr *adj, void *stream, int32_t *order_out);

/*
 * Smallest-last processing order (Section VI compares the natural order with
 * ColPack's smallest-last order), computed on the device by removal steps:
 * with key(u) = the number of (net, other member) pairs of u among the
 * vertices still present (the largest-first key, recounted as vertices
 * leave; distance-2: over the closed neighbourhoods), each step removes every
 * present vertex whose key is at most d + (d >> slack_shift), d the smallest
 * key present (slack_shift >= 63: exactly the vertices at d).  Ranks run
 * over the steps in reverse (the last step's vertices first), a step's
 * vertices in ascending id.  The one-vertex-at-a-time peeling of ColPack is
 * sequential; the steps trade its tie order for parallel removal, and a
 * slack of 1/8 (slack_shift 3) keeps the steps to a few hundred on the
 * workloads measured (an exact minimum takes thousands to tens of thousands).
 *   csr_A, csr_B / adj  as for bgpc_color / d2gc_color (trusted)
 *   stream              hipStream_t or NULL; returns once the order is done
 *   order_out           device int32[|V_A|] (resp. [n]): the vertex of each rank
 *   steps_out           optional host int32: removal steps taken
 * Allocates its own workspace (two uint64 and five int32 per vertex, one
 * int32 per net, the selection scratch); every step waits for the host once.
 * BGPC_E_INVALID for inconsistent sizes, a NULL output or slack_shift < 0.
 */
BGPC_API int bgpc_order_smallest_last(const bgpc_csr *csr_A, const bgpc_csr *csr_B, int32_t slack_shift,
                                      void *stream, int32_t *order_out, int32_t *steps_out);
BGPC_API int d2gc_order_smallest_last(const bgpc_csr *adj, int32_t slack_shift, void *stream, int32_t *order_out,
                                      int32_t *steps_out);

/*
 * Color-set statistics of a coloring (the metrics of the balancing
 * experiments, Section VI): non-empty color sets, largest color, min / max /
 * mean / population standard deviation of the non-empty set cardinalities,
 * empty sets below the largest color.  Entries < 0 are ignored.
 * colors: device int32[n]; stream: hipStream_t or NULL.
 */
typedef struct {
    int64_t n_distinct;
    int64_t max_color;
    int64_t card_min;
    int64_t card_max;
    int64_t n_empty_below_max;
    double card_mean;
    double card_std;
} bgpc_stats;

BGPC_API int color_stats(const int32_t *colors, int64_t n, void *stream, bgpc_stats *out);

/*
 * Batched coloring: many independent graphs.  Every graph's colors and rounds
 * equal what bgpc_color (d2gc_color for d2gc items) returns for it alone with
 * the same options and order.  Items with the default options (vertex-based
 * first-fit rounds, flags 0 or BGPC_STRICT), no order and no d2gc share the
 * persistent launch described next; every other item, and every item when
 * opts asks for anything else (net-based rounds, a balancing policy,
 * BGPC_RESUME, Algorithm 6, vertex-form removal), takes the whole-device
 * route.  A shape pass on the device measures each
 * graph (and checks its arrays, below); then one persistent launch gives whole
 * graphs, largest first, to workgroups that run all of a graph's rounds.  Per
 * graph the workgroup keeps per-net masks of colors 0..127 (sparse graphs),
 * a conflict bit matrix (n_A <= 16384 and colors expected past 127, or nets
 * overlapping more than the vertex pairs), or per-vertex forbidden-color
 * bitmaps.  Graphs that one workgroup would color far slower than the whole
 * device (more than 10^6 memberships, or colors past 127 on more than 16384
 * vertices with more than 5 * 10^4 memberships) are colored by bgpc_color on
 * three more streams (one host thread each) while the launch runs.
 *   items    host array; csr_A / csr_B / colors_out / order device pointers
 *            as in bgpc_color; status, rounds and route are written per item
 *   opts     NULL or the options of bgpc_color (log and prof are ignored;
 *            max_rounds applies per graph)
 * Checks: offsets start at 0, never decrease and end at nnz, indices in range
 * (else BGPC_E_INVALID for the batch, that item's status BGPC_E_INVALID and
 * nothing colored).  The two CSRs must be transposes of each other, with
 * sorted rows; unlike bgpc_color this is not checked.
 * Returns BGPC_OK, or the first non-OK item status (BGPC_E_NOT_CONVERGED).
 * Scratch: allocated per call, split into several launches when the sum over
 * the graphs exceeds half of the free device memory.
 */
typedef struct {
    bgpc_csr csr_A;       /* d2gc items: the symmetric adjacency (csr_B is ignored) */
    bgpc_csr csr_B;
    int32_t *colors_out;
    int32_t status;       /* out */
    int32_t rounds;       /* out */
    const int32_t *order; /* NULL or a device permutation, as for bgpc_color */
    int32_t d2gc;         /* nonzero: distance-2 coloring of csr_A (as d2gc_color) */
    int32_t route;        /* out: BGPC_ROUTE_* the item took */
} bgpc_batch_item;

/* bgpc_batch_item.route */
enum {
    BGPC_ROUTE_NET_MASKS = 0,     /* persistent launch, per-net masks of colors 0..127 */
    BGPC_ROUTE_BITMAPS = 1,       /* persistent launch, per-vertex forbidden-color bitmaps */
    BGPC_ROUTE_DENSE = 2,         /* persistent launch, conflict bit matrix */
    BGPC_ROUTE_WHOLE_DEVICE = 3   /* bgpc_color / d2gc_color on a side stream */
};

BGPC_API int bgpc_color_batch(bgpc_batch_item *items, int32_t n_items, const bgpc_opts *opts);

/*
 * Serving: a session colors requests as they arrive (continuous batching).
 * A worker thread admits waiting requests in arrival order while one of
 * `max_slots` slots is free and its device pool of `mem_budget` bytes has room
 * for the request (CSR arrays, colors, scratch; at most `max_group` admissions
 * per pass), copies the request's arrays in, and once they have arrived
 * publishes its descriptor on a ring that a persistent kernel drains: each
 * workgroup claims the next descriptor and runs all of its graph's rounds
 * (the rounds and per-graph modes of bgpc_color_batch), so requests admitted
 * while others run overlap on the device.  A request completes as soon as
 * its own graph is done: its workgroup copies the colors to host memory and
 * then sets a done word that the worker polls.  The kernel's workgroups leave
 * after about 20 ms without work and when the session is destroyed; the
 * worker launches the kernel again when work is published, and launches more
 * (as many workgroups as requests wait) when requests wait unclaimed while
 * fewer workgroups than compute units remain -- up to six launches at once
 * when the process has 16 or more hardware queues (GPU_MAX_HW_QUEUES, read
 * when the HIP runtime starts; HIP's default is 4, and then one launch, since
 * kernels on one hardware queue run in order).  Requests that
 * bgpc_color_batch would give to the whole device are colored by bgpc_color
 * on three more threads, each with a stream of its own; under light load a
 * request of 50,000 or more memberships also takes such a thread when one is
 * idle.  Their arrays are allocated outside the pool.  With 4 hardware
 * queues those streams share queues with the serving kernel and wait for it:
 * serving processes should start with GPU_MAX_HW_QUEUES of 16 or more.  A
 * request's colors equal what bgpc_color returns for its graph alone.  Calls
 * on one session may come from any thread.
 *
 * bgpc_request: host arrays (csr_A offsets / indices = a_off / a_idx, csr_B =
 * b_off / b_idx), read at submit (shape and checks, as in bgpc_color_batch)
 * and when the request is admitted; colors_out (host, int32[n_a]) is written
 * before its completion is reported; all must stay valid until then.  With
 * BGPC_REQ_PINNED every array is pinned host memory (hipHostMalloc) and is
 * copied directly, without the session's staging area.  tag is returned with
 * the completion.
 * bgpc_session_create returns NULL on failure.  submit returns BGPC_E_INVALID
 * for malformed arrays and BGPC_E_OOM for a request larger than the pool.
 * poll hands out up to `cap` completions (waiting up to wait_ms for the
 * first) and returns the session's error status (BGPC_OK normally).  destroy
 * completes every submitted request, then frees the session.  Times are
 * steady-clock seconds.
 */
typedef struct bgpc_session bgpc_session;

typedef struct {
    int32_t n_a;
    int32_t n_b;
    int64_t nnz;
    const int32_t *a_off;
    const int32_t *a_idx;
    const int32_t *b_off;
    const int32_t *b_idx;
    int32_t *colors_out;
    uint64_t tag;
    uint32_t flags;       /* BGPC_REQ_PINNED: the arrays above are pinned host memory */
    uint32_t reserved;
} bgpc_request;

enum {
    BGPC_REQ_PINNED = 1u  /* upload / download directly, without the session's staging copy */
};

typedef struct {
    uint64_t tag;
    int32_t status;
    int32_t rounds;
    double t_submit;
    double t_admit;
    double t_done;
} bgpc_completion;

BGPC_API bgpc_session *bgpc_session_create(size_t mem_budget, int32_t max_slots, int32_t max_group,
                                           int32_t max_rounds);
BGPC_API int bgpc_session_submit(bgpc_session *session, const bgpc_request *request);
BGPC_API int bgpc_session_poll(bgpc_session *session, bgpc_completion *out, int32_t cap, int32_t *n_out,
                               int32_t wait_ms);
BGPC_API void bgpc_session_destroy(bgpc_session *session);

/*
 * Allocation-free bgpc_color, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same rounds and colors as bgpc_color(csr_A, csr_B, NULL,
 * opts, colors_out), with the workspace in a static device array of
 * BGPC_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library runs on holds
 * until the process ends.  Calls no hipMalloc / hipFree / hipHostMalloc.
 *   Limits: |V_A| <= BGPC_NOALLOC_MAX_VERTICES, |V_B| <= BGPC_NOALLOC_MAX_NETS,
 *   nnz <= BGPC_NOALLOC_MAX_NNZ, the natural order only, and a workspace
 *   that fits the array (BGPC_E_UNSUPPORTED otherwise, before anything runs);
 *   no BGPC_INCREMENTAL, prof, or log hashes / round times
 *   (BGPC_E_UNSUPPORTED).  Colors past 63 are found through per-vertex LDS
 *   bitmaps instead of per-net color words (same colors; BGPC_E_UNSUPPORTED
 *   when a vertex's distance-2 colors pass the LDS bitmap).
 *   Every call on one GPU uses that GPU's one array and leaves its contents
 *   behind (each call initializes what it reads): calls that overlap on one
 *   GPU, from any stream or thread, race and must be serialized by the caller.
 */
#define BGPC_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define BGPC_NOALLOC_MAX_VERTICES (1 << 20)
#define BGPC_NOALLOC_MAX_NETS (1 << 20)
#define BGPC_NOALLOC_MAX_NNZ (1ll << 24)
BGPC_API int bgpc_color_noalloc(const bgpc_csr *csr_A, const bgpc_csr *csr_B, const bgpc_opts *opts,
                                int32_t *colors_out);

/* Human-readable name of a status code (static storage). */
BGPC_API const char *bgpc_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* BGPC_H */
