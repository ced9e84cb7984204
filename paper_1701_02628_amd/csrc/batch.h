// Many graphs in one launch: one workgroup colors one graph at a time, all of
// its rounds, with workgroup barriers only (no inter-workgroup waits).
// Workgroups take graphs from an atomic queue in the order the host gives
// (largest first) until the queue is empty, so every workgroup exits.
//
// A graph's rounds are the vertex-based first-fit rounds of Algorithm 1 with
// the rules of bgpc_color (snapshot, lower rank keeps, losers -> -1): the
// result of a graph depends on that graph only, never on the rest of the
// batch, on its mode or on the workgroup that ran it.  Three modes, chosen per
// graph from its shape (same results, different costs):
//   MASKS  per-net masks of colors 0..127 held by colored members; first-fit
//          ORs the masks of nets(w); removal scans the active nets
//   FORB   per-vertex forbidden-color bitmaps: a winner sets its color in the
//          bitmap of every vertex sharing a net with it; first-fit is the
//          first clear bit; removal scans the active nets (graphs whose
//          colors run far past 127)
//   DENSE  an explicit conflict bit matrix (n_A <= DENSE_N); removal buckets
//          the worklist by proposal and tests lower-ranked bucket members
//          against the matrix (short list per small bucket, member bitmap per
//          large one); the forbidden-color bitmaps take the winners' colors by
//          pull (each loser tests the round's winners against its matrix row)
//          or push (each winner walks its row), whichever touches less
// A net stays active while it has two or more uncolored members: with one or
// none left, no two of its members can ever propose in the same round again.
#pragma once

#include <algorithm>

#include "common.h"

namespace bgpc {

constexpr int BATCH_BLOCK = 512;   // threads per workgroup
constexpr int DENSE_N = 16384;     // largest graph of the DENSE mode
constexpr int BUCKET_T = 32;       // DENSE: buckets up to this size are lists, larger ones bitmaps
enum { MODE_MASKS = 0, MODE_FORB = 1, MODE_DENSE = 2 };

struct BatchItem {
    int n_a, n_b;
    const int *a_off, *a_idx;   // nets(u)
    const int *b_off, *b_idx;   // vtxs(v)
    int *colors;                // int32[n_a]
    char *scratch;              // batch_scratch_bytes(mode, n_a, n_b, cap) bytes
    int *log;                   // optional: per round (|W| at its start, losers, largest color after it)
    int log_cap;                // rounds the log can hold
    int max_rounds;
    int mode;                   // MODE_*
    int cap;                    // FORB / DENSE: every color stays below cap
    int status;                 // out: 0 ok, -6 not converged
    int rounds;                 // out
    double walk;                // shape: sum over nets of |vtxs(v)|^2, or -1 if the arrays are malformed
    int walk_max;               // shape: largest sum of |vtxs(v)| over the nets of one vertex
    int nnz;                    // memberships
    int *host_colors;           // optional, host memory: the colors, copied there when the graph is done
    long long *host_done;       // optional, host memory: set to (rounds << 32) | (status + 256) after that copy
};

__host__ __device__ inline long long words32(long long n) { return (n + 31) >> 5; }
__host__ __device__ inline long long al256(long long x) { return (x + 255) & ~255ll; }

// Mode of a graph from its shape.  The first-fit color of u is at most the
// number of other members of its nets, so colors stay below walk_max + 1
// (and below n_a); FORB and DENSE size their bitmaps by that bound.  Graphs
// whose colors are expected past the net masks (walk > 128 n_a) or whose
// nets overlap so much that walking them costs more than the vertex pairs
// (walk > 4 n_a^2) take DENSE when the matrix is small enough, else FORB.
__host__ inline int batch_mode(int n_a, double walk, long long walk_max, int *cap)
{
    const long long c = std::min<long long>(walk_max + 2, (long long)n_a + 1);
    const bool heavy = walk > 128.0 * (double)n_a || walk > 4.0 * (double)n_a * (double)n_a;
    if (n_a > 0 && heavy && n_a <= DENSE_N) {
        *cap = (int)c;
        return MODE_DENSE;
    }
    if (n_a > 0 && heavy && (long long)n_a * words32(c) * 4 <= (64ll << 20)) {
        *cap = (int)c;
        return MODE_FORB;
    }
    *cap = 128;
    return MODE_MASKS;
}

// words per conflict-matrix row (a multiple of 4 for 16-byte loads)
__host__ __device__ inline long long dense_wpr(long long n) { return ((n + 127) >> 7) << 2; }

__host__ __device__ inline long long batch_scratch_bytes(int mode, int n_a, int n_b, int cap)
{
    long long b = 2 * al256(4ll * (n_a + 1)) + al256(n_a + 1ll);
    if (mode != MODE_DENSE) b += 2 * al256(4ll * (n_b + 1));
    if (mode == MODE_MASKS) return b + al256(16ll * (n_b + 1));
    b += al256(4ll * n_a * words32(cap)) + al256(4ll * (n_a + 2));
    if (mode == MODE_DENSE) {
        const long long wpr = dense_wpr(n_a);
        b += al256(4ll * n_a * wpr) + 2 * al256(4ll * (cap + 2)) + al256(4ll * (cap + 2) * BUCKET_T) +
             al256(4ll * (n_a / BUCKET_T + 2) * wpr) + al256(4ll * (n_a + 1));
    }
    return b;
}

struct Scratch {
    int *w0, *w1;               // worklists
    uint8_t *lose;              // loser flags
    int *nl0, *nl1;             // active net lists (MASKS, FORB)
    unsigned long long *mask;   // MASKS: two words per net
    unsigned *forb;             // FORB, DENSE: n_a rows of words32(cap)
    int *ff;                    // FORB, DENSE: last proposal per vertex
    unsigned *adj;              // DENSE: n_a rows of dense_wpr(n_a) words
    int *cnt, *slot;            // DENSE: bucket sizes, bitmap row of each large bucket
    int *small;                 // DENSE: BUCKET_T members per small bucket
    unsigned *bits;             // DENSE: member bitmaps of the large buckets
    int *win;                   // DENSE: the round's winners
};

__device__ inline Scratch batch_scratch(const BatchItem &it)
{
    char *p = it.scratch;
    Scratch sc = {};
    sc.w0 = (int *)p;
    p += al256(4ll * (it.n_a + 1));
    sc.w1 = (int *)p;
    p += al256(4ll * (it.n_a + 1));
    sc.lose = (uint8_t *)p;
    p += al256(it.n_a + 1ll);
    if (it.mode != MODE_DENSE) {
        sc.nl0 = (int *)p;
        p += al256(4ll * (it.n_b + 1));
        sc.nl1 = (int *)p;
        p += al256(4ll * (it.n_b + 1));
    }
    if (it.mode == MODE_MASKS) {
        sc.mask = (unsigned long long *)p;
        return sc;
    }
    sc.forb = (unsigned *)p;
    p += al256(4ll * it.n_a * words32(it.cap));
    sc.ff = (int *)p;
    p += al256(4ll * (it.n_a + 2));
    if (it.mode == MODE_DENSE) {
        const long long wpr = dense_wpr(it.n_a);
        sc.adj = (unsigned *)p;
        p += al256(4ll * it.n_a * wpr);
        sc.cnt = (int *)p;
        p += al256(4ll * (it.cap + 2));
        sc.slot = (int *)p;
        p += al256(4ll * (it.cap + 2));
        sc.small = (int *)p;
        p += al256(4ll * (it.cap + 2) * BUCKET_T);
        sc.bits = (unsigned *)p;
        p += al256(4ll * (it.n_a / BUCKET_T + 2) * wpr);
        sc.win = (int *)p;
    }
    return sc;
}

// raise *p to v; reads first so that equal values skip the atomic
__device__ __forceinline__ void max_to(int *p, int v)
{
    if (*(volatile int *)p < v) atomicMax(p, v);
}

// Shape pass, one workgroup per graph: walk and walk_max of each item, and a
// check that every offset lies in [0, nnz], offsets never decrease, and every
// index is in range (walk = -1 otherwise).  An index is read only after the
// offsets around it passed, so malformed arrays are never followed.
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch_shape(BatchItem *items, int n_items)
{
    __shared__ double s_walk;
    __shared__ int s_max;
    __shared__ int s_bad;
    for (int k = blockIdx.x; k < n_items; k += gridDim.x) {
        const BatchItem it = items[k];
        const int nnz = it.nnz;
        if (threadIdx.x == 0) {
            s_walk = 0.0;
            s_max = 0;
            s_bad = (it.a_off[0] != 0 || it.a_off[it.n_a] != nnz || it.b_off[0] != 0 || it.b_off[it.n_b] != nnz);
        }
        __syncthreads();
        int bad = 0;
        double walk = 0.0;
        for (int v = threadIdx.x; v < it.n_b; v += blockDim.x) {
            int b = it.b_off[v], e = it.b_off[v + 1];
            if (b < 0 || e < b || e > nnz) {
                bad = 1;
                continue;
            }
            for (int j = b; j < e; j++) {
                unsigned x = (unsigned)it.b_idx[j];
                bad |= x >= (unsigned)it.n_a;
            }
            walk += (double)(e - b) * (double)(e - b);
        }
        if (__syncthreads_or(bad | s_bad) == 0) {
            int mx = 0;
            for (int u = threadIdx.x; u < it.n_a; u += blockDim.x) {
                int b = it.a_off[u], e = it.a_off[u + 1];
                if (b < 0 || e < b || e > nnz) {
                    bad = 1;
                    continue;
                }
                long long sum = 0;
                for (int q = b; q < e; q++) {
                    unsigned v = (unsigned)it.a_idx[q];
                    if (v >= (unsigned)it.n_b) {
                        bad = 1;
                        break;
                    }
                    sum += it.b_off[v + 1] - it.b_off[v];
                }
                mx = max(mx, (int)min(sum, (long long)0x3fffffff));
            }
            for (int d = WAVE / 2; d > 0; d >>= 1) {
                walk += __shfl_xor(walk, d);
                mx = max(mx, __shfl_xor(mx, d));
            }
            if (lane_id() == 0) {
                atomicAdd(&s_walk, walk);
                atomicMax(&s_max, mx);
            }
        }
        if (bad) s_bad = 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            items[k].walk = s_bad ? -1.0 : s_walk;
            items[k].walk_max = s_max;
        }
        __syncthreads();
    }
}

// first clear bit of a forbidden-color row at or after c (one exists below
// the row's width: a vertex has fewer colored neighbours than the width)
__device__ __forceinline__ int first_clear(const unsigned *row, int c)
{
    for (;;) {
        unsigned fr = ~row[c >> 5] & (~0u << (c & 31));
        if (fr) return (c & ~31) + __builtin_ctz(fr);
        c = (c & ~31) + 32;
    }
}

// MASKS: first-fit at or above `from` once colors 0..from-1 are forbidden,
// window by window of 128 colors over the distance-2 neighbourhood
__device__ int masks_first_fit_above(const BatchItem &it, const int *st, int w, int from)
{
    for (int base = from;; base += 128) {
        unsigned long long m0 = 0, m1 = 0;
        for (int k = it.a_off[w]; k < it.a_off[w + 1]; k++) {
            int v = it.a_idx[k];
            for (int j = it.b_off[v]; j < it.b_off[v + 1]; j++) {
                int x = it.b_idx[j];
                if (x == w) continue;
                int c = snap_color(st[x]) - base;
                if (c >= 0 && c < 64) m0 |= 1ull << c;
                else if (c >= 64 && c < 128) m1 |= 1ull << (c - 64);
            }
        }
        if (~m0) return base + __builtin_ctzll(~m0);
        if (~m1) return base + 64 + __builtin_ctzll(~m1);
    }
}

// Removal over the active nets: in a net, the first proposer of a color in
// rank order keeps it, later ones lose.  Nets with two or more proposals stay
// active (appended to Ln through the LDS counter *s_nl).
__device__ void net_removal(const BatchItem &it, const Scratch &sc, const int *st, const int *L, int nl, int *Ln,
                            int *s_nl)
{
    for (int i = threadIdx.x; i < nl; i += blockDim.x) {
        const int v = L[i];
        const int b = it.b_off[v], e = it.b_off[v + 1];
        unsigned long long s0 = 0, s1 = 0;
        bool wide = false;
        int pending = 0;
        for (int j = b; j < e; j++) {
            int x = it.b_idx[j];
            int s = st[x];
            if (s >= 0 && !(s & TENT)) continue;
            pending++;
            if (s < 0) continue;
            int c = s & COLOR_MASK;
            if (c < 64) {
                if ((s0 >> c) & 1ull) sc.lose[x] = 1;
                s0 |= 1ull << c;
            } else if (c < 128) {
                if ((s1 >> (c - 64)) & 1ull) sc.lose[x] = 1;
                s1 |= 1ull << (c - 64);
            } else {
                wide = true;
            }
        }
        if (wide) {
            // colors past 127: compare with the earlier proposers of the net
            for (int j = b; j < e; j++) {
                int x = it.b_idx[j];
                int s = st[x];
                if (s < 0 || !(s & TENT) || (s & COLOR_MASK) < 128) continue;
                for (int j2 = b; j2 < j; j2++) {
                    if (st[it.b_idx[j2]] == s) {
                        sc.lose[x] = 1;
                        break;
                    }
                }
            }
        }
        if (pending >= 2) Ln[atomicAdd(s_nl, 1)] = v;
    }
}

__device__ __forceinline__ bool adj_bit(const unsigned *row, int x) { return (row[x >> 5] >> (x & 31)) & 1u; }

// DENSE removal.  Proposals of the round lie in [cmin, cmax]; the worklist is
// bucketed by proposal.  w loses iff a lower-ranked member of its bucket is in
// its matrix row: a small bucket (<= BUCKET_T members) is a list that w scans,
// a large one a member bitmap that w ANDs with the part of its row below w.
__device__ void dense_removal(const BatchItem &it, const Scratch &sc, const int *st, const int *W, int nw, int cmin,
                              int cmax, int *s_nslot)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int R = cmax - cmin + 1;
    const long long wpr = dense_wpr(it.n_a);
    for (int c = tid; c < R; c += nt) sc.cnt[c] = 0;
    if (tid == 0) *s_nslot = 0;
    __syncthreads();
    for (int i = tid; i < nw; i += nt) {
        int w = W[i];
        int c = (st[w] & COLOR_MASK) - cmin;
        int k = atomicAdd(&sc.cnt[c], 1);
        if (k < BUCKET_T) sc.small[c * BUCKET_T + k] = w;
    }
    __syncthreads();
    for (int c = tid; c < R; c += nt)
        if (sc.cnt[c] > BUCKET_T) sc.slot[c] = atomicAdd(s_nslot, 1);
    __syncthreads();
    const long long nbits = (long long)(*s_nslot) * wpr;
    for (long long i = tid; i < nbits; i += nt) sc.bits[i] = 0;
    __syncthreads();
    for (int i = tid; i < nw; i += nt) {
        int w = W[i];
        int c = (st[w] & COLOR_MASK) - cmin;
        if (sc.cnt[c] > BUCKET_T) atomicOr(&sc.bits[sc.slot[c] * wpr + (w >> 5)], 1u << (w & 31));
    }
    __syncthreads();
    for (int i = tid; i < nw; i += nt) {
        const int w = W[i];
        const int c = (st[w] & COLOR_MASK) - cmin;
        const int n = sc.cnt[c];
        const unsigned *row = sc.adj + w * wpr;
        bool lost = false;
        if (n <= BUCKET_T) {
            const int *lst = sc.small + c * BUCKET_T;
            for (int k = 0; k < n && !lost; k++) {
                int x = lst[k];
                lost = x < w && adj_bit(row, x);
            }
        } else {
            const unsigned *P = sc.bits + sc.slot[c] * wpr;
            const int qw = w >> 5;
            const int q4 = qw >> 2;
            const uint4 *r4 = (const uint4 *)row, *p4 = (const uint4 *)P;
            for (int q = 0; q < q4 && !lost; q += 2) {
                uint4 a = r4[q], b = p4[q];
                unsigned acc = (a.x & b.x) | (a.y & b.y) | (a.z & b.z) | (a.w & b.w);
                if (q + 1 < q4) {
                    uint4 a2 = r4[q + 1], b2 = p4[q + 1];
                    acc |= (a2.x & b2.x) | (a2.y & b2.y) | (a2.z & b2.z) | (a2.w & b2.w);
                }
                lost = acc != 0;
            }
            for (int q = q4 * 4; q < qw && !lost; q++) lost = (row[q] & P[q]) != 0;
            if (!lost) lost = (row[qw] & P[qw] & ((1u << (w & 31)) - 1u)) != 0;
        }
        if (lost) sc.lose[w] = 1;
    }
    __syncthreads();
}

// FORB: a winner's color enters the forbidden rows of the vertices that
// share a net with it.
__device__ void push_color_nets(const BatchItem &it, const Scratch &sc, int w, int c)
{
    const long long fw = words32(it.cap);
    const unsigned bit = 1u << (c & 31);
    unsigned *col_word = sc.forb + (c >> 5);
    for (int k = it.a_off[w]; k < it.a_off[w + 1]; k++) {
        int v = it.a_idx[k];
        for (int j = it.b_off[v]; j < it.b_off[v + 1]; j++) {
            int y = it.b_idx[j];
            if (y != w) atomicOr(col_word + y * fw, bit);
        }
    }
}

// DENSE: the round's winners' colors enter the forbidden rows of their
// neighbours.  Pull: each vertex left uncolored tests every winner against
// its own row (its row is written by its thread only).  Push: each winner
// walks its row and sets its color in every neighbour's row.
__device__ void dense_propagate(const BatchItem &it, const Scratch &sc, const int *st, const int *Wn, int nw_next,
                                int nwin, bool pull)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const long long fw = words32(it.cap), wpr = dense_wpr(it.n_a);
    if (pull) {
        for (int i = tid; i < nw_next; i += nt) {
            const int y = Wn[i];
            const unsigned *row = sc.adj + y * wpr;
            unsigned *frow = sc.forb + y * fw;
            for (int j = 0; j < nwin; j++) {
                int x = sc.win[j];
                if (adj_bit(row, x)) {
                    int c = st[x];
                    frow[c >> 5] |= 1u << (c & 31);
                }
            }
        }
        return;
    }
    for (int j = tid; j < nwin; j += nt) {
        const int x = sc.win[j];
        const int c = st[x];
        const unsigned bit = 1u << (c & 31);
        unsigned *col_word = sc.forb + (c >> 5);
        const unsigned *row = sc.adj + x * wpr;
        for (int q = 0; q < wpr; q++) {
            unsigned m = row[q];
            while (m) {
                int y = (q << 5) + __builtin_ctz(m);
                m &= m - 1;
                atomicOr(col_word + y * fw, bit);
            }
        }
    }
}

// All rounds of one graph on the calling workgroup (every thread calls);
// returns the rounds run, *status 0 or -6 (round cap reached).
__device__ int batch_run_item(const BatchItem it, int *status)
{
    __shared__ int s_scan[20];
    __shared__ int s_maxc;
    __shared__ int s_nl;
    __shared__ int s_cmin, s_cmax, s_nslot;
    const int tid = threadIdx.x, nt = blockDim.x;
    {
        const Scratch sc = batch_scratch(it);
        int *st = it.colors;
        const int n_a = it.n_a, n_b = it.n_b;
        const int mode = it.mode;
        for (int u = tid; u < n_a; u += nt) {
            st[u] = -1;
            sc.w0[u] = u;
            sc.lose[u] = 0;
        }
        if (mode != MODE_DENSE)
            for (int v = tid; v < n_b; v += nt) sc.nl0[v] = v;
        if (mode == MODE_MASKS) {
            for (int v = tid; v < 2 * n_b; v += nt) sc.mask[v] = 0;
        } else {
            const long long fwords = (long long)n_a * words32(it.cap);
            for (long long i = tid; i < fwords; i += nt) sc.forb[i] = 0;
            for (int u = tid; u < n_a; u += nt) sc.ff[u] = 0;
        }
        int avg_deg2 = 0;
        if (mode == MODE_DENSE) {
            // conflict matrix: bit y of row x iff x != y share a net
            const long long wpr = dense_wpr(n_a);
            for (long long i = tid; i < (long long)n_a * wpr; i += nt) sc.adj[i] = 0;
            __syncthreads();
            for (int v = tid; v < n_b; v += nt) {
                int b = it.b_off[v], e = it.b_off[v + 1];
                for (int i = b; i < e; i++) {
                    int x = it.b_idx[i];
                    for (int j = b; j < e; j++) {
                        int y = it.b_idx[j];
                        if (y != x) atomicOr(&sc.adj[x * wpr + (y >> 5)], 1u << (y & 31));
                    }
                }
            }
            __syncthreads();
            int pc = 0;
            for (long long i = tid; i < (long long)n_a * wpr; i += nt) pc += __builtin_popcount(sc.adj[i]);
            long long tot = 0;
            {
                // block sum in 64 bits: popcounts can exceed 2^31 in total
                unsigned long long v = (unsigned long long)pc;
                for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
                __shared__ unsigned long long s_pc;
                if (tid == 0) s_pc = 0;
                __syncthreads();
                if (lane_id() == 0) atomicAdd(&s_pc, v);
                __syncthreads();
                tot = (long long)s_pc;
            }
            avg_deg2 = n_a ? (int)(tot / n_a) : 0;
        }
        if (tid == 0) {
            s_maxc = -1;
            s_cmin = 0x7fffffff;
            s_cmax = -1;
        }
        __syncthreads();
        int *W = sc.w0, *Wn = sc.w1;
        int *L = sc.nl0, *Ln = sc.nl1;
        int nw = n_a, nl = n_b;
        int rounds = 0;
        const long long fw = words32(it.cap);
        while (nw > 0 && rounds < it.max_rounds) {
            // first-fit proposals against the snapshot
            int lo = 0x7fffffff, hi = -1;
            for (int i = tid; i < nw; i += nt) {
                int w = W[i];
                int col;
                if (mode == MODE_MASKS) {
                    unsigned long long m0 = 0, m1 = 0;
                    for (int q = it.a_off[w]; q < it.a_off[w + 1]; q++) {
                        int v = it.a_idx[q];
                        m0 |= sc.mask[2 * v];
                        m1 |= sc.mask[2 * v + 1];
                    }
                    if (~m0) col = __builtin_ctzll(~m0);
                    else if (~m1) col = 64 + __builtin_ctzll(~m1);
                    else col = masks_first_fit_above(it, st, w, 128);
                } else {
                    col = first_clear(sc.forb + w * fw, sc.ff[w]);
                    sc.ff[w] = col;
                }
                st[w] = TENT | col;
                lo = min(lo, col);
                hi = max(hi, col);
            }
            if (mode == MODE_DENSE) {
                for (int d = WAVE / 2; d > 0; d >>= 1) {
                    lo = min(lo, __shfl_xor(lo, d));
                    hi = max(hi, __shfl_xor(hi, d));
                }
                if (lane_id() == 0 && hi >= 0) {
                    atomicMin(&s_cmin, lo);
                    atomicMax(&s_cmax, hi);
                }
            }
            if (tid == 0) s_nl = 0;
            __syncthreads();
            if (mode == MODE_DENSE) {
                dense_removal(it, sc, st, W, nw, s_cmin, s_cmax, &s_nslot);
            } else {
                net_removal(it, sc, st, L, nl, Ln, &s_nl);
                __syncthreads();
            }
            // winners keep their colors, losers -> -1 (stable compaction);
            // DENSE also lists the winners
            int base_out = 0;
            for (int i0 = 0; i0 < nw; i0 += nt) {
                int i = i0 + tid;
                int flag = 0;
                int w = -1;
                if (i < nw) {
                    w = W[i];
                    if (sc.lose[w]) {
                        sc.lose[w] = 0;
                        st[w] = -1;
                        flag = 1;
                    } else {
                        int col = st[w] & COLOR_MASK;
                        st[w] = col;
                        max_to(&s_maxc, col);
                        if (mode == MODE_MASKS) {
                            if (col < 128) {
                                unsigned long long bit = 1ull << (col & 63);
                                int half = col >> 6;
                                for (int q = it.a_off[w]; q < it.a_off[w + 1]; q++)
                                    atomicOr(&sc.mask[2 * it.a_idx[q] + half], bit);
                            }
                        } else if (mode == MODE_FORB) {
                            push_color_nets(it, sc, w, col);
                        }
                    }
                }
                int total;
                int pos = block_excl_scan(flag, s_scan, &total);
                if (flag) Wn[base_out + pos] = w;
                else if (i < nw && mode == MODE_DENSE) sc.win[i - base_out - pos] = w;
                base_out += total;
            }
            if (tid == 0) {
                s_cmin = 0x7fffffff;
                s_cmax = -1;
            }
            __syncthreads();
            if (mode == MODE_DENSE) {
                const int nwin = nw - base_out;
                dense_propagate(it, sc, st, Wn, base_out, nwin, base_out <= avg_deg2);
                __syncthreads();
            }
            if (tid == 0 && it.log && rounds < it.log_cap) {
                it.log[3 * rounds] = nw;
                it.log[3 * rounds + 1] = base_out;
                it.log[3 * rounds + 2] = s_maxc;
            }
            if (mode != MODE_DENSE) {
                nl = s_nl;
                int *t = L;
                L = Ln;
                Ln = t;
            }
            int *tmp = W;
            W = Wn;
            Wn = tmp;
            nw = base_out;
            rounds++;
            __syncthreads();
        }
        *status = nw == 0 ? 0 : -6;
        if (it.host_done) {
            // hand the graph over to the host: colors first, then (after every
            // wave's system-scope fence, which also writes back this graph's
            // scratch from L2) the done word
            if (it.host_colors)
                for (int u = tid; u < n_a; u += nt) it.host_colors[u] = st[u];
            __threadfence_system();
            __syncthreads();
            if (tid == 0) {
                __atomic_store_n(it.host_done, ((long long)rounds << 32) | (unsigned)(*status + 256),
                                 __ATOMIC_RELAXED);
                __threadfence_system();
            }
        }
        __syncthreads();
        return rounds;
    }
}

__global__ void __launch_bounds__(BATCH_BLOCK) k_batch(BatchItem *items, const int *order, int n_items, int *next)
{
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(next, 1);
        __syncthreads();
        const int k = s_item;
        __syncthreads();
        if (k >= n_items) break;
        int status = 0;
        const int rounds = batch_run_item(items[order[k]], &status);
        if (threadIdx.x == 0) {
            items[order[k]].rounds = rounds;
            items[order[k]].status = status;
        }
        __syncthreads();
    }
}

// Serving ring in coherent pinned host memory: the host writes descriptors
// and then publishes them by raising tail; workgroups claim them in order
// through a device counter.
struct ServeRing {
    int tail;       // descriptors published (items[k % cap] for k < tail)
    int stop;       // set by the host: workgroups exit
    int active;     // workgroups inside k_serve (read by the host)
    int claimed;    // descriptors claimed so far (the largest claim + 1; read by the host)
    int pad[60];
    BatchItem items[1];
};

// Persistent serving kernel.  A workgroup claims the next published
// descriptor, invalidates its caches (the descriptor's arrays were copied in
// by DMA after this kernel started, possibly into memory an earlier request
// used), copies the descriptor to LDS and runs the graph; the graph's
// completion reaches the host through its done word.  A workgroup leaves
// after idle_spins empty polls (about 14 us apart) or when stop is set, so
// every wave exits.  Workgroups count themselves in `active` and publish the
// claims in `claimed`, so the host can launch more workgroups (another launch
// of this kernel, on another stream) while published requests wait
// unclaimed behind the few workgroups still busy with long graphs.
__global__ void __launch_bounds__(BATCH_BLOCK) k_serve(ServeRing *ring, int cap, int *head, int idle_spins)
{
    __shared__ int s_k;
    __shared__ unsigned long long s_desc[(sizeof(BatchItem) + 7) / 8];
    const int tid = threadIdx.x;
    if (tid == 0) __hip_atomic_fetch_add(&ring->active, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (;;) {
        if (tid == 0) {
            int k = -1;
            for (int spin = 0; spin < idle_spins; spin++) {
                const int t = __hip_atomic_load(&ring->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                const int h = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h < t) {
                    if (atomicCAS(head, h, h + 1) == h) {
                        k = h;
                        __hip_atomic_fetch_max(&ring->claimed, h + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        break;
                    }
                    spin = 0;   // another workgroup took it: not idle
                    continue;
                }
                if ((spin & 15) == 15 && __hip_atomic_load(&ring->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
                    break;
                // about 14 us between polls of host memory: hundreds of idle
                // workgroups polling faster load the path that the uploads
                // and the done words take
                __builtin_amdgcn_s_sleep(127);
                __builtin_amdgcn_s_sleep(127);
                __builtin_amdgcn_s_sleep(127);
                __builtin_amdgcn_s_sleep(127);
            }
            if (k >= 0) __threadfence_system();
            s_k = k;
        }
        __syncthreads();
        const int k = s_k;
        if (k < 0) {
            if (tid == 0) __hip_atomic_fetch_add(&ring->active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            break;
        }
        const unsigned long long *src = (const unsigned long long *)&ring->items[k % cap];
        for (int i = tid; i < (int)((sizeof(BatchItem) + 7) / 8); i += blockDim.x) s_desc[i] = src[i];
        __syncthreads();
        const BatchItem it = *(const BatchItem *)s_desc;
        __syncthreads();
        int status = 0;
        batch_run_item(it, &status);
    }
}

}  // namespace bgpc
