// Many graphs in one launch: one workgroup colors one graph at a time, all of
// its rounds, with workgroup barriers only (no inter-workgroup waits).
// Workgroups take graphs from an atomic queue in the order the host gives
// (largest first) until the queue is empty, so every workgroup exits.
//
// A graph's rounds are the vertex-based first-fit rounds of Algorithm 1 with
// the rules of bgpc_color (snapshot, lower rank keeps, losers -> -1): the
// result of a graph depends on that graph only, never on the rest of the
// batch or on which workgroup ran it.
#pragma once

#include "common.h"

namespace bgpc {

constexpr int BATCH_BLOCK = 512;   // threads per workgroup

struct BatchItem {
    int n_a, n_b;
    const int *a_off, *a_idx;   // nets(u)
    const int *b_off, *b_idx;   // vtxs(v)
    int *colors;                // int32[n_a]
    char *scratch;              // own scratch (serving) or nullptr (the workgroup's slot)
    int *log;                   // optional: per round (|W| at its start, losers, largest color after it)
    int log_cap;                // rounds the log can hold
    int max_rounds;
    int status;                 // out: 0 ok, -6 not converged
    int rounds;                 // out
    int dense;                  // out: 1 if the graph ran in dense mode
};

// Graphs with at most DENSE_N vertices whose nets overlap heavily (walking
// every vertex's nets would visit far more memberships than there are vertex
// pairs) run in dense mode: an explicit conflict bit matrix and per-vertex
// forbidden-color bitmaps.
constexpr int DENSE_N = 4096;

__host__ __device__ inline int dense_words(int n) { return (n + 31) >> 5; }

// raise *p to v; reads first so that equal values skip the atomic
__device__ __forceinline__ void max_to(int *p, int v)
{
    if (*(volatile int *)p < v) atomicMax(p, v);
}

// scratch of one graph: two worklists, loser flags, done flags per net, two
// mask words per net (colors 0..127 of its colored members); dense mode adds
// the conflict bit matrix, the forbidden bitmaps, the first-fit cursor per
// vertex and the color buckets
struct BatchSlot {
    int *w0, *w1;
    uint8_t *lose;
    uint8_t *done;
    unsigned long long *mask;
    unsigned *adj, *forb;
    int *ff, *cnt, *cur, *list;
    int dense_cap;   // vertices the dense arrays can hold
};

__host__ __device__ inline long long batch_slot_bytes(int cap_a, int cap_b)
{
    auto al = [](long long x) { return (x + 255) & ~255ll; };
    long long dn = cap_a < DENSE_N ? cap_a : DENSE_N;
    long long dense = 2 * al(4ll * dn * dense_words((int)dn)) + 4 * al(4ll * (dn + 2));
    return 2 * al(4ll * (cap_a + 1)) + al(16ll * (cap_b + 1)) + al(cap_a + 1ll) + al(cap_b + 1ll) + dense;
}

__device__ inline BatchSlot batch_slot(char *p, int cap_a, int cap_b)
{
    auto al = [](long long x) { return (x + 255) & ~255ll; };
    BatchSlot sl;
    sl.w0 = (int *)p;
    p += al(4ll * (cap_a + 1));
    sl.w1 = (int *)p;
    p += al(4ll * (cap_a + 1));
    sl.mask = (unsigned long long *)p;
    p += al(16ll * (cap_b + 1));
    sl.lose = (uint8_t *)p;
    p += al(cap_a + 1ll);
    sl.done = (uint8_t *)p;
    p += al(cap_b + 1ll);
    const long long dn = cap_a < DENSE_N ? cap_a : DENSE_N;
    sl.dense_cap = (int)dn;
    sl.adj = (unsigned *)p;
    p += al(4ll * dn * dense_words((int)dn));
    sl.forb = (unsigned *)p;
    p += al(4ll * dn * dense_words((int)dn));
    sl.ff = (int *)p;
    p += al(4ll * (dn + 2));
    sl.cnt = (int *)p;
    p += al(4ll * (dn + 2));
    sl.cur = (int *)p;
    p += al(4ll * (dn + 2));
    sl.list = (int *)p;
    return sl;
}

// Dense mode: all rounds of one graph.  adj row u holds bit x iff x != u
// shares a net with u; forb row u holds bit c iff a colored vertex of u's
// row has color c (colors stay below n_a in first-fit rounds).  A round:
// first-fit = first clear bit of forb[w] (from the vertex's last answer, which
// can only grow); the worklist is bucketed by proposed color; w loses iff a
// lower-ranked vertex of its bucket is in its adj row; winners set their
// color in the forb rows of their adj row.  Returns the rounds run; *nw_out
// the worklist left.
__device__ int batch_dense(const BatchItem &it, const BatchSlot &sl, int *st, int *s_scan, int *s_maxc, int *nw_out)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n = it.n_a, wpr = dense_words(n);
    for (long long i = tid; i < (long long)n * wpr; i += nt) {
        sl.adj[i] = 0;
        sl.forb[i] = 0;
    }
    for (int u = tid; u < n; u += nt) sl.ff[u] = 0;
    __syncthreads();
    for (int v = tid; v < it.n_b; v += nt) {
        int b = it.b_off[v], e = it.b_off[v + 1];
        for (int i = b; i < e; i++) {
            int x = it.b_idx[i];
            for (int j = b; j < e; j++) {
                int y = it.b_idx[j];
                if (y != x) atomicOr(&sl.adj[(long long)x * wpr + (y >> 5)], 1u << (y & 31));
            }
        }
    }
    __syncthreads();
    int *W = sl.w0, *Wn = sl.w1;
    int nw = n, rounds = 0, maxc = -1;
    while (nw > 0 && rounds < it.max_rounds) {
        // first-fit from the bitmaps; bucket counts
        for (int c = tid; c <= n; c += nt) sl.cnt[c] = 0;
        __syncthreads();
        for (int i = tid; i < nw; i += nt) {
            int w = W[i];
            const unsigned *row = sl.forb + (long long)w * wpr;
            int c = sl.ff[w];
            for (;;) {
                unsigned fr = ~row[c >> 5] & (~0u << (c & 31));
                if (fr) {
                    c = (c & ~31) + __builtin_ctz(fr);
                    break;
                }
                c = (c & ~31) + 32;
            }
            sl.ff[w] = c;
            st[w] = TENT | c;
            atomicAdd(&sl.cnt[c], 1);
        }
        __syncthreads();
        // bucket starts (exclusive scan over colors 0..n)
        int carry = 0;
        for (int c0 = 0; c0 <= n; c0 += nt) {
            int c = c0 + tid;
            int v = c <= n ? sl.cnt[c] : 0;
            int total;
            int ex = block_excl_scan(v, s_scan, &total);
            if (c <= n) {
                sl.cnt[c] = carry + ex;
                sl.cur[c] = carry + ex;
            }
            carry += total;
        }
        __syncthreads();
        for (int i = tid; i < nw; i += nt) {
            int w = W[i];
            int c = st[w] & COLOR_MASK;
            sl.list[atomicAdd(&sl.cur[c], 1)] = w;
        }
        __syncthreads();
        // removal: a lower-ranked conflicting vertex with the same proposal
        for (int i = tid; i < nw; i += nt) {
            int w = W[i];
            int c = st[w] & COLOR_MASK;
            const unsigned *row = sl.adj + (long long)w * wpr;
            int b = sl.cnt[c], e = sl.cur[c];
            for (int j = b; j < e; j++) {
                int x = sl.list[j];
                if (x < w && ((row[x >> 5] >> (x & 31)) & 1u)) {
                    sl.lose[w] = 1;
                    break;
                }
            }
        }
        __syncthreads();
        // apply + stable compaction; winners feed their neighbours' bitmaps
        int base_out = 0;
        for (int i0 = 0; i0 < nw; i0 += nt) {
            int i = i0 + tid;
            int flag = 0;
            if (i < nw) {
                int w = W[i];
                if (sl.lose[w]) {
                    sl.lose[w] = 0;
                    flag = 1;
                } else {
                    int c = st[w] & COLOR_MASK;
                    st[w] = c;
                    max_to(s_maxc, c);
                    const unsigned *row = sl.adj + (long long)w * wpr;
                    const unsigned bit = 1u << (c & 31);
                    for (int q = 0; q < wpr; q++) {
                        unsigned m = row[q];
                        while (m) {
                            int y = (q << 5) + __builtin_ctz(m);
                            m &= m - 1;
                            atomicOr(&sl.forb[(long long)y * wpr + (c >> 5)], bit);
                        }
                    }
                }
            }
            int total;
            int pos = block_excl_scan(flag, s_scan, &total);
            if (flag) Wn[base_out + pos] = W[i];
            base_out += total;
        }
        __syncthreads();
        maxc = *s_maxc;
        if (tid == 0 && it.log && rounds < it.log_cap) {
            it.log[3 * rounds] = nw;
            it.log[3 * rounds + 1] = base_out;
            it.log[3 * rounds + 2] = maxc;
        }
        int *tmp = W;
        W = Wn;
        Wn = tmp;
        nw = base_out;
        rounds++;
        __syncthreads();
    }
    // proposals of vertices still uncolored (round cap reached) become -1
    for (int i = tid; i < nw; i += nt) st[W[i]] = -1;
    __syncthreads();
    *nw_out = nw;
    return rounds;
}

__device__ __forceinline__ int batch_block_scan(int v, int *scratch, int *total)
{
    return block_excl_scan(v, scratch, total);
}

// First-fit color of w for colors >= `from`: window by window of 128 colors,
// walking the distance-2 neighbourhood (used once colors 0..127 are all
// forbidden).
__device__ int batch_first_fit_above(const BatchItem &it, const int *st, int w, int from)
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

__global__ void __launch_bounds__(BATCH_BLOCK) k_batch(BatchItem *items, const int *order, int n_items,
                                                       int *next, char *slot_base, long long slot_bytes,
                                                       int slot_cap_a, int slot_cap_b)
{
    __shared__ int s_scan[20];
    __shared__ int s_item;
    __shared__ int s_nw;
    __shared__ double s_walk;
    __shared__ int s_maxc;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(next, 1);
        __syncthreads();
        const int k = s_item;
        __syncthreads();
        if (k >= n_items) break;
        BatchItem it = items[order[k]];
        const BatchSlot sl = it.scratch ? batch_slot(it.scratch, it.n_a, it.n_b)
                                        : batch_slot(slot_base + (long long)blockIdx.x * slot_bytes, slot_cap_a,
                                                     slot_cap_b);
        int *st = it.colors;
        const int n_a = it.n_a, n_b = it.n_b;
        // dense mode when the net walk would exceed four times the vertex pairs
        double walk = 0.0;
        for (int v = tid; v < n_b; v += nt) {
            double k = (double)(it.b_off[v + 1] - it.b_off[v]);
            walk += k * k;
        }
        for (int d = WAVE / 2; d > 0; d >>= 1) walk += __shfl_xor(walk, d);
        if (tid == 0) s_walk = 0.0;
        __syncthreads();
        if (lane_id() == 0) atomicAdd(&s_walk, walk);
        __syncthreads();
        const bool dense = n_a <= sl.dense_cap && s_walk > 4.0 * (double)n_a * (double)n_a;
        __syncthreads();
        if (dense) {
            for (int u = tid; u < n_a; u += nt) {
                st[u] = -1;
                sl.w0[u] = u;
                sl.lose[u] = 0;
            }
            __syncthreads();
            int nw_left = 0;
            if (tid == 0) s_maxc = -1;
            __syncthreads();
            int rounds = batch_dense(it, sl, st, s_scan, &s_maxc, &nw_left);
            if (tid == 0) {
                items[order[k]].rounds = rounds;
                items[order[k]].status = nw_left == 0 ? 0 : -6;
                items[order[k]].dense = 1;
            }
            __syncthreads();
            continue;
        }
        for (int u = tid; u < n_a; u += nt) {
            st[u] = -1;
            sl.w0[u] = u;
            sl.lose[u] = 0;
        }
        for (int v = tid; v < n_b; v += nt) {
            sl.mask[2 * v] = 0;
            sl.mask[2 * v + 1] = 0;
            sl.done[v] = 0;
        }
        if (tid == 0) s_nw = n_a;
        __syncthreads();
        int *W = sl.w0, *Wn = sl.w1;
        int rounds = 0;
        int nw = s_nw;
        if (tid == 0) s_maxc = -1;
        __syncthreads();
        while (nw > 0 && rounds < it.max_rounds) {
            // coloring: OR of the nets' masks, first clear bit
            for (int i = tid; i < nw; i += nt) {
                int w = W[i];
                unsigned long long m0 = 0, m1 = 0;
                for (int q = it.a_off[w]; q < it.a_off[w + 1]; q++) {
                    int v = it.a_idx[q];
                    m0 |= sl.mask[2 * v];
                    m1 |= sl.mask[2 * v + 1];
                }
                int col;
                if (~m0) col = __builtin_ctzll(~m0);
                else if (~m1) col = 64 + __builtin_ctzll(~m1);
                else col = batch_first_fit_above(it, st, w, 128);
                st[w] = TENT | col;
            }
            __syncthreads();
            // removal, net side: first proposed holder of a color (rank order) keeps
            for (int v = tid; v < n_b; v += nt) {
                if (sl.done[v]) continue;
                int b = it.b_off[v], e = it.b_off[v + 1];
                unsigned long long s0 = 0, s1 = 0;
                bool wide = false;
                int pending = 0;
                for (int j = b; j < e; j++) {
                    int x = it.b_idx[j];
                    int s = st[x];
                    if (s < 0) {
                        pending++;
                        continue;
                    }
                    if (!(s & TENT)) continue;
                    pending++;
                    int c = s & COLOR_MASK;
                    if (c < 64) {
                        if ((s0 >> c) & 1ull) sl.lose[x] = 1;
                        s0 |= 1ull << c;
                    } else if (c < 128) {
                        if ((s1 >> (c - 64)) & 1ull) sl.lose[x] = 1;
                        s1 |= 1ull << (c - 64);
                    } else {
                        wide = true;
                    }
                }
                if (wide) {
                    for (int j = b; j < e; j++) {
                        int x = it.b_idx[j];
                        int s = st[x];
                        if (s < 0 || !(s & TENT) || (s & COLOR_MASK) < 128) continue;
                        for (int j2 = b; j2 < j; j2++) {
                            int t = st[it.b_idx[j2]];
                            if (t >= 0 && (t & TENT) && (t & COLOR_MASK) == (s & COLOR_MASK)) {
                                sl.lose[x] = 1;
                                break;
                            }
                        }
                    }
                }
                if (pending == 0) sl.done[v] = 1;
            }
            __syncthreads();
            // apply + stable compaction of the losers
            int base_out = 0;
            for (int i0 = 0; i0 < nw; i0 += nt) {
                int i = i0 + tid;
                int flag = 0;
                if (i < nw) {
                    int w = W[i];
                    int s = st[w];
                    if (sl.lose[w]) {
                        sl.lose[w] = 0;
                        st[w] = -1;
                        flag = 1;
                    } else {
                        int col = s & COLOR_MASK;
                        st[w] = col;
                        max_to(&s_maxc, col);
                        if (col < 128) {
                            unsigned long long bit = 1ull << (col & 63);
                            int wsel = col >> 6;
                            for (int q = it.a_off[w]; q < it.a_off[w + 1]; q++)
                                atomicOr(&sl.mask[2 * it.a_idx[q] + wsel], bit);
                        }
                    }
                }
                int total;
                int pos = batch_block_scan(flag, s_scan, &total);
                if (flag) Wn[base_out + pos] = W[i];
                base_out += total;
            }
            __syncthreads();
            if (tid == 0 && it.log && rounds < it.log_cap) {
                it.log[3 * rounds] = nw;
                it.log[3 * rounds + 1] = base_out;
                it.log[3 * rounds + 2] = s_maxc;
            }
            int *tmp = W;
            W = Wn;
            Wn = tmp;
            nw = base_out;
            rounds++;
            __syncthreads();
        }
        if (tid == 0) {
            items[order[k]].rounds = rounds;
            items[order[k]].status = nw == 0 ? 0 : -6;
            items[order[k]].dense = 0;
        }
        __syncthreads();
    }
}

}  // namespace bgpc
