// Round kernels of the speculative coloring loop (gfx950, wave64).
//
// One round of Algorithm 1 is a fixed sequence of launches that all read the
// worklist length from device memory, so the host never waits on a round:
//
//   coloring   vertex-based: k_vcolor_ff (first-fit through per-net masks of
//              colors 0..63) + k_vcolor_wide (block per vertex whose colors
//              spill past 63), or k_vcolor_chunked (B1 / B2, wave per chunk);
//              net-based: k_ncolor_small (thread per net) + k_ncolor_big
//              (block per net)
//   removal    k_conflict_small (thread per net) + k_conflict_big (block per
//              net)
//   apply      k_apply: losers -> -1, winners keep their color and set their
//              bit in the masks of their nets; per-tile loser counts
//   compaction k_compact: stable scatter of the losers into the next worklist
#pragma once

#include "common.h"

namespace bgpc {

constexpr int SMALL_NET = 64;       // nets up to this size run thread-per-net
constexpr int NBIG_BLOCK = 256;     // threads of k_ncolor_big
constexpr int TILE = 2048;          // worklist entries per compaction tile
constexpr int TILE_BLOCK = 256;     // threads of the apply / compaction blocks
constexpr int HASH_MAX = 4096;      // big nets up to this size use an LDS hash
constexpr int WIN_COLORS = 16384;   // color window of the largest nets
constexpr int STAGE = 2048;         // net-list entries staged in LDS per wave

// Blocks are dealt to the 8 XCDs round-robin.  With a grid that is a multiple
// of 8, logical block (x * nb/8 + k) runs on XCD x, so each XCD walks one
// contiguous stretch of items and the neighbourhoods it gathers stay in its
// own L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    return (nb & 7) ? bid : (bid & 7) * (nb >> 3) + (bid >> 3);
}

// largest j in [0, 64) with pre[j] <= f, for non-decreasing pre[] with pre[0] <= f
__device__ __forceinline__ int row_of(const int *pre, int f)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (pre[lo + step] <= f) lo += step;
    return lo;
}

// atomicMax that skips the atomic when a plain read already shows a value
// at least as large: many waves end with the same value, and same-address
// atomics serialize at the L2.
__device__ __forceinline__ void max_to(int *p, int v)
{
    if (*(volatile int *)p < v) atomicMax(p, v);
}

// Counters and helpers of the incremental first-fit rounds (see below).
struct IncCtrl {
    int n_d[2];     // dirty list, double-buffered by round parity
    int n_a;        // vertices whose removal test is redone
    int n_win;      // winners of the round
    int n_tcn;      // nets holding a changed proposal
    int n_cn;       // nets holding a winner
    int pad[2];
};

// set bit id once; true for the caller that set it
__device__ __forceinline__ bool set_once(unsigned *bits, int id)
{
    unsigned b = 1u << (id & 31);
    if (bits[id >> 5] & b) return false;
    return !(atomicOr(&bits[id >> 5], b) & b);
}

__device__ __forceinline__ void clear_bit(unsigned *bits, int id)
{
    atomicAnd(&bits[id >> 5], ~(1u << (id & 31)));
}

__device__ __forceinline__ bool is_tent(int s) { return s >= 0 && (s & TENT); }

// record that w's proposal changed: its nets are queued for k_expand into A
template <bool D2>
__device__ __forceinline__ void mark_proposal_change(const Graph &g, int w, unsigned *tchg_bits, int *tcn,
                                                     IncCtrl *ic)
{
    int k = Acc<D2>::nets_count(g, w);
    for (int j = 0; j < k; j++) {
        int v = Acc<D2>::net_at(g, w, j);
        if (set_once(tchg_bits, v)) tcn[atomicAdd(&ic->n_tcn, 1)] = v;
    }
}

// ---------------------------------------------------------------------------
// setup

__global__ void k_fill_i32(int *p, int v, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_iota(int *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

__global__ void k_init_ctrl(Ctrl *c, int n_w, int max_color)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->n_w[0] = n_w;
        c->n_w[1] = 0;
        c->n_heavy = 0;
        c->max_color = max_color;
        c->rounds = 0;
        c->error = 0;
        c->pad[0] = max_color;   // largest color present (max_final)
        c->pad[1] = 0;
        c->fl_n[0] = c->fl_n[1] = 0;
        c->zl_n[0] = c->zl_n[1] = 0;
        c->dl_n = 0;
        c->win = 0;
        c->done_blocks = 0;
        c->z0n[0] = c->z0n[1] = 0;
    }
}

// Per-graph shape figures: largest net, and a bound on every vertex's
// distance-2 neighbourhood (sum of the sizes of its nets); lists of the nets
// above SMALL_NET and above HASH_MAX members.
template <bool D2>
__global__ void k_net_shape(Graph g, int *max_net, int *big_list, int *n_big, unsigned long long *walk,
                            int *max_deg, int *huge_list, int *n_huge)
{
    int local = 0, deg = 0;
    unsigned long long w = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n_b; v += gridDim.x * blockDim.x) {
        int sz = Acc<D2>::size(g, v);
        local = max(local, sz);
        w += (unsigned long long)sz * (unsigned long long)sz;
        if (sz > SMALL_NET) big_list[atomicAdd(n_big, 1)] = v;
        if (sz > HASH_MAX) huge_list[atomicAdd(n_huge, 1)] = v;
    }
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < g.n_a; u += gridDim.x * blockDim.x)
        deg = max(deg, Acc<D2>::nets_count(g, u));
    local = wave_max(local);
    deg = wave_max(deg);
    if (lane_id() == 0) {
        max_to(max_net, local);
        max_to(max_deg, deg);
    }
    if (w) atomicAdd(walk, w);
}

// owner(u): the largest net containing u, ties to the lowest net id
template <bool D2>
__global__ void k_owner(Graph g, int *owner)
{
    // key of a net: larger size first, then lower id (0: no net)
    auto key_of = [&](int v) {
        return ((unsigned long long)(Acc<D2>::size(g, v) + 1) << 32) | (unsigned)(0x7fffffff - v);
    };
    const int lane = lane_id();
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x + threadIdx.x - lane; base < g.n_a; base += stride) {
        const int u = base + lane;
        const int k = u < g.n_a ? Acc<D2>::nets_count(g, u) : 0;
        const bool coop = k > 4 * WAVE;   // long rows: the whole wave, below
        unsigned long long key = 0;
        if (!coop)
            for (int j = 0; j < k; j++) key = max(key, key_of(Acc<D2>::net_at(g, u, j)));
        for (uint64_t bal = __ballot(coop); bal; bal &= bal - 1) {
            const int j = __builtin_ctzll(bal);
            const int uj = __shfl(u, j), kj = __shfl(k, j);
            unsigned long long acc = 0;
            for (int t = lane; t < kj; t += WAVE) acc = max(acc, key_of(Acc<D2>::net_at(g, uj, t)));
            for (int o = WAVE / 2; o > 0; o >>= 1) acc = max(acc, shfl64(acc, lane ^ o));
            if (lane == j) key = acc;
        }
        if (u < g.n_a) owner[u] = key ? 0x7fffffff - (int)(unsigned)(key & 0xffffffffull) : -1;
    }
}

// ---------------------------------------------------------------------------
// validation (BGPC_STRICT)

__global__ void k_check_sorted(const int *off, const int *idx, int n_rows, int n_cols, int *err)
{
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n_rows; r += gridDim.x * blockDim.x) {
        int b = off[r], e = off[r + 1];
        if (b > e) {
            atomicOr(err, 1);
            continue;
        }
        int prev = -1;
        for (int k = b; k < e; k++) {
            int x = idx[k];
            if (x < 0 || x >= n_cols) atomicOr(err, 1);
            else if (x <= prev) atomicOr(err, 2);
            prev = x;
        }
    }
}

__device__ __forceinline__ bool sorted_contains(const int *idx, int b, int e, int key)
{
    while (b < e) {
        int m = (b + e) >> 1;
        int x = idx[m];
        if (x == key) return true;
        if (x < key) b = m + 1;
        else e = m;
    }
    return false;
}

// every entry (u, v) of `a` appears as (v, u) in `b`; with no_self, u != v
__global__ void k_check_transpose(const int *a_off, const int *a_idx, int n_rows,
                                  const int *b_off, const int *b_idx, int no_self, int *err)
{
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n_rows; u += gridDim.x * blockDim.x) {
        for (int k = a_off[u]; k < a_off[u + 1]; k++) {
            int v = a_idx[k];
            if (no_self && v == u) atomicOr(err, 8);
            if (!sorted_contains(b_idx, b_off[v], b_off[v + 1], u)) atomicOr(err, 4);
        }
    }
}

// resumed colorings: entries must be -1 or a color below the cap
__global__ void k_check_colors(const int *st, int n, int cap, int *err)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int s = st[i];
        if (s < -1 || s >= cap) atomicOr(err, 16);
    }
}

// ---------------------------------------------------------------------------
// masks of colors 0..63 held by the colored members of each net

// Per-net color words.  mask0[v] holds the colors 0..63 of the colored
// members of net v; colors 64 and up, when the driver has allocated them,
// sit net-major in hw: word p of net v (colors 64(p+1) .. 64(p+1)+63) at
// hw[v * PH + p].  Both hold snapshot colors only and are updated by the
// winners of each vertex-based round.
template <bool D2>
__global__ void k_mask_rebuild(Graph g, const int *st, uint64_t *mask0, uint64_t *hw, int PH)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n_b; v += gridDim.x * blockDim.x) {
        uint64_t m = 0;
        int sz = Acc<D2>::size(g, v);
        uint64_t *row = hw ? hw + (long)v * PH : nullptr;
        for (int p = 0; row && p < PH; p++) row[p] = 0;
        for (int k = 0; k < sz; k++) {
            int c = snap_color(st[Acc<D2>::member(g, v, k)]);
            if (c >= 0 && c < 64) m |= 1ull << c;
            else if (c >= 64 && row && (c >> 6) - 1 < PH) row[(c >> 6) - 1] |= 1ull << (c & 63);
        }
        mask0[v] = m;
    }
}

// hw rows of PHo words -> rows of PHn >= PHo words (the new words zero)
__global__ void k_grow_planes(const uint64_t *old, int PHo, uint64_t *neu, int PHn, int n_b)
{
    const long total = (long)n_b * PHn;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        long v = i / PHn;
        int p = (int)(i - v * PHn);
        neu[i] = (p < PHo && old) ? old[v * PHo + p] : 0ull;
    }
}

// Front-driven rounds list the nets to rescan instead of flagging them: a net
// joins the list once per round (stamped with round + 1).
struct DirtyList {
    int *list;   // null: nets are flagged in the dirty bytes instead
    int *n;
    int *stamp;
    int round;
};

// stamps v for this round; true for the one caller that did
__device__ __forceinline__ bool dl_claim(const DirtyList &dl, int v)
{
    return __atomic_load_n(&dl.stamp[v], __ATOMIC_RELAXED) != dl.round + 1 &&
           atomicExch(&dl.stamp[v], dl.round + 1) != dl.round + 1;
}

__device__ __forceinline__ void dl_mark(const DirtyList &dl, int v)
{
    if (dl_claim(dl, v)) dl.list[atomicAdd(dl.n, 1)] = v;
}

// Nets of w, marked for a new scan (standing proposals): w's proposal changed.
template <bool D2>
__device__ __forceinline__ void mark_nets_dirty(const Graph &g, int w, uint8_t *dirty, int first, int step,
                                                const DirtyList *dl = nullptr)
{
    const int nn = Acc<D2>::nets_count(g, w);
    for (int k = first; k < nn; k += step) {
        const int v = Acc<D2>::net_at(g, w, k);
        if (dl && dl->list) dl_mark(*dl, v);
        else dirty[v] = 1;
    }
}

// Smallest color >= from (from >= 64) that no net of w holds, searched one
// 64-color word at a time by one thread; -1 when the search passes the
// allocated words.
template <bool D2>
__device__ int hw_first_free(const Graph &g, int w, const uint64_t *hw, int PH, int from)
{
    const int nn = Acc<D2>::nets_count(g, w);
    for (int p = (from >> 6) - 1; p < PH; p++) {
        uint64_t m = 0;
        for (int k = 0; k < nn; k++) m |= hw[(long)Acc<D2>::net_at(g, w, k) * PH + p];
        if (p == (from >> 6) - 1) m |= (1ull << (from & 63)) - 1ull;
        if (~m) return 64 * (p + 1) + __builtin_ctzll(~m);
    }
    return -1;
}

__global__ void k_max_color(const int *st, int n, Ctrl *ctrl)
{
    int local = -1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        local = max(local, cur_color(st[i]));
    local = wave_max(local);
    if (lane_id() == 0 && local >= 0) {
        max_to(&ctrl->max_color, local);
        max_to(&ctrl->pad[0], local);
    }
}

// ---------------------------------------------------------------------------
// forbidden-color bitmaps built cooperatively by a block (wide path)

// Sets bit c of `bits` for every snapshot color c < cap_bits found among the
// vertices sharing a net with w (w excluded): F(w) of Algorithm 4.  The
// distance-2 neighbourhood is enumerated flat: the sizes of a block-sized
// batch of nets are prefix-summed, then every thread walks the batch's
// members by position.  `s_net`, `s_pre` hold blockDim.x + 1 ints each.
template <bool D2>
__device__ void build_forbidden(const Graph &g, const int *st, int w, uint32_t *bits, int cap_bits,
                                int *s_net, int *s_pre, int *scan_scratch)
{
    const int nt = blockDim.x, tid = threadIdx.x;
    int nn = Acc<D2>::nets_count(g, w);
    for (int base = 0; base < nn; base += nt) {
        int k = base + tid;
        int v = k < nn ? Acc<D2>::net_at(g, w, k) : -1;
        int sz = v >= 0 ? Acc<D2>::size(g, v) : 0;
        int total;
        int ex = block_excl_scan(sz, scan_scratch, &total);
        s_net[tid] = v;
        s_pre[tid] = ex;
        if (tid == 0) s_pre[nt] = total;
        __syncthreads();
        int cnt = min(nt, nn - base);
        for (int f = tid; f < total; f += nt) {
            int lo = 0, hi = cnt - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (s_pre[mid] <= f) lo = mid;
                else hi = mid - 1;
            }
            int x = Acc<D2>::member(g, s_net[lo], f - s_pre[lo]);
            if (x == w) continue;
            int c = snap_color(st[x]);
            if (c >= 0 && c < cap_bits) atomicOr(&bits[c >> 5], 1u << (c & 31));
        }
        __syncthreads();
    }
}

// smallest color >= from that is not in the bitmap (colors >= cap are free)
__device__ int block_find_free_up(const uint32_t *bits, int cap_bits, int from, int *s_res)
{
    const int nt = blockDim.x, tid = threadIdx.x;
    if (from >= cap_bits) return from;
    int nwords = (cap_bits + 31) >> 5;
    int w0 = from >> 5;
    for (int base = w0; base < nwords; base += nt) {
        if (tid == 0) *s_res = 0x7fffffff;
        __syncthreads();
        int wi = base + tid;
        if (wi < nwords) {
            uint32_t free_bits = ~bits[wi];
            if (wi == w0) free_bits &= ~0u << (from & 31);
            if (free_bits) atomicMin(s_res, (wi << 5) + __builtin_ctz(free_bits));
        }
        __syncthreads();
        int r = *s_res;
        __syncthreads();
        if (r != 0x7fffffff) return r;
    }
    return max(from, nwords << 5);
}

// largest color <= from that is not in the bitmap, or -1
__device__ int block_find_free_down(const uint32_t *bits, int cap_bits, int from, int *s_res)
{
    const int nt = blockDim.x, tid = threadIdx.x;
    if (from < 0) return -1;
    if (from >= cap_bits) return from;
    int w0 = from >> 5;
    for (int top = w0; top >= 0; top -= nt) {
        if (tid == 0) *s_res = -1;
        __syncthreads();
        int wi = top - tid;
        if (wi >= 0) {
            uint32_t free_bits = ~bits[wi];
            if (wi == w0) {
                int sh = from & 31;
                free_bits &= (sh == 31) ? ~0u : ((2u << sh) - 1u);
            }
            if (free_bits) atomicMax(s_res, (wi << 5) + 31 - __builtin_clz(free_bits));
        }
        __syncthreads();
        int r = *s_res;
        __syncthreads();
        if (r != -1) return r;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// vertex-based coloring, first-fit

constexpr int COOP_NETS = 256;   // rows longer than this are ORed by the whole wave

// OR of mask0 over the d nets in row[0..d), by the whole wave (eight loads in
// flight per lane); every lane gets the result.
// zf[w] = some net of w holds color 0, from the masks (after a net-based
// round or a resumed start)
template <bool D2>
__global__ void k_zero_front_init(Graph g, const uint64_t *mask0, uint8_t *zf)
{
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < g.n_a; w += gridDim.x * blockDim.x) {
        uint64_t m = D2 ? mask0[w] : 0ull;
        for (int k = g.a_off[w]; k < g.a_off[w + 1] && !(m & 1ull); k++) m |= mask0[g.a_idx[k]];
        zf[w] = (uint8_t)(m & 1ull);
    }
}

__device__ uint64_t wave_row_or(const int *row, int d, const uint64_t *mask0)
{
    const int lane = lane_id();
    uint64_t m = 0;
    for (int k0 = 0; k0 < d; k0 += 8 * WAVE) {
        int nets[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int k = k0 + q * WAVE + lane;
            nets[q] = k < d ? row[k] : -1;
        }
        uint64_t mm[8];
#pragma unroll
        for (int q = 0; q < 8; q++) mm[q] = nets[q] >= 0 ? mask0[nets[q]] : 0ull;
#pragma unroll
        for (int q = 0; q < 8; q++) m |= mm[q];
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) m |= shfl64(m, lane ^ o);
    return m;
}

// One wave per 64 worklist entries: F(w) restricted to colors 0..63 is the OR
// of the masks of w's nets.  The wave first copies the 64 rows of nets(w)
// into LDS as one flat range (coalesced index loads, four in flight per
// lane), then every lane ORs the masks of its own row, eight gathers in
// flight.  The first clear bit is the first-fit color.  Entries whose 64 low
// colors are all forbidden are queued for k_vcolor_wide.
// zf (vertex rounds with standing proposals): zf[w] is set once some net of
// w holds color 0; entries without it whose standing proposal is 0 are
// skipped (first-fit would give 0 again).
// Front mode (FRONT, fl_out set): W is the front list (uncolored vertices whose
// nets hold color 0, unordered, with the last round's winners still in it),
// its length is *n_p; winners are dropped and every other entry is appended
// to fl_out, the next round's front list.
template <bool D2, bool FRONT = false>
__global__ void __launch_bounds__(64) k_vcolor_ff(Graph g, const int *W, Ctrl *ctrl, int par, int *st,
                                                  const uint64_t *mask0, int *heavy, unsigned long long *prof,
                                                  const uint64_t *hw, int PH, int *ffc, uint8_t *dirty,
                                                  const int *n_p = nullptr, int *fl_out = nullptr,
                                                  int *fl_out_n = nullptr,
                                                  DirtyList dl = DirtyList{nullptr, nullptr, nullptr, 0},
                                                  const uint8_t *zf = nullptr)
{
    unsigned long long rows = 0;
    __shared__ int s_pre[65], s_beg[64];
    __shared__ int s_idx[STAGE];
    const int n = n_p ? *n_p : ctrl->n_w[par];
    const int lane = threadIdx.x, nb = gridDim.x, lb = xcd_remap(blockIdx.x, nb);
    const int stride = nb * 64;
    int local_max = -1;
    // the next 64 entries and their row offsets are loaded while the current
    // ones are colored
    int nw_ = -1, nbeg = 0, nend = 0, nst = -1, nffc = 0;
    uint8_t nzf = 1;
    auto fetch = [&](int bs) {
        int i = bs + lane;
        nw_ = i < n ? W[i] : -1;
        if (nw_ >= 0) {
            nbeg = g.a_off[nw_];
            nend = g.a_off[nw_ + 1];
            nffc = ffc[nw_];
            if ((FRONT && fl_out) || (!FRONT && zf)) nst = st[nw_];
            if (!FRONT && zf) nzf = zf[nw_];
        }
    };
    fetch(lb * 64);
    for (int base = lb * 64; base < n; base += stride) {
        int w = nw_;
        // (zf) no net of w holds color 0, so its first-fit answer is 0: a
        // standing proposal 0 stays as it is
        if (!FRONT && zf && w >= 0 && !nzf && nst == TENT) w = -1;
        if (FRONT && fl_out) {
            // front list: last round's winners leave it, the rest stays
            if (w >= 0 && nst >= 0 && !(nst & TENT)) w = -1;
            const uint64_t bal = __ballot(w >= 0);
            int fbase = 0;
            if (lane == 0 && bal) fbase = atomicAdd(fl_out_n, __builtin_popcountll(bal));
            fbase = __shfl(fbase, 0);
            if (w >= 0) fl_out[fbase + __builtin_popcountll(bal & ((1ull << lane) - 1ull))] = w;
        }
        // a vertex of more than 64 nets whose last first-fit answer was 64 or
        // more still has colors 0..63 all forbidden (F only grows in these
        // rounds): its nets' masks are not read, it goes to k_vcolor_wide
        const bool full64 = w >= 0 && nend - nbeg > 64 && nffc >= 64;
        const int beg = w >= 0 ? nbeg : 0, d = (w >= 0 && !full64) ? nend - nbeg : 0;
        fetch(base + stride);
        uint64_t m = 0;
        if (D2 && w >= 0 && !full64) m = mask0[w];
        int incl = wave_incl_scan(d);
        int total = __shfl(incl, 63);
        int pre = incl - d;
        rows += total;
        // the worklist is ascending, so the 64 rows lie in one stretch of the
        // row ids; when that stretch fits, it is copied flat (rows of
        // vertices between worklist entries included), else row by row
        // (the front list is unordered: the stretch starts at the smallest row)
        const int beg0 = wave_min(w >= 0 && d > 0 ? beg : 0x7fffffff);
        const int span = beg0 == 0x7fffffff ? 0 : wave_max(w >= 0 && d > 0 ? beg + d : 0) - beg0;
        const bool flat = span <= STAGE;
        const int sofs = flat ? beg - beg0 : pre;   // lane's row in s_idx
        if (flat) {
            for (int f0 = 0; f0 < span; f0 += 1024) {
                int v[16];
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    int f = f0 + q * 64 + lane;
                    v[q] = f < span ? g.a_idx[beg0 + f] : 0;
                }
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    int f = f0 + q * 64 + lane;
                    if (f < span) s_idx[f] = v[q];
                }
            }
        } else if (total <= STAGE) {
            s_pre[lane] = pre;
            s_beg[lane] = beg;
            __syncthreads();
            for (int f0 = 0; f0 < total; f0 += 1024) {
                int v[16];
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    int f = f0 + q * 64 + lane;
                    v[q] = 0;
                    if (f < total) {
                        int j = row_of(s_pre, f);
                        v[q] = g.a_idx[s_beg[j] + f - s_pre[j]];
                    }
                }
#pragma unroll
                for (int q = 0; q < 16; q++) {
                    int f = f0 + q * 64 + lane;
                    if (f < total) s_idx[f] = v[q];
                }
            }
        }
        __syncthreads();
        const bool staged = flat || total <= STAGE;
        if (staged) {
            for (int k0 = 0; k0 < d; k0 += 16) {
                uint64_t mm[16];
#pragma unroll
                for (int q = 0; q < 16; q++) mm[q] = (k0 + q < d) ? mask0[s_idx[sofs + k0 + q]] : 0ull;
#pragma unroll
                for (int q = 0; q < 16; q++) m |= mm[q];
            }
        } else {
            // rows read in place; rows longer than COOP_NETS are ORed by the
            // whole wave afterwards
            const int dl = d > COOP_NETS ? 0 : d;
            for (int k0 = 0; k0 < dl; k0 += 8) {
                int nets[8];
#pragma unroll
                for (int q = 0; q < 8; q++) nets[q] = (k0 + q < dl) ? g.a_idx[beg + k0 + q] : -1;
                uint64_t mm[8];
#pragma unroll
                for (int q = 0; q < 8; q++) mm[q] = nets[q] >= 0 ? mask0[nets[q]] : 0ull;
#pragma unroll
                for (int q = 0; q < 8; q++) m |= mm[q];
            }
            for (uint64_t bal = __ballot(d > COOP_NETS); bal; bal &= bal - 1) {
                const int j = __builtin_ctzll(bal);
                const uint64_t acc = wave_row_or(g.a_idx + __shfl(beg, j), __shfl(d, j), mask0);
                if (lane == j) m |= acc;
            }
        }
        bool coop_mark = false;   // a long row's nets re-opened by the whole wave
        bool changed = false;     // (front-driven rounds) w's nets go on the dirty list
        if (w >= 0) {
            int col = -1;
            if (full64) {
                // k_vcolor_wide, below
            } else if (~m) {
                col = __builtin_ctzll(~m);
            } else if (PH > 0 && d <= 64) {
                // colors 0..63 all forbidden: the higher words, from the
                // vertex's last first-fit answer (F only grows in these rounds)
                col = hw_first_free<D2>(g, w, hw, PH, max(64, ffc[w]));
                if (col >= 0) ffc[w] = col;
            }
            if (col >= 0) {
                const int nv = TENT | col;
                if (!dirty) {
                    st[w] = nv;
                } else if (st[w] != nv) {
                    // standing proposals: a changed proposal re-opens w's nets
                    st[w] = nv;
                    if (FRONT && dl.list) {
                        changed = true;
                    } else if (staged) {
                        if (D2) dirty[w] = 1;
                        for (int k = 0; k < d; k++) dirty[s_idx[sofs + k]] = 1;
                    } else if (d > COOP_NETS) {
                        if (D2) dirty[w] = 1;
                        coop_mark = true;
                    } else {
                        mark_nets_dirty<D2>(g, w, dirty, 0, 1);
                    }
                }
                local_max = max(local_max, col);
            } else {
                heavy[atomicAdd(&ctrl->n_heavy, 1)] = w;
            }
        }
        for (uint64_t bal = __ballot(coop_mark); bal; bal &= bal - 1) {
            const int j = __builtin_ctzll(bal);
            const int bj = __shfl(beg, j), dj = __shfl(d, j);
            for (int k = lane; k < dj; k += WAVE) dirty[g.a_idx[bj + k]] = 1;
        }
        if (FRONT && dl.list) {
            // the nets of changed proposals onto the dirty list: each lane
            // claims its row's nets (first 32 through a position mask, the
            // rest one by one), one atomic per wave for the slots
            uint64_t newm = 0;
            if (changed) {
                if (D2) dl_mark(dl, w);   // w's own closed neighbourhood
                // the stamps of the first 32 nets read together, then the
                // exchanges of the unstamped ones issued together
                const int r1 = dl.round + 1;
                int vs[32], sv[32];
#pragma unroll
                for (int k = 0; k < 32; k++) vs[k] = k < d ? (staged ? s_idx[sofs + k] : g.a_idx[beg + k]) : -1;
#pragma unroll
                for (int k = 0; k < 32; k++) sv[k] = vs[k] >= 0 ? dl.stamp[vs[k]] : r1;
#pragma unroll
                for (int k = 0; k < 32; k++) sv[k] = sv[k] != r1 ? atomicExch(&dl.stamp[vs[k]], r1) : r1;
#pragma unroll
                for (int k = 0; k < 32; k++)
                    if (sv[k] != r1) newm |= 1ull << k;
                for (int k = 32; k < d; k++) dl_mark(dl, staged ? s_idx[sofs + k] : g.a_idx[beg + k]);
            }
            const int cnt = __builtin_popcountll(newm);
            const int incl = wave_incl_scan(cnt);
            const int tot = __shfl(incl, WAVE - 1);
            if (tot) {
                int dbase = 0;
                if (lane == WAVE - 1) dbase = atomicAdd(dl.n, tot);
                dbase = __shfl(dbase, WAVE - 1) + incl - cnt;
                for (uint64_t t = newm; t; t &= t - 1) {
                    const int k = __builtin_ctzll(t);
                    dl.list[dbase++] = staged ? s_idx[sofs + k] : g.a_idx[beg + k];
                }
            }
        }
        __syncthreads();
    }
    local_max = wave_max(local_max);
    if (lane == 0 && local_max >= 0) max_to(&ctrl->max_color, local_max);
    if (prof && lane == 0 && rows) atomicAdd(&prof[4 * (blockIdx.x & 63) + 2], rows);
}

// Block per queued vertex.  With the higher color words allocated, the block
// ORs the words of all nets of w, eight words per pass from the vertex's last
// first-fit answer; past the allocated words (or without them) it builds the
// full forbidden bitmap in LDS from the distance-2 neighbourhood.  First
// clear bit either way.
template <bool D2>
__global__ void k_vcolor_wide(Graph g, const int *heavy, Ctrl *ctrl, int *st, int lds_bits, IncCtrl *ic,
                              unsigned *aff_bits, int *A, unsigned *tchg_bits, int *tcn, const uint64_t *hw, int PH,
                              int *ffc, uint8_t *dirty, DirtyList dl = DirtyList{nullptr, nullptr, nullptr, 0})
{
    extern __shared__ uint32_t dyn[];
    __shared__ int s_net[1025], s_pre[1025], s_scan[20], s_res;
    __shared__ unsigned long long s_or[8];
    const int nh = ctrl->n_heavy;
    if (nh == 0) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        int w = heavy[h];
        int col = -1;
        if (PH > 0) {
            const int nn = Acc<D2>::nets_count(g, w);
            const int from = max(64, ffc ? ffc[w] : 0);
            for (int p0 = (from >> 6) - 1; p0 < PH && col < 0; p0 += 8) {
                unsigned long long acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                // four nets per thread per step: their ids, then their 32 words, in flight
                for (int k0 = tid; k0 < nn; k0 += 4 * nt) {
                    int vs[4];
#pragma unroll
                    for (int i = 0; i < 4; i++) vs[i] = k0 + i * nt < nn ? Acc<D2>::net_at(g, w, k0 + i * nt) : -1;
                    unsigned long long x[4][8];
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const uint64_t *row = hw + (long)(vs[i] < 0 ? 0 : vs[i]) * PH;
#pragma unroll
                        for (int q = 0; q < 8; q++) x[i][q] = (vs[i] >= 0 && p0 + q < PH) ? row[p0 + q] : 0ull;
                    }
#pragma unroll
                    for (int i = 0; i < 4; i++)
#pragma unroll
                        for (int q = 0; q < 8; q++) acc[q] |= x[i][q];
                }
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    for (int dd = WAVE / 2; dd > 0; dd >>= 1) acc[q] |= shfl64(acc[q], lane_id() ^ dd);
                }
                if (tid < 8) s_or[tid] = 0;
                __syncthreads();
                if (lane_id() == 0)
                    for (int q = 0; q < 8; q++) atomicOr(&s_or[q], acc[q]);
                __syncthreads();
                for (int q = 0; q < 8 && p0 + q < PH; q++) {
                    unsigned long long m = s_or[q];
                    if (q == 0 && p0 == (from >> 6) - 1) m |= (1ull << (from & 63)) - 1ull;
                    if (~m) {
                        col = 64 * (p0 + q + 1) + __builtin_ctzll(~m);
                        break;
                    }
                }
                __syncthreads();
            }
        }
        if (col < 0) {
            int cap = ctrl->max_color + 2;
            if (cap > lds_bits) {
                if (tid == 0) atomicOr(&ctrl->error, ERR_COLOR_CAP);
                return;
            }
            int nwords = (cap + 31) >> 5;
            for (int i = tid; i < nwords; i += nt) dyn[i] = 0;
            __syncthreads();
            build_forbidden<D2>(g, st, w, dyn, cap, s_net, s_pre, s_scan);
            col = block_find_free_up(dyn, cap, 0, &s_res);
        }
        if (dirty) {
            // standing proposals: a changed proposal re-opens w's nets
            const bool changed = st[w] != (TENT | col);
            __syncthreads();
            if (changed) mark_nets_dirty<D2>(g, w, dirty, tid, nt, &dl);
        }
        if (tid == 0) {
            int nw = TENT | col;
            if (ic) {   // incremental rounds: note a changed proposal, join A
                if (st[w] != nw) {
                    st[w] = nw;
                    mark_proposal_change<D2>(g, w, tchg_bits, tcn, ic);
                }
                if (set_once(aff_bits, w)) A[atomicAdd(&ic->n_a, 1)] = w;
            } else {
                st[w] = nw;
            }
            if (ffc) ffc[w] = col;
            max_to(&ctrl->max_color, col);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// vertex-based coloring with the balancing policies (Algorithms 11 and 12)

struct PolicyState {
    int col_max, col_next;
};

__device__ __forceinline__ uint64_t bits_upto(int a)  // bits 0..a
{
    return a >= 63 ? ~0ull : ((1ull << (a + 1)) - 1ull);
}

// Resolve one pick from the 64 low forbidden bits alone; false when the
// answer may depend on colors >= 64.
__device__ __forceinline__ bool pick_low(int policy, uint64_t m, int rank, const PolicyState &s, int *col)
{
    uint64_t fr = ~m;
    if ((policy == 1 || policy == 3) && (rank & 1) == 0) {  // B1 (B1G: col_max fixed), even rank
        if (s.col_max > 63) return false;
        uint64_t low = fr & bits_upto(s.col_max);
        if (low) {
            *col = 63 - __builtin_clzll(low);
            return true;
        }
        uint64_t high = fr & ~bits_upto(s.col_max);
        if (high) {
            *col = __builtin_ctzll(high);
            return true;
        }
        return false;
    }
    if (policy == 2) {  // B2
        if (s.col_next > 63) return false;
        uint64_t z = fr & (~0ull << s.col_next);
        if (!z) return false;
        int c = __builtin_ctzll(z);
        if (c > s.col_max) c = __builtin_ctzll(fr);
        *col = c;
        return true;
    }
    // first-fit (also B1 with an odd rank)
    if (!fr) return false;
    *col = __builtin_ctzll(fr);
    return true;
}

__device__ __forceinline__ int pick_bitmap(int policy, const uint32_t *bits, int cap, int rank, const PolicyState &s,
                                           int *s_res)
{
    if ((policy == 1 || policy == 3) && (rank & 1) == 0) {
        int c = block_find_free_down(bits, cap, s.col_max, s_res);
        if (c == -1) c = block_find_free_up(bits, cap, s.col_max + 1, s_res);
        return c;
    }
    if (policy == 2) {
        int c = block_find_free_up(bits, cap, s.col_next, s_res);
        if (c > s.col_max) c = block_find_free_up(bits, cap, 0, s_res);
        return c;
    }
    return block_find_free_up(bits, cap, 0, s_res);
}

__device__ __forceinline__ void policy_update(int policy, int col, PolicyState &s)
{
    if (policy == 3) return;   // B1G: col_max stays the snapshot's largest color
    s.col_max = max(s.col_max, col);
    if (policy == 2) s.col_next = min(col + 1, s.col_max / 3 + 1);
}

// OR over the nets of w of color word p (p = 0: mask0; p >= 1: hw word
// p - 1), lanes of the wave splitting the nets; every lane gets the result.
template <bool D2>
__device__ uint64_t wave_word_or(const Graph &g, int w, const uint64_t *mask0, const uint64_t *hw, int PH, int p)
{
    const int nn = Acc<D2>::nets_count(g, w);
    uint64_t m = 0;
    for (int k = lane_id(); k < nn; k += WAVE) {
        int v = Acc<D2>::net_at(g, w, k);
        m |= p == 0 ? mask0[v] : hw[(long)v * PH + p - 1];
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) m |= shfl64(m, lane_id() ^ d);
    return m;
}

// The policies' searches over the color words of w (m0: word 0, already
// gathered).  up: smallest free color >= from; down: largest free color
// <= from, or -1 when there is none.  -2: the search needs words beyond the
// allocated ones.
template <bool D2>
__device__ int words_free_up(const Graph &g, int w, uint64_t m0, const uint64_t *mask0, const uint64_t *hw, int PH,
                             int from)
{
    for (int p = from >> 6; p <= PH; p++) {
        uint64_t m = p == 0 ? m0 : wave_word_or<D2>(g, w, mask0, hw, PH, p);
        if (p == (from >> 6)) m |= (1ull << (from & 63)) - 1ull;
        if (~m) return 64 * p + __builtin_ctzll(~m);
    }
    return -2;
}

template <bool D2>
__device__ int words_free_down(const Graph &g, int w, uint64_t m0, const uint64_t *mask0, const uint64_t *hw, int PH,
                               int from)
{
    if (from < 0) return -1;
    if ((from >> 6) > PH) return -2;
    for (int p = from >> 6; p >= 0; p--) {
        uint64_t m = p == 0 ? m0 : wave_word_or<D2>(g, w, mask0, hw, PH, p);
        uint64_t fr = ~m;
        if (p == (from >> 6)) fr &= bits_upto(from & 63);
        if (fr) return 64 * p + 63 - __builtin_clzll(fr);
    }
    return -1;
}

// The same two searches over a precomputed row of words Fw[0..PH] (a vertex
// of many nets), 64 words per step with the whole wave.
__device__ int row_free_up(const uint64_t *Fw, int PH, int from)
{
    const int lane = lane_id();
    for (int pb = from >> 6; pb <= PH; pb += WAVE) {
        const int p = pb + lane;
        uint64_t fr = 0;
        if (p <= PH) {
            uint64_t m = Fw[p];
            if (p == (from >> 6)) m |= (1ull << (from & 63)) - 1ull;
            fr = ~m;
        }
        const uint64_t bal = __ballot(fr != 0);
        if (bal) {
            const int j = __builtin_ctzll(bal);
            return 64 * (pb + j) + __builtin_ctzll(shfl64(fr, j));
        }
    }
    return -2;
}

__device__ int row_free_down(const uint64_t *Fw, int PH, int from)
{
    if (from < 0) return -1;
    if ((from >> 6) > PH) return -2;
    const int lane = lane_id();
    for (int pb = from >> 6; pb >= 0; pb -= WAVE) {
        const int p = pb - lane;
        uint64_t fr = 0;
        if (p >= 0) {
            fr = ~Fw[p];
            if (p == (from >> 6)) fr &= bits_upto(from & 63);
        }
        const uint64_t bal = __ballot(fr != 0);
        if (bal) {
            const int j = __builtin_ctzll(bal);
            return 64 * (pb - j) + 63 - __builtin_clzll(shfl64(fr, j));
        }
    }
    return -1;
}

// The nets of a vertex of at most 2 * WAVE nets held in registers for the
// searches of one pick: lanes form groups of L (a power of two >= the net
// count, at most WAVE); each group ORs one word, WAVE / L words per pass.
struct NetRegs {
    int v0, v1, L;
};

template <bool D2>
__device__ NetRegs load_nets(const Graph &g, int w, int nn)
{
    NetRegs r;
    r.L = 1;
    while (r.L < nn && r.L < WAVE) r.L <<= 1;
    const int k = lane_id() & (r.L - 1);
    r.v0 = k < nn ? Acc<D2>::net_at(g, w, k) : -1;
    r.v1 = (r.L == WAVE && k + WAVE < nn) ? Acc<D2>::net_at(g, w, k + WAVE) : -1;
    return r;
}

// word p (0 <= p <= PH, else 0) of the group's nets, in every lane of the group
__device__ __forceinline__ uint64_t group_word_or(const NetRegs &r, const uint64_t *mask0, const uint64_t *hw, int PH,
                                                  int p)
{
    uint64_t m = 0;
    if (p >= 0 && p <= PH) {
        if (r.v0 >= 0) m |= p == 0 ? mask0[r.v0] : hw[(long)r.v0 * PH + p - 1];
        if (r.v1 >= 0) m |= p == 0 ? mask0[r.v1] : hw[(long)r.v1 * PH + p - 1];
    }
    for (int d = r.L / 2; d > 0; d >>= 1) m |= shfl64(m, lane_id() ^ d);
    return m;
}

__device__ int regs_free_up(const NetRegs &r, uint64_t m0, const uint64_t *mask0, const uint64_t *hw, int PH, int from)
{
    const int lane = lane_id(), G = WAVE / r.L, q = lane / r.L;
    const bool lead = (lane & (r.L - 1)) == 0;
    for (int pb = from >> 6; pb <= PH; pb += G) {
        const int p = pb + q;
        uint64_t m = group_word_or(r, mask0, hw, PH, p);   // every lane: the groups shuffle
        if (p == 0) m = m0;
        if (p == (from >> 6)) m |= (1ull << (from & 63)) - 1ull;
        const uint64_t fr = p <= PH ? ~m : 0ull;
        const uint64_t bal = __ballot(lead && fr != 0);
        if (bal) {
            const int j = __builtin_ctzll(bal);
            return 64 * (pb + j / r.L) + __builtin_ctzll(shfl64(fr, j));
        }
    }
    return -2;
}

__device__ int regs_free_down(const NetRegs &r, uint64_t m0, const uint64_t *mask0, const uint64_t *hw, int PH,
                              int from)
{
    if (from < 0) return -1;
    if ((from >> 6) > PH) return -2;
    const int lane = lane_id(), G = WAVE / r.L, q = lane / r.L;
    const bool lead = (lane & (r.L - 1)) == 0;
    for (int pb = from >> 6; pb >= 0; pb -= G) {
        const int p = pb - q;
        uint64_t m = group_word_or(r, mask0, hw, PH, p);   // every lane: the groups shuffle
        if (p == 0) m = m0;
        uint64_t fr = p >= 0 ? ~m : 0ull;
        if (p == (from >> 6)) fr &= bits_upto(from & 63);
        const uint64_t bal = __ballot(lead && fr != 0);
        if (bal) {
            const int j = __builtin_ctzll(bal);   // lowest lane: highest word
            return 64 * (pb - j / r.L) + 63 - __builtin_clzll(shfl64(fr, j));
        }
    }
    return -1;
}

// One policy pick from the color words (Fw: w's precomputed row, or null);
// -2 when they do not reach far enough.
template <bool D2>
__device__ int pick_words(const Graph &g, int w, uint64_t m0, const uint64_t *mask0, const uint64_t *hw, int PH,
                          int policy, const PolicyState &s, const uint64_t *Fw)
{
    const int nn = Fw ? 0 : Acc<D2>::nets_count(g, w);
    const bool regs = !Fw && nn <= 2 * WAVE;
    NetRegs r = {-1, -1, 1};
    if (regs) r = load_nets<D2>(g, w, nn);
    auto up = [&](int from) {
        return Fw ? row_free_up(Fw, PH, from)
                  : regs ? regs_free_up(r, m0, mask0, hw, PH, from) : words_free_up<D2>(g, w, m0, mask0, hw, PH, from);
    };
    auto down = [&](int from) {
        return Fw ? row_free_down(Fw, PH, from)
                  : regs ? regs_free_down(r, m0, mask0, hw, PH, from)
                         : words_free_down<D2>(g, w, m0, mask0, hw, PH, from);
    };
    if ((policy == 1 || policy == 3) && (w & 1) == 0) {   // B1 / B1G, even rank
        int c = down(s.col_max);
        if (c == -1) c = up(s.col_max + 1);
        return c;
    }
    if (policy == 2) {
        int c = up(s.col_next);
        if (c == -2) return -2;
        if (c > s.col_max) c = up(0);
        return c;
    }
    return up(0);
}

// Vertices of many nets under the balancing policies: their color words are
// ORed over all their nets once per round by the whole device (a wave per
// slice of HEAVY_SLICE nets, lanes over consecutive words of each net's row),
// not by the single wave that walks their chunk.
constexpr int HEAVY_NETS = 128;    // more nets than this: words precomputed
constexpr int HEAVY_SLICE = 256;   // nets per wave of the precomputation

struct HeavySlice {
    int h, k0;   // heavy vertex index, first net of the slice
};

// hid[w] = index of w among the heavy vertices, or -1; hlist[h] = w; slices
// of each heavy vertex's nets.  counts[0] = heavy vertices, counts[1] = slices.
template <bool D2>
__global__ void k_heavy_mark(Graph g, int *hid, int *hlist, HeavySlice *slices, int *counts)
{
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < g.n_a; w += gridDim.x * blockDim.x) {
        const int d = Acc<D2>::nets_count(g, w);
        if (d <= HEAVY_NETS) {
            hid[w] = -1;
            continue;
        }
        const int h = atomicAdd(&counts[0], 1);
        const int k = (d + HEAVY_SLICE - 1) / HEAVY_SLICE;
        const int base = atomicAdd(&counts[1], k);
        hlist[h] = w;
        hid[w] = h;
        for (int j = 0; j < k; j++) slices[base + j] = HeavySlice{h, j * HEAVY_SLICE};
    }
}

// Row h of F (words 0..PH, zeroed before): OR over the nets of heavy vertex
// hlist[h] of word p (mask0 for p = 0, else color word p - 1), for the heavy
// vertices not yet colored.  Words past the largest color so far stay zero.
template <bool D2>
__global__ void __launch_bounds__(256) k_heavy_words(Graph g, const int *st, const int *hlist,
                                                     const HeavySlice *slices, const int *counts,
                                                     const uint64_t *mask0, const uint64_t *hw, int PH,
                                                     const Ctrl *ctrl, uint64_t *F)
{
    constexpr int NWV = 256 / WAVE;
    __shared__ int s_net[NWV][HEAVY_SLICE];
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    const int ns = counts[1];
    const int pmax = min(PH, max(ctrl->max_color, 0) >> 6);
    const int nwv = gridDim.x * NWV;
    for (int sl = blockIdx.x * NWV + wid; sl < ns; sl += nwv) {
        const HeavySlice S = slices[sl];
        const int w = hlist[S.h];
        const int sw = st[w];
        if (sw >= 0 && !(sw & TENT)) continue;   // colored: not in the worklist
        const int cnt = min(HEAVY_SLICE, Acc<D2>::nets_count(g, w) - S.k0);
        for (int k = lane; k < cnt; k += WAVE) s_net[wid][k] = Acc<D2>::net_at(g, w, S.k0 + k);
        wave_sync();
        uint64_t *row = F + (long)S.h * (PH + 1);
        for (int p0 = 0; p0 <= pmax; p0 += WAVE) {
            const int p = p0 + lane;
            uint64_t acc = 0;
            if (p <= pmax) {
                int k = 0;
                for (; k + 8 <= cnt; k += 8) {
                    uint64_t x[8];
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const int v = s_net[wid][k + q];
                        x[q] = p == 0 ? mask0[v] : hw[(long)v * PH + p - 1];
                    }
#pragma unroll
                    for (int q = 0; q < 8; q++) acc |= x[q];
                }
                for (; k < cnt; k++) {
                    const int v = s_net[wid][k];
                    acc |= p == 0 ? mask0[v] : hw[(long)v * PH + p - 1];
                }
            }
            if (acc) atomicOr((unsigned long long *)&row[p], acc);
        }
        wave_sync();
    }
}

// One wave (block of 64) per chunk of `chunk` consecutive worklist entries;
// the policy state runs through the chunk in worklist order.  Lanes compute
// the low masks of 64 entries at a time; an entry whose pick needs colors
// >= 64 searches the higher color words with the whole wave (a vertex of many
// nets in its precomputed row of F), or, past the allocated words, builds its
// full forbidden bitmap with the whole wave.
template <bool D2>
__global__ void __launch_bounds__(64) k_vcolor_chunked(Graph g, const int *W, Ctrl *ctrl, int par, int *st,
                                                        const uint64_t *mask0, int policy, int chunk, int lds_bits,
                                                        const uint64_t *hw, int PH, uint8_t *dirty, const int *hid,
                                                        const uint64_t *F)
{
    extern __shared__ uint32_t dyn[];
    __shared__ int s_net[65], s_pre[65], s_scan[4], s_res;
    const int n = ctrl->n_w[par];
    const int nchunks = (n + chunk - 1) / chunk;
    const int lane = threadIdx.x;
    // B1G: col_max is the largest color of the round's snapshot (the running
    // maximum of the colors kept, final before this launch)
    const int g_max = policy == 3 ? ctrl->pad[0] : 0;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        PolicyState s = {g_max, 0};
        int lo = ch * chunk, hi = min(lo + chunk, n);
        int cap = -1, cmax = -1;
        for (int sub = lo; sub < hi; sub += WAVE) {
            int i = sub + lane;
            int w = -1, h = -1, sw = 0;
            uint64_t m = 0;
            if (i < hi) {
                w = W[i];
                if (dirty) sw = st[w];   // only this wave writes st[w] in this launch
                h = F ? hid[w] : -1;
                if (h >= 0) {
                    m = F[(long)h * (PH + 1)];
                } else {
                    m = D2 ? mask0[w] : 0ull;
                    for (int k = g.a_off[w]; k < g.a_off[w + 1]; k++) m |= mask0[g.a_idx[k]];
                }
            }
            int cnt = min(WAVE, hi - sub);
            for (int j = 0; j < cnt; j++) {
                int wj = __shfl(w, j);
                const int hj = __shfl(h, j);
                uint64_t mj = shfl64(m, j);
                int col;
                if (!pick_low(policy, mj, wj, s, &col)) {
                    col = PH > 0 ? pick_words<D2>(g, wj, mj, mask0, hw, PH, policy, s,
                                                  hj >= 0 ? F + (long)hj * (PH + 1) : nullptr)
                                 : -2;
                    if (col == -2) {
                        if (cap < 0) cap = ctrl->max_color + 2;
                        if (cap > lds_bits) {
                            if (lane == 0) atomicOr(&ctrl->error, ERR_COLOR_CAP);
                            return;
                        }
                        int nwords = (cap + 31) >> 5;
                        for (int q = lane; q < nwords; q += WAVE) dyn[q] = 0;
                        __syncthreads();
                        build_forbidden<D2>(g, st, wj, dyn, cap, s_net, s_pre, s_scan);
                        col = pick_bitmap(policy, dyn, cap, wj, s, &s_res);
                    }
                }
                policy_update(policy, col, s);
                if (dirty) {
                    // standing proposals: a changed proposal re-opens wj's nets
                    const bool changed = __shfl(sw, j) != (TENT | col);
                    if (changed) mark_nets_dirty<D2>(g, wj, dirty, lane, WAVE);
                }
                if (lane == 0) st[wj] = TENT | col;
                cmax = max(cmax, col);
            }
        }
        // colors >= cap count as free in the fallback bitmaps, and cap was read
        // from the largest color of the snapshot: the chunk's own picks need not
        // be visible before it ends
        if (lane == 0 && cmax >= 0) max_to(&ctrl->max_color, cmax);
    }
}

// ---------------------------------------------------------------------------
// net-based coloring (Algorithm 8; Algorithm 9 in distance-2 mode)

// Thread per net of at most SMALL_NET members: the forbidden colors below
// |vtxs(v)| fit in one 64-bit word; only the owner net writes.
// alg 0 (Algorithm 8): the colored members' colors first, then the uncolored
// members in adjacency order take the free colors from |vtxs(v)| - 1 down.
// alg 1 / 2 (Algorithm 6, forward / reverse start): one pass in adjacency
// order, a colored member's color joining F where it stands; a pick is the
// nearest free color from the previous pick (up from 0 / down from
// |vtxs(v)| - 1) and joins F.  Every pick stays inside [0, |vtxs(v)|): at a
// member's turn F holds fewer colors than the members before it.
template <bool D2>
__global__ void k_ncolor_small(Graph g, int *st, const int *owner, Ctrl *ctrl, int alg)
{
    int local_max = -1;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n_b; v += gridDim.x * blockDim.x) {
        int sz = Acc<D2>::size(g, v);
        if (sz == 0 || sz > SMALL_NET) continue;
        if (alg != 0) {
            uint64_t F = 0;
            int col = alg == 1 ? 0 : sz - 1;
            for (int k = 0; k < sz; k++) {
                const int x = Acc<D2>::member(g, v, k);
                const int c = snap_color(st[x]);
                if (c >= 0) {
                    if (c < 64) F |= 1ull << c;
                    continue;
                }
                const uint64_t fr = alg == 1 ? (~F & (~0ull << col)) : (~F & bits_upto(col));
                if (!fr) {
                    atomicOr(&ctrl->error, ERR_REVERSE_NEG);
                    break;
                }
                col = alg == 1 ? __builtin_ctzll(fr) : 63 - __builtin_clzll(fr);
                F |= 1ull << col;
                if (owner[x] == v) {
                    st[x] = TENT | col;
                    local_max = max(local_max, col);
                }
            }
            continue;
        }
        uint64_t F = 0;
        int nun = 0;
        for (int k = 0; k < sz; k++) {
            int c = snap_color(st[Acc<D2>::member(g, v, k)]);
            if (c < 0) {
                nun++;
            } else if (c < sz) {
                if ((F >> c) & 1ull) atomicOr(&ctrl->error, ERR_NET_DUP);
                F |= 1ull << c;
            }
        }
        if (nun == 0) continue;
        int col = sz - 1;
        for (int k = 0; k < sz; k++) {
            int x = Acc<D2>::member(g, v, k);
            if (snap_color(st[x]) >= 0) continue;
            while (col >= 0 && ((F >> col) & 1ull)) col--;
            if (col < 0) atomicOr(&ctrl->error, ERR_REVERSE_NEG);
            if (owner[x] == v) {
                st[x] = TENT | col;
                local_max = max(local_max, col);
            }
            col--;
        }
    }
    local_max = wave_max(local_max);
    if (lane_id() == 0 && local_max >= 0) max_to(&ctrl->max_color, local_max);
}

// Block per net larger than SMALL_NET.  LDS: forbidden bitmap of |vtxs(v)|
// bits and the suffix counts of its free colors per 32-bit word; the p-th
// uncolored member (adjacency order) takes the p-th free color counted from
// the top.
// Algorithm 6 (alg 1 / 2) in a big net: the members' snapshot colors are
// staged blockDim.x at a time and one thread makes the single pass over them
// (the bitmap of [0, |vtxs(v)|) in LDS), since each pick depends on every
// member before it.
template <bool D2>
__global__ void __launch_bounds__(NBIG_BLOCK) k_ncolor_big(Graph g, int *st, const int *owner, const int *big,
                                                           const int *n_big_p, Ctrl *ctrl, int lds_words, int alg)
{
    extern __shared__ uint32_t dyn[];
    __shared__ int s_scan[20];
    __shared__ int s_x[NBIG_BLOCK], s_c[NBIG_BLOCK];
    const int n_big = *n_big_p;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int bi = blockIdx.x; bi < n_big; bi += gridDim.x) {
        int v = big[bi];
        int sz = Acc<D2>::size(g, v);
        int nwords = (sz + 31) >> 5;
        if (2 * nwords + 1 > lds_words) {
            if (tid == 0) atomicOr(&ctrl->error, ERR_NET_TOO_BIG);
            continue;
        }
        uint32_t *bits = dyn;
        int *suf = (int *)(dyn + nwords);
        for (int i = tid; i < nwords; i += nt) bits[i] = 0;
        __syncthreads();
        if (alg != 0) {
            int col = alg == 1 ? 0 : sz - 1;   // meaningful in thread 0 only
            int lmax = -1;
            for (int k0 = 0; k0 < sz; k0 += nt) {
                const int k = k0 + tid;
                const int x = k < sz ? Acc<D2>::member(g, v, k) : -1;
                s_x[tid] = x;
                s_c[tid] = x >= 0 ? snap_color(st[x]) : -2;
                __syncthreads();
                if (tid == 0) {
                    const int cnt = min(nt, sz - k0);
                    for (int j = 0; j < cnt; j++) {
                        const int c = s_c[j];
                        if (c >= 0) {
                            if (c < sz) bits[c >> 5] |= 1u << (c & 31);
                            continue;
                        }
                        if (alg == 1) {
                            while (col < sz && ((bits[col >> 5] >> (col & 31)) & 1u)) col++;
                        } else {
                            while (col >= 0 && ((bits[col >> 5] >> (col & 31)) & 1u)) col--;
                        }
                        if (col < 0 || col >= sz) {
                            atomicOr(&ctrl->error, ERR_REVERSE_NEG);
                            break;
                        }
                        bits[col >> 5] |= 1u << (col & 31);
                        const int xj = s_x[j];
                        if (owner[xj] == v) {
                            st[xj] = TENT | col;
                            lmax = max(lmax, col);
                        }
                    }
                }
                __syncthreads();
            }
            if (tid == 0 && lmax >= 0) max_to(&ctrl->max_color, lmax);
            __syncthreads();
            continue;
        }
        int nun = 0;
        for (int k = tid; k < sz; k += nt) {
            int c = snap_color(st[Acc<D2>::member(g, v, k)]);
            if (c < 0) nun++;
            else if (c < sz) {
                uint32_t old = atomicOr(&bits[c >> 5], 1u << (c & 31));
                if (old & (1u << (c & 31))) atomicOr(&ctrl->error, ERR_NET_DUP);
            }
        }
        nun = block_sum(nun, s_scan);
        if (nun == 0) continue;
        // free colors of word i, restricted to [0, sz); suffix sums from the top word
        int carry = 0;
        for (int top = nwords - 1; top >= 0; top -= nt) {
            int wi = top - tid;
            int cnt = 0;
            if (wi >= 0) {
                uint32_t fr = ~bits[wi];
                int rem = sz - (wi << 5);
                if (rem < 32) fr &= (1u << rem) - 1u;
                cnt = __builtin_popcount(fr);
            }
            int total;
            int ex = block_excl_scan(cnt, s_scan, &total);
            if (wi >= 0) suf[wi] = carry + ex + cnt;   // free colors in words >= wi
            carry += total;
        }
        if (tid == 0) suf[nwords] = 0;
        __syncthreads();
        int local_max = -1;
        int base = 0;
        for (int k0 = 0; k0 < sz; k0 += nt) {
            int k = k0 + tid;
            int x = k < sz ? Acc<D2>::member(g, v, k) : -1;
            int unc = (x >= 0 && snap_color(st[x]) < 0) ? 1 : 0;
            int total;
            int p = base + block_excl_scan(unc, s_scan, &total);
            if (unc && owner[x] == v) {
                // word wi with suf[wi + 1] <= p < suf[wi]
                int lo = 0, hi = nwords - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (suf[mid] > p) lo = mid;
                    else hi = mid - 1;
                }
                int q = p - suf[lo + 1];
                uint32_t fr = ~bits[lo];
                int rem = sz - (lo << 5);
                if (rem < 32) fr &= (1u << rem) - 1u;
                if (p >= suf[0]) {
                    atomicOr(&ctrl->error, ERR_REVERSE_NEG);
                } else {
                    for (int t = 0; t < q; t++) fr &= ~(1u << (31 - __builtin_clz(fr)));
                    int col = (lo << 5) + 31 - __builtin_clz(fr);
                    st[x] = TENT | col;
                    local_max = max(local_max, col);
                }
            }
            base += total;
        }
        local_max = block_max(local_max, s_scan);
        if (tid == 0 && local_max >= 0) max_to(&ctrl->max_color, local_max);
        __syncthreads();
    }
}

// Worklist vertices without any net take color 0 (every policy's pick for an
// empty forbidden set) in net-based rounds.
__global__ void k_ncolor_isolated(Graph g, const int *W, Ctrl *ctrl, int par, int *st)
{
    const int n = ctrl->n_w[par];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int w = W[i];
        if (g.a_off[w + 1] == g.a_off[w]) st[w] = TENT | 0;
    }
}

// Net-based rounds under a balancing policy (BGPC_NET_BALANCE): one wave per
// chunk of `chunk` consecutive net ids, the policy state running through the
// chunk's nets in id order.  Per net with an uncolored member: an LDS bitmap
// of the colored members' snapshot colors below cap = col_max + |vtxs(v)| + 2,
// then the uncolored members in adjacency order each take the policy's pick
// (B1's parity from the net id), which joins the bitmap; only the owner net
// writes the proposal.  No pick reaches cap: F never holds |vtxs(v)| colors,
// so a search that passes col_max (B1 upward, B2's fallback) only happens
// when [0, col_max] is all in F and then lands below |vtxs(v)|; every other
// pick is at most col_max, which therefore stays below
// max(starting col_max, |vtxs(v)|).
template <bool D2>
__global__ void __launch_bounds__(64) k_ncolor_balanced(Graph g, int *st, const int *owner, Ctrl *ctrl, int policy,
                                                         int chunk, int lds_bits)
{
    extern __shared__ uint32_t dyn[];
    __shared__ int s_res;
    const int lane = threadIdx.x;
    const int nch = (g.n_b + chunk - 1) / chunk;
    // B1G: col_max is the snapshot's largest color for the whole round
    const int g_max = policy == 3 ? ctrl->pad[0] : 0;
    int local_max = -1;
    for (int ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        PolicyState s = {g_max, 0};
        const int hi = min(ch * chunk + chunk, g.n_b);
        for (int v = ch * chunk; v < hi; v++) {
            const int sz = Acc<D2>::size(g, v);
            if (sz == 0) continue;
            int nun = 0;
            for (int k = lane; k < sz; k += WAVE) nun += snap_color(st[Acc<D2>::member(g, v, k)]) < 0 ? 1 : 0;
            if (wave_sum(nun) == 0) continue;
            const int cap = max(s.col_max, 0) + sz + 2;
            if (cap > lds_bits) {
                if (lane == 0) atomicOr(&ctrl->error, ERR_COLOR_CAP);
                return;
            }
            const int nwords = (cap + 31) >> 5;
            for (int q = lane; q < nwords; q += WAVE) dyn[q] = 0;
            __syncthreads();
            for (int k = lane; k < sz; k += WAVE) {
                const int c = snap_color(st[Acc<D2>::member(g, v, k)]);
                if (c >= 0 && c < cap) atomicOr(&dyn[c >> 5], 1u << (c & 31));
            }
            __syncthreads();
            for (int k0 = 0; k0 < sz; k0 += WAVE) {
                const int k = k0 + lane;
                const int x = k < sz ? Acc<D2>::member(g, v, k) : -1;
                const bool unc = x >= 0 && snap_color(st[x]) < 0;
                for (uint64_t bal = __ballot(unc); bal; bal &= bal - 1) {
                    const int j = __builtin_ctzll(bal);
                    const int xj = __shfl(x, j);
                    const int col = pick_bitmap(policy, dyn, cap, v, s, &s_res);
                    if (col >= cap) {   // cannot happen (see above); never write past the bitmap
                        if (lane == 0) atomicOr(&ctrl->error, ERR_COLOR_CAP);
                        return;
                    }
                    if (lane == 0) {
                        dyn[col >> 5] |= 1u << (col & 31);
                        if (owner[xj] == v) st[xj] = TENT | col;
                    }
                    __syncthreads();
                    policy_update(policy, col, s);
                    if (owner[xj] == v) local_max = max(local_max, col);
                }
            }
        }
    }
    if (lane == 0 && local_max >= 0) max_to(&ctrl->max_color, local_max);
}

// ---------------------------------------------------------------------------
// removal: per net, every holder of a color except its lowest-ranked one loses

// members of a net in ascending rank; distance-2 merges the center into the
// sorted neighbour list
template <bool D2>
struct RankIter {
    const int *idx;
    int pos, end, center;
    bool center_pending;
    __device__ RankIter(const Graph &g, int v)
    {
        idx = g.b_idx;
        pos = g.b_off[v];
        end = g.b_off[v + 1];
        center = v;
        center_pending = D2;
    }
    __device__ __forceinline__ bool next(int *x)
    {
        int nx = pos < end ? idx[pos] : 0x7fffffff;
        if (D2 && center_pending && center < nx) {
            center_pending = false;
            *x = center;
            return true;
        }
        if (pos < end) {
            *x = nx;
            pos++;
            return true;
        }
        return false;
    }
};

// Scan of one net of at most SMALL_NET members in rank order (distance-2:
// the center merged in at its rank); src[k - rel] is entry k of the net
// lists.  The first holder of a color keeps it.  Colors below 64 use a bit
// set; larger colors are compared pairwise against earlier members.  States
// are gathered SCAN_BATCH members at a time.  Returns the number of members still
// uncolored or proposed (0: the net is finished).
//
// Standing proposals (vertex-based rounds): a loser keeps its proposal into
// the next round, and a net is scanned again only when one of its members'
// proposals changed (the net is "dirty").  Every other net's verdict carries
// over: lbits holds one bit per (net, member position), set when that member
// loses in that net, and lcnt[u] counts the nets in which u loses; a scan
// updates both for the positions whose verdict changed.  u loses the round
// iff lcnt[u] > 0 -- the same verdict as a full scan, since a net's verdict
// depends only on its members' proposals.
struct SPState {
    unsigned long long *lbits;   // bit of position p of net v at lpos(v) + p
    int *lcnt;
    uint8_t *dirty;
    // nets above SMALL_NET (optional): the positions of the members still
    // uncolored or proposing, at lpos(v) .. lpos(v) + pn[v] - 1, in any
    // order.  A member colored in a vertex-based round stays colored, so
    // each scan keeps only the pending ones and later scans read fewer.
    int *pl;
    int *pn;
};

// first position of net v in lbits (distance-2 nets hold one more member)
template <bool D2>
__device__ __forceinline__ long sp_lpos(const Graph &g, int v)
{
    return (long)g.b_off[v] + (D2 ? v : 0);
}

// verdict of one position; only the calling thread changes this bit
__device__ __forceinline__ void sp_set(const SPState &sp, long pos, int x, bool lost)
{
    unsigned long long *wd = sp.lbits + (pos >> 6);
    const unsigned long long bit = 1ull << (pos & 63);
    const bool old = (__atomic_load_n(wd, __ATOMIC_RELAXED) & bit) != 0;
    if (old != lost) {
        atomicXor(wd, bit);
        atomicAdd(&sp.lcnt[x], lost ? 1 : -1);
    }
}

// Column-major copy of the first ELL_W members of every net: member p of
// net v at ell[p * n_b + v] (-1 past the net's size).  Lanes that scan
// neighbouring nets then read neighbouring words at every position, where
// the row-major lists put each lane on its own cache line.  Members past
// ELL_W come from the row-major lists.
constexpr int ELL_W = 32;
struct EllSrc {
    const int *ell, *idx;   // ell: this net's column (ell + v)
    int n_b, b, w;          // w * n_b < 2^31
    __device__ __forceinline__ int operator[](int k) const
    {
        const int p = k - b;
        return p < w ? ell[p * n_b] : idx[k];
    }
};

// a wave per 64 nets: their first w members gathered net by net into LDS
// (neighbouring lanes read neighbouring members), then written position by
// position (neighbouring lanes write neighbouring nets)
constexpr int ELL_BLOCK = 256;
__global__ void __launch_bounds__(ELL_BLOCK) k_build_ell(Graph g, int w, int *ell)
{
    constexpr int NW = ELL_BLOCK / WAVE;
    __shared__ int s_t[NW][WAVE * ELL_W];
    __shared__ int s_b[NW][WAVE], s_d[NW][WAVE];
    const int wid = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    for (int v0 = (blockIdx.x * NW + wid) * WAVE; v0 < g.n_b; v0 += gridDim.x * NW * WAVE) {
        const int v = v0 + lane;
        int b = 0, d = 0;
        if (v < g.n_b) {
            b = g.b_off[v];
            d = min(g.b_off[v + 1] - b, w);
        }
        s_b[wid][lane] = b;
        s_d[wid][lane] = d;
        wave_sync();
        for (int f0 = 0; f0 < WAVE * w; f0 += 8 * WAVE) {
            int x[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int f = f0 + q * WAVE + lane;
                const bool in = f < WAVE * w;
                const int j = in ? f / w : 0, p = f - j * w;
                x[q] = (in && p < s_d[wid][j]) ? g.b_idx[s_b[wid][j] + p] : -1;
            }
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int f = f0 + q * WAVE + lane;
                if (f < WAVE * w) s_t[wid][f] = x[q];
            }
        }
        wave_sync();
        if (v < g.n_b)
            for (int p = 0; p < w; p++) ell[p * g.n_b + v] = s_t[wid][lane * w + p];
        wave_sync();
    }
}

constexpr int SCAN_BATCH = 16;   // member states gathered per batch (all in flight)
template <bool D2, class Src>
__device__ __forceinline__ int scan_net(int v, int b, int e, Src src, int rel, const int *st, uint8_t *lose,
                                        int tent_only, const SPState *sp, long lpos)
{
    const int size = e - b + (D2 ? 1 : 0);
    int cpos = size;   // rank position of the center (distance-2)
    if (D2) {
        int lo = b, hi = e;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (src[mid - rel] < v) lo = mid + 1;
            else hi = mid;
        }
        cpos = lo - b;
    }
    auto member = [&](int p) {
        if (!D2) return (int)src[b + p - rel];
        if (p < cpos) return (int)src[b + p - rel];
        if (p == cpos) return v;
        return (int)src[b + p - 1 - rel];
    };
    // stored verdicts of this net's positions, loaded before the members
    // (size <= 64: at most two words; only this thread changes these bits)
    unsigned long long a0 = 0, a1 = 0;
    const long w0 = lpos >> 6;
    const int sh = (int)(lpos & 63);
    if (sp) {
        a0 = __atomic_load_n(&sp->lbits[w0], __ATOMIC_RELAXED);
        if (sh + size > 64) a1 = __atomic_load_n(&sp->lbits[w0 + 1], __ATOMIC_RELAXED);
    }
    uint64_t seen = 0, lm = 0;   // lm: positions that lose (standing proposals)
    bool wide = false;
    int pending = 0;
    for (int p0 = 0; p0 < size; p0 += SCAN_BATCH) {
        int xs[SCAN_BATCH], ss[SCAN_BATCH];
#pragma unroll
        for (int q = 0; q < SCAN_BATCH; q++) xs[q] = (p0 + q < size) ? member(p0 + q) : -1;
#pragma unroll
        for (int q = 0; q < SCAN_BATCH; q++) ss[q] = xs[q] >= 0 ? st[xs[q]] : 0;
#pragma unroll
        for (int q = 0; q < SCAN_BATCH; q++) {
            int x = xs[q], s = ss[q];
            if (x < 0) continue;
            if (s < 0) {
                pending++;
                continue;
            }
            bool tent = (s & TENT) != 0;
            pending += tent;
            if (tent_only && !tent) continue;
            int c = s & COLOR_MASK;
            if (c < 64) {
                if ((seen >> c) & 1ull) {
                    if (sp) lm |= 1ull << (p0 + q);
                    else lose[x] = 1;
                }
                seen |= 1ull << c;
            } else {
                wide = true;
            }
        }
    }
    if (wide) {
        // pairwise for colors >= 64, in rank order
        for (int p = 0; p < size; p++) {
            int x = member(p);
            int s = st[x];
            if (s < 0 || (tent_only && !(s & TENT))) continue;
            int c = s & COLOR_MASK;
            if (c < 64) continue;
            for (int p2 = 0; p2 < p; p2++) {
                int t = st[member(p2)];
                if (t < 0 || (tent_only && !(t & TENT))) continue;
                if ((t & COLOR_MASK) == c) {
                    if (sp) lm |= 1ull << p;
                    else lose[x] = 1;
                    break;
                }
            }
        }
    }
    if (sp) {
        // changed verdicts against the stored bits
        unsigned long long old = (a0 >> sh) | (sh ? (a1 << (64 - sh)) : 0ull);
        if (size < 64) old &= (1ull << size) - 1ull;
        unsigned long long chg = old ^ lm;
        if (chg) {
            atomicXor(&sp->lbits[w0], chg << sh);
            if (sh + size > 64) atomicXor(&sp->lbits[w0 + 1], chg >> (64 - sh));
            for (unsigned long long m = chg; m; m &= m - 1) {
                int p = __builtin_ctzll(m);
                atomicAdd(&sp->lcnt[member(p)], ((lm >> p) & 1ull) ? 1 : -1);
            }
        }
    }
    return pending;
}

// scan_net over the pending list of a net of at most SMALL_NET members
// (standing proposals; positions in rank order, the distance-2 center merged
// at its rank): only the listed members are read, and the list keeps, in
// order, those still pending.  Colored members take no part in a
// vertex-based round's removal and carry no verdict bits, so the verdicts
// equal scan_net's.  Returns the number of members still pending.
template <bool D2>
__device__ __forceinline__ int scan_net_list(const Graph &g, int v, int b, int e, const int *st, const SPState &sp,
                                             long lpos)
{
    const int *src = g.b_idx;
    const int size = e - b + (D2 ? 1 : 0);
    int cpos = size;
    if (D2) {
        int lo = b, hi = e;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (src[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        cpos = lo - b;
    }
    auto member = [&](int p) {
        if (!D2) return src[b + p];
        if (p < cpos) return src[b + p];
        if (p == cpos) return v;
        return src[b + p - 1];
    };
    const long w0 = lpos >> 6;
    const int sh = (int)(lpos & 63);
    unsigned long long a0 = __atomic_load_n(&sp.lbits[w0], __ATOMIC_RELAXED);
    unsigned long long a1 = sh + size > 64 ? __atomic_load_n(&sp.lbits[w0 + 1], __ATOMIC_RELAXED) : 0ull;
    const int np = sp.pn[v];
    uint64_t seen = 0, lm = 0;
    bool wide = false;
    int kept = 0;
    for (int k0 = 0; k0 < np; k0 += SCAN_BATCH) {
        int ps[SCAN_BATCH], xs[SCAN_BATCH], ss[SCAN_BATCH];
#pragma unroll
        for (int q = 0; q < SCAN_BATCH; q++) ps[q] = k0 + q < np ? sp.pl[lpos + k0 + q] : -1;
#pragma unroll
        for (int q = 0; q < SCAN_BATCH; q++) xs[q] = ps[q] >= 0 ? member(ps[q]) : -1;
#pragma unroll
        for (int q = 0; q < SCAN_BATCH; q++) ss[q] = xs[q] >= 0 ? st[xs[q]] : 0;
#pragma unroll
        for (int q = 0; q < SCAN_BATCH; q++) {
            if (xs[q] < 0) continue;
            const int s = ss[q];
            // in place: every entry up to k0 + q has been read
            if (s < 0 || (s & TENT)) sp.pl[lpos + kept++] = ps[q];
            if (!(s >= 0 && (s & TENT))) continue;
            const int c = s & COLOR_MASK;
            if (c < 64) {
                if ((seen >> c) & 1ull) lm |= 1ull << ps[q];
                seen |= 1ull << c;
            } else {
                wide = true;
            }
        }
    }
    if (wide) {
        // pairwise for colors >= 64 over the kept list, in rank order
        for (int k = 0; k < kept; k++) {
            const int p = sp.pl[lpos + k];
            const int s = st[member(p)];
            if (!(s >= 0 && (s & TENT))) continue;
            const int c = s & COLOR_MASK;
            if (c < 64) continue;
            for (int k2 = 0; k2 < k; k2++) {
                const int t = st[member(sp.pl[lpos + k2])];
                if (t >= 0 && (t & TENT) && (t & COLOR_MASK) == c) {
                    lm |= 1ull << p;
                    break;
                }
            }
        }
    }
    unsigned long long old = (a0 >> sh) | (sh ? (a1 << (64 - sh)) : 0ull);
    if (size < 64) old &= (1ull << size) - 1ull;
    const unsigned long long chg = old ^ lm;
    if (chg) {
        atomicXor(&sp.lbits[w0], chg << sh);
        if (sh + size > 64) atomicXor(&sp.lbits[w0 + 1], chg >> (64 - sh));
        for (unsigned long long m = chg; m; m &= m - 1) {
            const int p = __builtin_ctzll(m);
            atomicAdd(&sp.lcnt[member(p)], ((lm >> p) & 1ull) ? 1 : -1);
        }
    }
    sp.pn[v] = kept;
    return kept;
}

// One wave per 64 consecutive nets of at most SMALL_NET members.  The wave
// copies its stretch of the net lists into LDS with coalesced loads, then
// every lane scans its own net.  Nets whose members were all colored at an
// earlier round are marked done (1) and skipped: no vertex can join them
// again until a net-based round evicts (the driver then clears the marks).
// Nets with one member still pending are marked 2: no clash can arise in
// them in vertex-based rounds, which skip them too; net-based rounds scan
// them.  With tent_only, only proposed colors take part (after a
// vertex-based round no colored vertex can clash).
// Standing proposals (SP): only dirty nets are scanned.  The wave reads the
// flags and row offsets of SP_PF of its stretches at once (coalesced, all in
// flight), queues the dirty nets with their offsets in LDS and scans them 64
// at a time, one net per lane, members read straight from the net lists.
constexpr int SP_PF = 4;
constexpr int SP_Q = 64 * SP_PF + 64;   // queue entries: the rest of a drain plus SP_PF stretches
template <bool D2, bool ELLS, bool LISTS>
__device__ void conflict_dirty(const Graph &g, const int *st, uint8_t *done, const SPState &sp, int lb, int nb,
                               int *qv, int *qb, int *qe, int &walked_nets, int &scanned_members, const int *ell,
                               int ell_w)
{
    const int lane = threadIdx.x, stride = nb * 64;
    int qn = 0;
    // scans queue entries off .. off + cnt - 1, one net per lane
    auto drain = [&](int off, int cnt) {
        const int v = lane < cnt ? qv[off + lane] : -1;
        if (v >= 0) {
            const int b = qb[off + lane], e = qe[off + lane];
            const int sz = e - b + (D2 ? 1 : 0);
            if (sz >= 2 && sz <= SMALL_NET) {
                const long lpos = (long)b + (D2 ? v : 0);
                int pending;
                if constexpr (ELLS)
                    pending = scan_net<D2>(v, b, e, EllSrc{ell + v, g.b_idx, g.n_b, b, ell_w}, 0, st, nullptr, 1, &sp,
                                           lpos);
                else if constexpr (LISTS)
                    pending = scan_net_list<D2>(g, v, b, e, st, sp, lpos);
                else
                    pending = scan_net<D2>(v, b, e, g.b_idx, 0, st, nullptr, 1, &sp, lpos);
                // at most one member still pending: no clash can arise in
                // this net in later vertex-based rounds (marked 2: skipped
                // there, scanned again by net-based rounds)
                if (pending <= 1) done[v] = pending == 0 ? 1 : 2;
                scanned_members += sz;
                walked_nets++;
            }
            if (sz <= SMALL_NET) sp.dirty[v] = 0;   // larger nets: k_conflict_big
        }
    };
    for (int base0 = lb * 64; base0 < g.n_b; base0 += SP_PF * stride) {
        uint8_t fd[SP_PF], fn[SP_PF];
        int ob[SP_PF], oe[SP_PF];
#pragma unroll
        for (int k = 0; k < SP_PF; k++) {
            const int v = base0 + k * stride + lane;
            const bool in = v < g.n_b;
            fd[k] = in ? sp.dirty[v] : 0;
            fn[k] = in ? done[v] : 1;
            ob[k] = in ? g.b_off[v] : 0;
            oe[k] = in ? g.b_off[v + 1] : 0;
        }
        // the dirty nets of the SP_PF stretches onto the queue (qn < 64 here)
#pragma unroll
        for (int k = 0; k < SP_PF; k++) {
            const bool d = fd[k] && !fn[k];
            const uint64_t bal = __ballot(d);
            if (d) {
                const int r = qn + __builtin_popcountll(bal & ((1ull << lane) - 1ull));
                qv[r] = base0 + k * stride + lane;
                qb[r] = ob[k];
                qe[r] = oe[k];
            }
            qn += __builtin_popcountll(bal);
        }
        __syncthreads();
        int qs = 0;
        for (; qn - qs >= 64; qs += 64) drain(qs, 64);
        // the rest (fewer than 64) to the front of the queue
        const int rest = qn - qs;
        int kv = 0, kb = 0, ke = 0;
        if (lane < rest) {
            kv = qv[qs + lane];
            kb = qb[qs + lane];
            ke = qe[qs + lane];
        }
        __syncthreads();
        if (lane < rest) {
            qv[lane] = kv;
            qb[lane] = kb;
            qe[lane] = ke;
        }
        qn = rest;
        __syncthreads();
    }
    if (qn > 0) drain(0, qn);
}

template <bool D2, bool SP = false, bool ELLS = false, bool LISTS = false>
__global__ void __launch_bounds__(64) k_conflict_small(Graph g, const int *st, uint8_t *lose, uint8_t *done,
                                                       int tent_only, unsigned long long *prof, SPState sp,
                                                       const int *ell = nullptr, int ell_w = 0)
{
    int walked_nets = 0, walked_members = 0;
    const int lane = threadIdx.x, nb = gridDim.x, lb = xcd_remap(blockIdx.x, nb);
    const int stride = nb * 64;
    if constexpr (SP) {
        // the round's nets are counted by k_census (profiling only)
        __shared__ int q[3][SP_Q];
        int scanned = 0;
        conflict_dirty<D2, ELLS, LISTS>(g, st, done, sp, lb, nb, q[0], q[1], q[2], walked_nets, scanned, ell, ell_w);
        if (prof) {
            int ws = wave_sum(scanned);
            if (lane == 0 && ws) atomicAdd(&prof[4 * (blockIdx.x & 63) + 3], (unsigned long long)ws);
        }
        return;
    } else {
        __shared__ int s_idx[STAGE];
        // the next stretch's offsets and flags are loaded while the current one
        // is scanned
        int nb_ = 0, ne_ = 0, noff0 = 0, noffe = 0;
        uint8_t nskip = 1;
        auto fetch = [&](int bs) {
            if (bs >= g.n_b) return;
            int v = bs + lane;
            if (v < g.n_b) {
                nb_ = g.b_off[v];
                ne_ = g.b_off[v + 1];
                nskip = tent_only ? done[v] : (uint8_t)(done[v] == 1);
            }
            noff0 = g.b_off[bs];
            noffe = g.b_off[min(bs + 64, g.n_b)];
        };
        fetch(lb * 64);
        for (int base = lb * 64; base < g.n_b; base += stride) {
            const int v = base + lane;
            const int b = nb_, e = ne_, off0 = noff0, seg = noffe - noff0;
            const uint8_t skip = nskip;
            fetch(base + stride);
            bool act = false;
            if (v < g.n_b) {
                int sz = e - b + (D2 ? 1 : 0);
                act = sz >= 2 && sz <= SMALL_NET && !skip;
            }
            if (!__ballot(act)) continue;
            bool staged = seg <= STAGE;
            if (staged) {
                // every load of the stretch in flight before the first LDS store
                int v32[STAGE / 64];
    #pragma unroll
                for (int q = 0; q < STAGE / 64; q++) {
                    int f = q * 64 + lane;
                    v32[q] = f < seg ? g.b_idx[off0 + f] : 0;
                }
    #pragma unroll
                for (int q = 0; q < STAGE / 64; q++) {
                    int f = q * 64 + lane;
                    if (f < seg) s_idx[f] = v32[q];
                }
            }
            __syncthreads();
            if (act) {
                const long lpos = (long)b + (D2 ? v : 0);
                int pending = staged ? scan_net<D2>(v, b, e, (const int *)s_idx, off0, st, lose, tent_only, nullptr, lpos)
                                     : scan_net<D2>(v, b, e, g.b_idx, 0, st, lose, tent_only, nullptr, lpos);
                if (pending == 0) done[v] = 1;
            }
            walked_nets += act ? 1 : 0;
            walked_members += act ? e - b + (D2 ? 1 : 0) : 0;
            __syncthreads();
        }
        if (prof) {
            int wn = wave_sum(walked_nets), wm = wave_sum(walked_members);
            if (lane == 0 && wn) {
                atomicAdd(&prof[4 * (blockIdx.x & 63) + 0], (unsigned long long)wn);
                atomicAdd(&prof[4 * (blockIdx.x & 63) + 1], (unsigned long long)wm);
                atomicAdd(&prof[4 * (blockIdx.x & 63) + 3], (unsigned long long)wm);
            }
        }
    }
}

// Removal in front-driven rounds: the nets listed dirty by this round's
// coloring (every net in the first round), one lane per net, scanned as in
// k_conflict_small's standing-proposal path.
constexpr int LIST_BLOCK = 256;
template <bool D2>
__global__ void __launch_bounds__(LIST_BLOCK) k_conflict_list(Graph g, const int *st, uint8_t *done, SPState sp,
                                                              const int *list, const int *n_p,
                                                              unsigned long long *prof)
{
    const int n = *n_p;
    int scanned = 0;
    for (int i = blockIdx.x * LIST_BLOCK + threadIdx.x; i < n; i += gridDim.x * LIST_BLOCK) {
        const int v = list[i];
        const int b = g.b_off[v], e = g.b_off[v + 1];
        const int sz = e - b + (D2 ? 1 : 0);
        if (sz >= 2 && sz <= SMALL_NET) {
            const int pending = scan_net<D2>(v, b, e, g.b_idx, 0, st, nullptr, 1, &sp, (long)b + (D2 ? v : 0));
            if (pending == 0) done[v] = 1;
            scanned += sz;
        }
    }
    if (prof) {
        const int ws = wave_sum(scanned);
        if (lane_id() == 0 && ws) atomicAdd(&prof[4 * (blockIdx.x & 63) + 3], (unsigned long long)ws);
    }
}

// Profiling only (launched after the timed removal launch): the round's nets
// of at most SMALL_NET members -- those with a member still uncolored or
// proposed -- and their sizes, the units the removal step is responsible for.
template <bool D2>
__global__ void k_census(Graph g, const int *st, unsigned long long *prof)
{
    int nets = 0, mem = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n_b; v += gridDim.x * blockDim.x) {
        const int sz = Acc<D2>::size(g, v);
        if (sz < 2 || sz > SMALL_NET) continue;
        bool open = false;
        for (int k0 = 0; k0 < sz && !open; k0 += SCAN_BATCH) {
            int ss[SCAN_BATCH];
#pragma unroll
            for (int j = 0; j < SCAN_BATCH; j++) ss[j] = k0 + j < sz ? st[Acc<D2>::member(g, v, k0 + j)] : 0;
#pragma unroll
            for (int j = 0; j < SCAN_BATCH; j++) open = open || ss[j] < 0 || (ss[j] & TENT);
        }
        if (open) {
            nets++;
            mem += sz;
        }
    }
    int wn = wave_sum(nets), wm = wave_sum(mem);
    if (lane_id() == 0 && wn) {
        atomicAdd(&prof[4 * (blockIdx.x & 63) + 0], (unsigned long long)wn);
        atomicAdd(&prof[4 * (blockIdx.x & 63) + 1], (unsigned long long)wm);
    }
}

__device__ __forceinline__ unsigned hash_color(int c) { return (unsigned)c * 2654435761u; }

// Block per net larger than SMALL_NET.  Nets up to HASH_MAX members use an
// LDS hash color -> lowest-ranked holder; larger nets sweep the colors in
// windows of WIN_COLORS with a direct-mapped table.
constexpr int BIG_BLOCK = 256;                          // threads of k_conflict_big
constexpr int BIG_PER_THREAD = HASH_MAX / BIG_BLOCK;    // members per thread of a hashed net
constexpr int BIG_LIST = 2048;   // proposals of a larger net resolved by the hash (3 + 4 ints each in LDS)
static_assert(3 * BIG_LIST + 2 * (2 * BIG_LIST) <= WIN_COLORS && (BIG_LIST & (BIG_LIST - 1)) == 0 && 2 * (2 * HASH_MAX) <= WIN_COLORS,
              "k_conflict_big's LDS layouts fit its WIN_COLORS-int allocation");
// Removal in one net larger than HASH_MAX, by the whole block.  One pass
// (four members per thread in flight) counts the pending members and, when
// only proposals take part, lists them in LDS; up to list_cap of them (a
// power of two; 7 ints each) are resolved with an LDS hash color -> lowest
// holder, otherwise the colors are swept in windows of WIN_COLORS.  sh holds
// max(7 * list_cap, WIN_COLORS) ints.
template <bool D2>
__device__ void conflict_large(const Graph &g, const int *st, uint8_t *lose, uint8_t *done, int v, int sz, long lpos,
                               int tent_only, const SPState &sp, int *sh, int list_cap, int maxc, int *s_scan,
                               int *s_cnt, int *s_keep)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    int *lst = sh;                      // (position, member, color) per proposal
    int *hsh = sh + 3 * list_cap;       // hash of the listed proposals
    const bool plm = sp.pl != nullptr && tent_only;
    const int np = plm ? sp.pn[v] : sz;
    if (tid == 0) {
        *s_cnt = 0;
        *s_keep = 0;
    }
    __syncthreads();
    int pending = 0;
    for (int base = 0; base < np; base += 4 * nt) {
        int ps[4], xs[4], ss[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int k = base + tid + i * nt;
            ps[i] = k < np ? (plm ? sp.pl[lpos + k] : k) : -1;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) xs[i] = ps[i] >= 0 ? Acc<D2>::member(g, v, ps[i]) : -1;
#pragma unroll
        for (int i = 0; i < 4; i++) ss[i] = xs[i] >= 0 ? st[xs[i]] : 0;
        bool keep[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            keep[i] = false;
            if (xs[i] < 0) continue;
            const int s = ss[i];
            keep[i] = s < 0 || (s & TENT);
            pending += keep[i] ? 1 : 0;
            if (tent_only && s >= 0 && (s & TENT)) {
                const int q = atomicAdd(s_cnt, 1);
                if (q < list_cap) {
                    lst[3 * q] = ps[i];
                    lst[3 * q + 1] = xs[i];
                    lst[3 * q + 2] = cur_color(s);
                }
            }
        }
        if (plm) {
            // this stretch read by every thread: its pending positions go to
            // the front of the list (never past entries not yet read)
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; i++)
                if (keep[i]) sp.pl[lpos + atomicAdd(s_keep, 1)] = ps[i];
        }
    }
    pending = block_sum(pending, s_scan);
    if (plm && tid == 0) sp.pn[v] = pending;
    if (sp.lbits && tid == 0) sp.dirty[v] = 0;
    if (pending == 0) {
        if (tid == 0) done[v] = 1;
        return;
    }
    const int nl = *s_cnt;
    if (tent_only && nl <= list_cap) {
        int cap = 64;
        while (cap < 2 * nl) cap <<= 1;
        int *keys = hsh, *minr = hsh + cap;
        for (int i = tid; i < cap; i += nt) {
            keys[i] = -1;
            minr[i] = 0x7fffffff;
        }
        __syncthreads();
        for (int q = tid; q < nl; q += nt) {
            const int x = lst[3 * q + 1], c = lst[3 * q + 2];
            unsigned h = hash_color(c) & (cap - 1);
            for (;;) {
                int prev = atomicCAS(&keys[h], -1, c);
                if (prev == -1 || prev == c) {
                    atomicMin(&minr[h], x);
                    break;
                }
                h = (h + 1) & (cap - 1);
            }
        }
        __syncthreads();
        for (int q = tid; q < nl; q += nt) {
            const int k = lst[3 * q], x = lst[3 * q + 1], c = lst[3 * q + 2];
            unsigned h = hash_color(c) & (cap - 1);
            while (keys[h] != c) h = (h + 1) & (cap - 1);
            if (sp.lbits) sp_set(sp, lpos + k, x, minr[h] != x);
            else if (minr[h] != x) lose[x] = 1;
        }
        __syncthreads();
        return;
    }
    // more proposals than the list holds: windows of WIN_COLORS colors, over
    // the pending positions (all positions without pending lists)
    const int nk = plm ? pending : sz;
    for (int base = 0; base <= maxc; base += WIN_COLORS) {
        for (int i = tid; i < WIN_COLORS; i += nt) sh[i] = 0x7fffffff;
        __syncthreads();
        for (int k = tid; k < nk; k += nt) {
            const int p = plm ? sp.pl[lpos + k] : k;
            int x = Acc<D2>::member(g, v, p);
            int s = st[x];
            if (tent_only && !(s >= 0 && (s & TENT))) continue;
            int c = cur_color(s) - base;
            if (c >= 0 && c < WIN_COLORS) atomicMin(&sh[c], x);
        }
        __syncthreads();
        for (int k = tid; k < nk; k += nt) {
            const int p = plm ? sp.pl[lpos + k] : k;
            int x = Acc<D2>::member(g, v, p);
            int s = st[x];
            if (tent_only && !(s >= 0 && (s & TENT))) continue;
            int c = cur_color(s) - base;
            if (c >= 0 && c < WIN_COLORS) {
                if (sp.lbits) sp_set(sp, lpos + p, x, sh[c] != x);
                else if (sh[c] != x) lose[x] = 1;
            }
        }
        __syncthreads();
    }
}

// A net whose pending members fit one wave (pending lists, vertex-based
// rounds): lane l takes the l-th listed position; a proposer loses iff a
// proposer of lower rank in the net proposes the same color (compared lane
// by lane through shuffles).  The list keeps the pending positions.
template <bool D2>
__device__ void wave_pending_net(const Graph &g, const int *st, uint8_t *done, const SPState &sp, int v, long lpos,
                                 int np)
{
    const int lane = lane_id();
    int p = -1, x = 0x7fffffff, s = -1;
    if (lane < np) {
        p = sp.pl[lpos + lane];
        x = Acc<D2>::member(g, v, p);
        s = st[x];
    }
    const bool keep = lane < np && (s < 0 || (s & TENT));
    const bool prop = lane < np && s >= 0 && (s & TENT);
    const int c = prop ? cur_color(s) : -1;
    bool lost = false;
    for (uint64_t b = __ballot(prop); b; b &= b - 1) {
        const int j = __builtin_ctzll(b);
        const int cj = __shfl(c, j), xj = __shfl(x, j);
        if (prop && cj == c && xj < x) lost = true;
    }
    if (prop) sp_set(sp, lpos + p, x, lost);
    const uint64_t kb = __ballot(keep);
    if (keep) sp.pl[lpos + __builtin_popcountll(kb & ((1ull << lane) - 1ull))] = p;
    if (lane == 0) {
        sp.pn[v] = __builtin_popcountll(kb);
        if (__builtin_popcountll(kb) <= 1) done[v] = kb ? 2 : 1;   // see conflict_dirty
        sp.dirty[v] = 0;
    }
}

// pending lists of the nets of at most SMALL_NET members (used by the
// standing-proposal scan without the column-major copy): every position
template <bool D2>
__global__ void k_pending_init_small(Graph g, int *pl, int *pn)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n_b; v += gridDim.x * blockDim.x) {
        const int sz = Acc<D2>::size(g, v);
        if (sz > SMALL_NET) continue;
        const long lpos = sp_lpos<D2>(g, v);
        for (int k = 0; k < sz; k++) pl[lpos + k] = k;
        pn[v] = sz;
    }
}

// pending lists of the nets above SMALL_NET: every position (standing
// proposals start, or restart after a net-based round)
template <bool D2>
__global__ void k_pending_init(Graph g, const int *big, const int *n_big_p, int *pl, int *pn)
{
    const int n_big = *n_big_p;
    for (int bi = blockIdx.x; bi < n_big; bi += gridDim.x) {
        const int v = big[bi];
        const int sz = Acc<D2>::size(g, v);
        const long lpos = sp_lpos<D2>(g, v);
        for (int k = threadIdx.x; k < sz; k += blockDim.x) pl[lpos + k] = k;
        if (threadIdx.x == 0) pn[v] = sz;
    }
}

template <bool D2>
__global__ void __launch_bounds__(BIG_BLOCK) k_conflict_big(Graph g, const int *st, uint8_t *lose, uint8_t *done,
                                                            const int *big, const int *n_big_p, Ctrl *ctrl,
                                                            int tent_only, SPState sp, int huge_elsewhere)
{
    extern __shared__ int sh[];
    __shared__ int s_scan[20], s_cnt, s_keep;
    constexpr int BIG_CHUNK = 64;
    __shared__ int s_list[BIG_CHUNK], s_ln;
    const int n_big = *n_big_p;
    const int tid = threadIdx.x, nt = blockDim.x;
    // BIG_CHUNK nets at a time: a thread per net checks its flags, the nets
    // to scan are listed in LDS, then the block scans them one by one
    for (int base = blockIdx.x * BIG_CHUNK; base < n_big; base += gridDim.x * BIG_CHUNK) {
        if (tid == 0) s_ln = 0;
        __syncthreads();
        if (tid < BIG_CHUNK && base + tid < n_big) {
            const int v = big[base + tid];
            const bool fin = tent_only ? done[v] != 0 : done[v] == 1;
            if (!fin && !(sp.lbits && !sp.dirty[v])) s_list[atomicAdd(&s_ln, 1)] = v;
        }
        __syncthreads();
        const int ln = s_ln;
        if (sp.pl && tent_only) {
            // nets with at most 64 pending members: a wave each, no barriers
            const int wid = tid / WAVE;
            for (int li = wid; li < ln; li += BIG_BLOCK / WAVE) {
                const int v = s_list[li];
                const int np = sp.pn[v];
                if (np <= WAVE && !(huge_elsewhere && Acc<D2>::size(g, v) > HASH_MAX)) {
                    wave_pending_net<D2>(g, st, done, sp, v, sp_lpos<D2>(g, v), np);
                    if (lane_id() == 0) s_list[li] = -1;
                }
            }
            __syncthreads();
        }
        for (int li = 0; li < ln; li++) {
            const int v = s_list[li];
            if (v < 0) continue;
            const long lpos = sp.lbits ? sp_lpos<D2>(g, v) : 0;
            int sz = Acc<D2>::size(g, v);
            if (sz <= HASH_MAX) {
                // members and states read once into registers (the block holds
                // BIG_PER_THREAD per thread), all loads of a batch in flight;
                // with pending lists only the listed positions
                const bool plm = sp.pl != nullptr && tent_only;
                const int np = plm ? sp.pn[v] : sz;
                int xs[BIG_PER_THREAD], ss[BIG_PER_THREAD], ps[BIG_PER_THREAD];
    #pragma unroll
                for (int i = 0; i < BIG_PER_THREAD; i++) {
                    const int k = tid + i * BIG_BLOCK;
                    ps[i] = k < np ? (plm ? sp.pl[lpos + k] : k) : -1;
                }
    #pragma unroll
                for (int i = 0; i < BIG_PER_THREAD; i++) xs[i] = ps[i] >= 0 ? Acc<D2>::member(g, v, ps[i]) : -1;
                // pending members (low 16 bits) and proposers (high bits), one sum
                int counts = 0;
    #pragma unroll
                for (int i = 0; i < BIG_PER_THREAD; i++) {
                    ss[i] = xs[i] >= 0 ? st[xs[i]] : 0;
                    counts += (xs[i] >= 0 && (ss[i] < 0 || (ss[i] & TENT))) ? 1 : 0;
                    counts += (xs[i] >= 0 && ss[i] >= 0 && (ss[i] & TENT)) ? (1 << 16) : 0;
                }
                if (tid == 0) s_cnt = 0;
                counts = block_sum(counts, s_scan);
                const int pending = counts & 0xffff, nprop = counts >> 16;
                if (plm) {
                    // the list keeps the pending positions (every read of it is done)
    #pragma unroll
                    for (int i = 0; i < BIG_PER_THREAD; i++)
                        if (xs[i] >= 0 && (ss[i] < 0 || (ss[i] & TENT))) sp.pl[lpos + atomicAdd(&s_cnt, 1)] = ps[i];
                    if (tid == 0) sp.pn[v] = pending;
                }
                if (sp.lbits && tid == 0) sp.dirty[v] = 0;
                if (pending == 0) {
                    if (tid == 0) done[v] = 1;
                    continue;
                }
                if (tent_only && nprop <= 1) {
                    // a lone proposer keeps its proposal in this net
                    if (sp.lbits) {
    #pragma unroll
                        for (int i = 0; i < BIG_PER_THREAD; i++)
                            if (xs[i] >= 0 && ss[i] >= 0 && (ss[i] & TENT)) sp_set(sp, lpos + ps[i], xs[i], false);
                    }
                    __syncthreads();
                    continue;
                }
                // hash of the proposed colors (tent_only: nprop entries at most)
                int cap = 64;
                while (cap < 2 * (tent_only ? nprop : sz)) cap <<= 1;
                int *keys = sh, *minr = sh + cap;
                for (int i = tid; i < cap; i += nt) {
                    keys[i] = -1;
                    minr[i] = 0x7fffffff;
                }
                __syncthreads();
    #pragma unroll
                for (int i = 0; i < BIG_PER_THREAD; i++) {
                    const int x = xs[i], s = ss[i];
                    if (x < 0 || (tent_only && !(s >= 0 && (s & TENT)))) continue;
                    const int c = cur_color(s);
                    if (c < 0) continue;
                    unsigned h = hash_color(c) & (cap - 1);
                    for (;;) {
                        int prev = atomicCAS(&keys[h], -1, c);
                        if (prev == -1 || prev == c) {
                            atomicMin(&minr[h], x);
                            break;
                        }
                        h = (h + 1) & (cap - 1);
                    }
                }
                __syncthreads();
    #pragma unroll
                for (int i = 0; i < BIG_PER_THREAD; i++) {
                    const int x = xs[i], s = ss[i];
                    if (x < 0 || (tent_only && !(s >= 0 && (s & TENT)))) continue;
                    const int c = cur_color(s);
                    if (c < 0) continue;
                    unsigned h = hash_color(c) & (cap - 1);
                    while (keys[h] != c) h = (h + 1) & (cap - 1);
                    if (sp.lbits) sp_set(sp, lpos + ps[i], x, minr[h] != x);
                    else if (minr[h] != x) lose[x] = 1;
                }
                __syncthreads();
                continue;
            }
            if (huge_elsewhere && sz > HASH_MAX) continue;   // k_conflict_huge
            conflict_large<D2>(g, st, lose, done, v, sz, lpos, tent_only, sp, sh, BIG_LIST, ctrl->max_color, s_scan,
                               &s_cnt, &s_keep);
        }
        __syncthreads();
    }
}

// Nets larger than HASH_MAX (their own list, built with the shape figures)
// in vertex-based rounds: a block of HUGE_BLOCK threads per net with a
// proposal list as large as the LDS holds.
constexpr int HUGE_BLOCK = 1024;
template <bool D2>
__global__ void __launch_bounds__(HUGE_BLOCK) k_conflict_huge(Graph g, const int *st, uint8_t *lose, uint8_t *done,
                                                              const int *huge, const int *n_huge_p, Ctrl *ctrl,
                                                              int tent_only, SPState sp, int list_cap)
{
    extern __shared__ int sh[];
    __shared__ int s_scan[20], s_cnt, s_keep;
    const int n_huge = *n_huge_p;
    for (int hi = blockIdx.x; hi < n_huge; hi += gridDim.x) {
        const int v = huge[hi];
        if ((tent_only ? done[v] != 0 : done[v] == 1) || (sp.lbits && !sp.dirty[v])) continue;
        const long lpos = sp.lbits ? sp_lpos<D2>(g, v) : 0;
        if (sp.pl && tent_only && sp.pn[v] <= WAVE) {
            // few pending members left: one wave, no barriers
            if (threadIdx.x < WAVE) wave_pending_net<D2>(g, st, done, sp, v, lpos, sp.pn[v]);
            continue;
        }
        conflict_large<D2>(g, st, lose, done, v, Acc<D2>::size(g, v), lpos, tent_only, sp, sh, list_cap,
                           ctrl->max_color, s_scan, &s_cnt, &s_keep);
    }
}

// Removal in the vertex form (Algorithm 5 with Algorithm 3's test): thread
// per worklist vertex w, which loses iff a lower-ranked vertex sharing a net
// with w holds w's current color.  Members are ascending in rank (distance-2:
// the center first, then the ascending neighbours), so a net's walk stops at
// the first member ranked above w.  Exact where no colored vertex can hold a
// color a worklist vertex proposes (the driver uses it only there).
template <bool D2>
__global__ void k_conflict_vertex(Graph g, const int *W, Ctrl *ctrl, int par, const int *st, uint8_t *lose)
{
    const int n = ctrl->n_w[par];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int w = W[i];
        const int c = cur_color(st[w]);
        if (c < 0) continue;
        bool lost = false;
        const int nn = Acc<D2>::nets_count(g, w);
        for (int a = 0; a < nn && !lost; a++) {
            const int v = Acc<D2>::net_at(g, w, a);
            const int sz = Acc<D2>::size(g, v);
            for (int k = 0; k < sz; k++) {
                const int x = Acc<D2>::member(g, v, k);
                if (x >= w) {
                    if (D2 && k == 0) continue;   // the center comes first, out of order
                    break;
                }
                if (cur_color(st[x]) == c) {
                    lost = true;
                    break;
                }
            }
        }
        if (lost) lose[w] = 1;
    }
}

// ---------------------------------------------------------------------------
// apply + compaction

// Over the worklist (list != nullptr) or over every vertex (list == nullptr,
// after a net-based round that may evict colored vertices): losers become
// uncolored, winners keep their proposal and, when the masks are maintained
// incrementally (update_masks), set its bit in the masks of their nets (each
// wave queues its winners of a tile in LDS and walks their rows 64 winners at
// a time as one flat range, so the row offsets and the rows are each one
// round of loads).  Writes the number of uncolored entries of each tile.
// With zf (first-fit vertex rounds with standing proposals) the winners of
// color 0 are listed in z0l for k_compact, which marks their neighbourhoods.
template <bool D2>
__global__ void __launch_bounds__(TILE_BLOCK) k_apply(Graph g, const int *list, Ctrl *ctrl, int par, int *st,
                                                      uint8_t *lose, uint64_t *mask0, int *tile_count,
                                                      RoundRec *rec, int round, int update_masks, uint64_t *hw,
                                                      int PH, const int *lcnt, const uint8_t *zf = nullptr,
                                                      int *z0l = nullptr)
{
    constexpr int NWV = TILE_BLOCK / WAVE;
    constexpr int WQ = 2 * WAVE;   // winners queued per wave before their rows are walked
    __shared__ int s_scan[8];
    __shared__ int s_u[NWV][WQ];
    __shared__ int s_col[NWV][WQ];
    __shared__ int s_pre[NWV][64], s_beg[NWV][64];
    const int n = list ? ctrl->n_w[par] : g.n_a;
    const int ntiles = (n + TILE - 1) / TILE;
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->n_w[par ^ 1] = 0;
        ctrl->n_heavy = 0;
        ctrl->z0n[par ^ 1] = 0;   // the next round's list of color-0 winners
    }
    // the queued winners' rows, 64 winners at a time: row offsets in one
    // pass, then the rows as one flat range, one color word update per entry
    // (mask0 for colors below 64, else the color's higher word)
    auto walk = [&](int qn) {
        for (int c0 = 0; c0 < qn; c0 += 64) {
            const int j = c0 + lane;
            int beg = 0, d = 0;
            if (j < qn) {
                const int u = s_u[wid][j];
                beg = g.a_off[u];
                d = g.a_off[u + 1] - beg;
            }
            const int incl = wave_incl_scan(d);
            const int total = __shfl(incl, 63);
            s_pre[wid][lane] = incl - d;
            s_beg[wid][lane] = beg;
            wave_sync();
            for (int f0 = 0; f0 < total; f0 += 256) {
                int tgt[4], cq[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    int f = f0 + q * 64 + lane;
                    tgt[q] = -1;
                    cq[q] = 0;
                    if (f < total) {
                        int r = row_of(s_pre[wid], f);
                        tgt[q] = g.a_idx[s_beg[wid][r] + f - s_pre[wid][r]];
                        cq[q] = s_col[wid][c0 + r];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    if (tgt[q] < 0) continue;
                    const int c = cq[q];
                    uint64_t *wd = c < 64 ? &mask0[tgt[q]] : &hw[(long)tgt[q] * PH + (c >> 6) - 1];
                    atomicOr((unsigned long long *)wd, 1ull << (c & 63));
                }
            }
            wave_sync();
        }
    };
    constexpr int KS = TILE / TILE_BLOCK;
    int evicted = 0, mx = -1;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int cnt = 0, qn = 0;
        int us[KS], ss[KS];
        uint8_t ls[KS];
#pragma unroll
        for (int k = 0; k < KS; k++) {
            int i = t * TILE + k * TILE_BLOCK + threadIdx.x;
            us[k] = i < n ? (list ? list[i] : i) : -1;
        }
#pragma unroll
        for (int k = 0; k < KS; k++) {
            ss[k] = us[k] >= 0 ? st[us[k]] : -1;
            ls[k] = us[k] >= 0 ? (lcnt ? (uint8_t)(lcnt[us[k]] > 0) : lose[us[k]]) : 0;
        }
        for (int k = 0; k < KS; k++) {
            bool q64 = false;
            int col = 0;
            bool z0 = false;   // (zf) a winner of color 0
            if (us[k] >= 0) {
                int u = us[k];
                int s = ss[k];
                if (ls[k]) {
                    if (!lcnt) {   // standing proposals: the loser keeps its proposal
                        lose[u] = 0;
                        if (s >= 0 && !(s & TENT)) evicted++;
                        st[u] = -1;
                    }
                    cnt++;
                } else if (s < 0) {
                    cnt++;
                } else {
                    col = s & COLOR_MASK;
                    if (s & TENT) {
                        st[u] = col;
                        // the color's word in every net of u (colors past the
                        // allocated words are not tracked)
                        if (update_masks && (col < 64 || (col >> 6) - 1 < PH)) {
                            q64 = true;
                            if (D2) {   // the closed neighbourhood of u itself
                                uint64_t *wd = col < 64 ? &mask0[u] : &hw[(long)u * PH + (col >> 6) - 1];
                                atomicOr((unsigned long long *)wd, 1ull << (col & 63));
                            }
                        }
                    }
                    mx = max(mx, col);
                    z0 = zf && (s & TENT) && col == 0;
                }
            }
            if (zf) {
                // winners of color 0 onto the list k_compact marks from
                const uint64_t zb = __ballot(z0);
                if (zb) {
                    int zbase = 0;
                    if (lane == 0) zbase = atomicAdd(&ctrl->z0n[par], __builtin_popcountll(zb));
                    zbase = __shfl(zbase, 0);
                    if (z0) z0l[zbase + __builtin_popcountll(zb & ((1ull << lane) - 1ull))] = us[k];
                }
            }
            if (update_masks) {
                const uint64_t bal = __ballot(q64);
                if (q64) {
                    const int r = qn + __builtin_popcountll(bal & ((1ull << lane) - 1ull));
                    s_u[wid][r] = us[k];
                    s_col[wid][r] = col;
                }
                qn += __builtin_popcountll(bal);
                if (qn > WQ - WAVE) {
                    wave_sync();
                    walk(qn);
                    qn = 0;
                }
            }
        }
        if (update_masks && qn > 0) {
            wave_sync();
            walk(qn);
        }
        cnt = block_sum(cnt, s_scan);
        if (threadIdx.x == 0) tile_count[t] = cnt;
    }
    evicted = wave_sum(evicted);
    mx = wave_max(mx);
    if (lane == 0) {
        if (evicted) atomicAdd(&rec[round].evicted, evicted);
        if (mx >= 0) max_to(&ctrl->pad[0], mx);
    }
}

// Closing kernel of a front-driven first-fit round.  A vertex-based
// first-fit proposal is 0 unless some net of the vertex holds color 0, so
// the uncolored vertices split into the front (F(w) holds 0: their first-fit
// is recomputed every round, on the front list) and the rest, whose standing
// proposal 0 never needs recomputing.  After the removal step the winners are
// exactly the vertices still holding a proposal with loss count 0 (every
// other one lost in some net), so this kernel streams over all vertices,
// four per thread: a winner's proposal becomes its color and the color's bit
// goes into the words of its nets (the exchanges issued together); a net that
// gains its first member of color 0 goes on the list zl for k_front_push.
// The last block to finish closes the round (worklist size, record, host
// mirror) and clears the counters of the lists this round consumed.
constexpr int APPLY_BLOCK = 256;
template <bool D2>
__global__ void __launch_bounds__(APPLY_BLOCK) k_front_apply(Graph g, const int *lcnt, int *st, uint64_t *mask0,
                                                             uint64_t *hw, int PH, int *zl, int *zl_n, Ctrl *ctrl,
                                                             int par, RoundRec *rec, int round, int *host,
                                                             int *clear_a, int *clear_b, int *clear_c)
{
    __shared__ int s_scan[8];
    __shared__ bool s_last;
    const int lane = lane_id();
    const int n = g.n_a;
    int wins = 0, mx = -1;
    const long nq = ((long)n + 3) / 4;   // groups of four vertices
    const long tstride = (long)gridDim.x * APPLY_BLOCK;
    const long nloop = (nq + tstride - 1) / tstride;
    for (long it = 0; it < nloop; it++) {
        const long qi = it * tstride + (long)blockIdx.x * APPLY_BLOCK + threadIdx.x;
        int xs[4], cs[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            xs[k] = -1;
            cs[k] = -1;
        }
        if (qi < nq) {
            const long x0 = qi * 4;
            int sv[4], lv[4];
            if (x0 + 3 < n && !((uintptr_t)st & 15)) {
                const int4 s4 = *(const int4 *)(st + x0);   // st 16-byte aligned, x0 a multiple of 4
                sv[0] = s4.x; sv[1] = s4.y; sv[2] = s4.z; sv[3] = s4.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; k++) sv[k] = x0 + k < n ? st[x0 + k] : -1;
            }
            bool any = false;
#pragma unroll
            for (int k = 0; k < 4; k++) any |= sv[k] >= 0 && (sv[k] & TENT);
            if (any) {
#pragma unroll
                for (int k = 0; k < 4; k++) lv[k] = (sv[k] >= 0 && (sv[k] & TENT)) ? lcnt[x0 + k] : 1;
#pragma unroll
                for (int k = 0; k < 4; k++)
                    if (sv[k] >= 0 && (sv[k] & TENT) && lv[k] == 0) {
                        xs[k] = (int)(x0 + k);
                        cs[k] = sv[k] & COLOR_MASK;
                        st[x0 + k] = cs[k];
                    }
            }
        }
        // the winners' colors in the words of their nets; nets gaining color 0
        for (int k = 0; k < 4; k++) {
            const int x = xs[k], col = cs[k];
            uint64_t zero_nets = 0;
            int nn = 0;
            if (x >= 0) {
                wins++;
                mx = max(mx, col);
                nn = Acc<D2>::nets_count(g, x);
                // all exchanges in flight before any result is looked at
                uint64_t olds[32];
#pragma unroll
                for (int j = 0; j < 32; j++) {
                    if (j < nn) {
                        const int v = Acc<D2>::net_at(g, x, j);
                        if (col == 0) olds[j] = atomicOr((unsigned long long *)&mask0[v], 1ull);
                        else if (col < 64) atomicOr((unsigned long long *)&mask0[v], 1ull << col);
                        else if ((col >> 6) - 1 < PH)
                            atomicOr((unsigned long long *)&hw[(long)v * PH + (col >> 6) - 1], 1ull << (col & 63));
                    }
                }
                if (col == 0) {
#pragma unroll
                    for (int j = 0; j < 32; j++)
                        if (j < nn && !(olds[j] & 1ull)) zero_nets |= 1ull << j;
                }
                for (int j = 32; j < nn; j++) {   // vertices of many nets: one by one
                    const int v = Acc<D2>::net_at(g, x, j);
                    if (col == 0) {
                        if (!(atomicOr((unsigned long long *)&mask0[v], 1ull) & 1ull)) zl[atomicAdd(zl_n, 1)] = v;
                    } else if (col < 64) {
                        atomicOr((unsigned long long *)&mask0[v], 1ull << col);
                    } else if ((col >> 6) - 1 < PH) {
                        atomicOr((unsigned long long *)&hw[(long)v * PH + (col >> 6) - 1], 1ull << (col & 63));
                    }
                }
            }
            // newly zero nets onto zl, one atomic per wave for the slots
            const int cnt = __builtin_popcountll(zero_nets);
            const int incl = wave_incl_scan(cnt);
            const int tot = __shfl(incl, WAVE - 1);
            if (tot) {
                int base = 0;
                if (lane == WAVE - 1) base = atomicAdd(zl_n, tot);
                base = __shfl(base, WAVE - 1) + incl - cnt;
                for (uint64_t t = zero_nets; t; t &= t - 1) zl[base++] = Acc<D2>::net_at(g, x, __builtin_ctzll(t));
            }
        }
    }
    wins = block_sum(wins, s_scan);
    mx = block_max(mx, s_scan);
    if (threadIdx.x == 0) {
        if (wins) atomicAdd(&ctrl->win, wins);
        if (mx >= 0) max_to(&ctrl->pad[0], mx);
        __threadfence();
        s_last = atomicAdd(&ctrl->done_blocks, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        const int w = ctrl->n_w[par];
        const int total_wins = atomicAdd(&ctrl->win, 0);
        const int left = w - total_wins;
        ctrl->n_w[par ^ 1] = left;
        ctrl->win = 0;
        ctrl->done_blocks = 0;
        ctrl->n_heavy = 0;
        *clear_a = 0;
        *clear_b = 0;
        *clear_c = 0;
        if (w > 0) {
            ctrl->rounds += 1;
            RoundRec &R = rec[round];
            R.mode = 0;
            R.w = w;
            R.losers = left;
            R.max_color = atomicAdd(&ctrl->pad[0], 0);
            if (host) {
                __atomic_store_n(&host[1], left, __ATOMIC_RELAXED);
                __atomic_store_n(&host[2], ctrl->error, __ATOMIC_RELAXED);
                __atomic_store_n(&host[3], R.max_color, __ATOMIC_RELAXED);
                __threadfence_system();
                __atomic_store_n(&host[0], round, __ATOMIC_RELAXED);
                __threadfence_system();
            }
        }
    }
}

// Members of the nets that gained color 0 join the front list (one lane per
// (net, member) pair: every exchange of the round in flight at once); a flag
// per vertex, taken by exchange, lets each vertex join once, so the front
// lists never hold more than |V_A| entries.
template <bool D2>
__global__ void __launch_bounds__(256) k_front_push(Graph g, const int *zl, const int *zl_n, const int *st,
                                                    int *infront, int *fl_out, int *fl_out_n)
{
    const long n = (long)*zl_n * SMALL_NET;
    for (long i = blockIdx.x * 256L + threadIdx.x; i - threadIdx.x < n; i += gridDim.x * 256L) {
        int y = -1;
        if (i < n) {
            const int v = zl[i / SMALL_NET];
            const int k = (int)(i % SMALL_NET);
            if (k < Acc<D2>::size(g, v)) {
                y = Acc<D2>::member(g, v, k);
                const int sy = st[y];
                if (!((sy < 0 || (sy & TENT)) && !infront[y] && atomicExch(&infront[y], 1) == 0)) y = -1;
            }
        }
        const uint64_t bal = __ballot(y >= 0);
        if (!bal) continue;
        int base = 0;
        if (lane_id() == 0) base = atomicAdd(fl_out_n, __builtin_popcountll(bal));
        base = __shfl(base, 0);
        if (y >= 0) fl_out[base + __builtin_popcountll(bal & ((1ull << lane_id()) - 1ull))] = y;
    }
}

// Stable scatter of the uncolored entries into the next worklist.  Tile t's
// offset is the sum of the counts of tiles < t; inside a tile, entries are
// ranked by wave ballots in index order.
// With count_round, a round whose worklist was empty leaves everything as is;
// otherwise the round is counted and its record completed.
// zf (first-fit vertex rounds with standing proposals): a winner of color 0
// proposed it because none of its nets held color 0 (a net that gains color
// 0 makes every member still proposing 0 lose and propose again), so each of
// its nets gains color 0 now, for the first time.  After the compaction,
// every wave takes winners from z0l and marks the members of their nets
// (distance-2: the centers too) in zf, one flat range per 64 nets.
template <bool D2>
__device__ void zero_front_mark(const Graph &g, const int *z0l, int nz, uint8_t *zf, int *s_pre, int *s_beg)
{
    const int lane = lane_id();
    const int nwv = blockDim.x / WAVE, wv = blockIdx.x * nwv + threadIdx.x / WAVE;
    for (int i = wv; i < nz; i += gridDim.x * nwv) {
        const int u = z0l[i];
        const int ab = g.a_off[u], ad = g.a_off[u + 1] - ab;
        for (int c0 = 0; c0 < ad + (D2 ? 1 : 0); c0 += WAVE) {
            // nets c0 .. c0 + 63 of u (distance-2: u's own net last)
            const int j = c0 + lane;
            int v = -1, beg = 0, d = 0;
            if (j < ad) v = g.a_idx[ab + j];
            else if (D2 && j == ad) v = u;
            if (v >= 0) {
                beg = g.b_off[v];
                d = g.b_off[v + 1] - beg;
                if (D2) zf[v] = 1;
            }
            const int incl = wave_incl_scan(d);
            const int total = __shfl(incl, WAVE - 1);
            s_pre[lane] = incl - d;
            s_beg[lane] = beg;
            wave_sync();
            for (int f0 = 0; f0 < total; f0 += 8 * WAVE) {
                int x[8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const int f = f0 + q * WAVE + lane;
                    x[q] = -1;
                    if (f < total) {
                        const int r = row_of(s_pre, f);
                        x[q] = g.b_idx[s_beg[r] + f - s_pre[r]];
                    }
                }
#pragma unroll
                for (int q = 0; q < 8; q++)
                    if (x[q] >= 0) zf[x[q]] = 1;
            }
            wave_sync();
        }
    }
}

template <bool D2 = false>
__global__ void __launch_bounds__(TILE_BLOCK) k_compact(const int *list, int n_static, Ctrl *ctrl, int par,
                                                        const int *st, const int *tile_count, int *out,
                                                        RoundRec *rec, int round, int mode, int count_round,
                                                        int *host, Graph g = Graph{}, const int *z0l = nullptr,
                                                        uint8_t *zf = nullptr)
{
    constexpr int KS = TILE / TILE_BLOCK;
    constexpr int NWV = TILE_BLOCK / WAVE;
    __shared__ int s_cnt[KS * NWV + 1];
    __shared__ int s_scan[8];
    if (count_round && ctrl->n_w[par] == 0) return;
    const int n = list ? ctrl->n_w[par] : n_static;
    const int ntiles = (n + TILE - 1) / TILE;
    const int lane = lane_id(), wid = threadIdx.x / WAVE;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int pre = 0;
        for (int j = threadIdx.x; j < t; j += TILE_BLOCK) pre += tile_count[j];
        pre = block_sum(pre, s_scan);
        int u_k[KS];
        uint64_t bal[KS];
        for (int k = 0; k < KS; k++) {
            int i = t * TILE + k * TILE_BLOCK + threadIdx.x;
            int u = -1;
            bool f = false;
            if (i < n) {
                u = list ? list[i] : i;
                f = st[u] < 0 || (st[u] & TENT);   // uncolored, or a standing proposal
            }
            u_k[k] = u;
            bal[k] = __ballot(f);
            if (lane == 0) s_cnt[k * NWV + wid] = __builtin_popcountll(bal[k]);
        }
        __syncthreads();
        if (threadIdx.x < WAVE) {
            int c = threadIdx.x < KS * NWV ? s_cnt[threadIdx.x] : 0;
            int inc = wave_incl_scan(c);
            if (threadIdx.x < KS * NWV) s_cnt[threadIdx.x] = inc - c;
            if (threadIdx.x == KS * NWV - 1) s_cnt[KS * NWV] = inc;
        }
        __syncthreads();
        uint64_t below = lane ? (~0ull >> (WAVE - lane)) : 0ull;
        for (int k = 0; k < KS; k++) {
            if ((bal[k] >> lane) & 1ull) {
                int r = __builtin_popcountll(bal[k] & below);
                out[pre + s_cnt[k * NWV + wid] + r] = u_k[k];
            }
        }
        if (t == ntiles - 1 && threadIdx.x == 0) {
            int total = pre + s_cnt[KS * NWV];
            ctrl->n_w[par ^ 1] = total;
            if (count_round) {
                ctrl->rounds += 1;
                RoundRec &R = rec[round];
                R.mode = mode;
                R.w = ctrl->n_w[par];
                R.losers = total;
                R.max_color = ctrl->pad[0];
                if (host) {
                    // pinned host mirror: (round, worklist, error, max color)
                    __atomic_store_n(&host[1], total, __ATOMIC_RELAXED);
                    __atomic_store_n(&host[2], ctrl->error, __ATOMIC_RELAXED);
                    __atomic_store_n(&host[3], ctrl->pad[0], __ATOMIC_RELAXED);
                    __threadfence_system();
                    __atomic_store_n(&host[0], round, __ATOMIC_RELAXED);
                    __threadfence_system();
                }
            }
        }
        __syncthreads();
    }
    if (zf) {
        __shared__ int s_zp[TILE_BLOCK / WAVE][WAVE], s_zb[TILE_BLOCK / WAVE][WAVE];
        const int wid = threadIdx.x / WAVE;
        zero_front_mark<D2>(g, z0l, ctrl->z0n[par], zf, s_zp[wid], s_zb[wid]);
    }
}

// counts of uncolored entries per tile over all vertices (resume set-up)
__global__ void __launch_bounds__(TILE_BLOCK) k_count_uncolored(const int *st, int n, int *tile_count)
{
    __shared__ int s_scan[8];
    const int ntiles = (n + TILE - 1) / TILE;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int cnt = 0;
        for (int k = 0; k < TILE / TILE_BLOCK; k++) {
            int i = t * TILE + k * TILE_BLOCK + threadIdx.x;
            if (i < n && st[i] < 0) cnt++;
        }
        cnt = block_sum(cnt, s_scan);
        if (threadIdx.x == 0) tile_count[t] = cnt;
    }
}

__global__ void k_set_max_final(Ctrl *ctrl, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->pad[0] = v;
}

// ---------------------------------------------------------------------------
// incremental first-fit vertex rounds
//
// Between two first-fit vertex-based rounds only two things can change the
// outcome for a worklist vertex w: a neighbour got colored (F(w) changes, so
// its proposal may change), or w or a lower-ranked neighbour changed its
// proposal (its removal test may change).  Everything else repeats: w makes
// the same proposal and loses again.  The incremental rounds therefore keep
// every worklist vertex's last proposal (TENT | col) and recompute only
//   D_r = worklist vertices sharing a net with a winner of round r-1
//         (first-fit again, k_inc_color),
//   A_r = D_r plus the worklist members of nets holding a vertex whose
//         proposal changed (removal test again, k_inc_conflict).
// The round's result is exactly the full round's result.  Sets are
// deduplicated with bit sets and kept as unordered lists; the order of a
// list never reaches a result.

__global__ void k_inc_reset(IncCtrl *ic)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ic->n_d[0] = ic->n_d[1] = 0;
        ic->n_a = ic->n_win = ic->n_tcn = ic->n_cn = 0;
    }
}

// Thread per dirty vertex: first-fit through the masks of its nets (eight
// gathers in flight).  A changed proposal queues w's nets; w itself always
// joins A.  Entries needing colors >= 64 go to k_vcolor_wide (incremental).
template <bool D2>
__global__ void k_inc_color(Graph g, IncCtrl *ic, int par, const int *D, unsigned *dirty_bits, int *st,
                            const uint64_t *mask0, unsigned *aff_bits, int *A, unsigned *tchg_bits, int *tcn,
                            int *heavy, Ctrl *ctrl)
{
    const int n = ic->n_d[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) ic->n_win = 0;
    int local_max = -1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int w = D[i];
        clear_bit(dirty_bits, w);
        uint64_t m = D2 ? mask0[w] : 0ull;
        int beg = g.a_off[w], d = g.a_off[w + 1] - beg;
        for (int k0 = 0; k0 < d; k0 += 8) {
            int nets[8];
#pragma unroll
            for (int q = 0; q < 8; q++) nets[q] = (k0 + q < d) ? g.a_idx[beg + k0 + q] : -1;
            uint64_t mm[8];
#pragma unroll
            for (int q = 0; q < 8; q++) mm[q] = nets[q] >= 0 ? mask0[nets[q]] : 0ull;
#pragma unroll
            for (int q = 0; q < 8; q++) m |= mm[q];
        }
        if (~m) {
            int col = __builtin_ctzll(~m);
            int nw = TENT | col;
            if (st[w] != nw) {
                st[w] = nw;
                mark_proposal_change<D2>(g, w, tchg_bits, tcn, ic);
            }
            if (set_once(aff_bits, w)) A[atomicAdd(&ic->n_a, 1)] = w;
            local_max = max(local_max, col);
        } else {
            heavy[atomicAdd(&ctrl->n_heavy, 1)] = w;
        }
    }
    local_max = wave_max(local_max);
    if (lane_id() == 0 && local_max >= 0) max_to(&ctrl->max_color, local_max);
}

// Thread per listed net: every worklist member (a vertex holding a proposal)
// joins `out` once.  Clears the net's bit.
template <bool D2>
__global__ void k_expand(Graph g, const int *nets, const int *n_nets_p, unsigned *net_bits, const int *st,
                         unsigned *item_bits, int *out, int *n_out)
{
    const int n = *n_nets_p;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int v = nets[i];
        clear_bit(net_bits, v);
        int sz = Acc<D2>::size(g, v);
        for (int k0 = 0; k0 < sz; k0 += 8) {
            int xs[8], ss[8];
#pragma unroll
            for (int q = 0; q < 8; q++) xs[q] = (k0 + q < sz) ? Acc<D2>::member(g, v, k0 + q) : -1;
#pragma unroll
            for (int q = 0; q < 8; q++) ss[q] = xs[q] >= 0 ? st[xs[q]] : -1;
#pragma unroll
            for (int q = 0; q < 8; q++)
                if (is_tent(ss[q]) && set_once(item_bits, xs[q])) out[atomicAdd(n_out, 1)] = xs[q];
        }
    }
}

// Thread per vertex of A: w loses iff a lower-ranked worklist vertex sharing
// a net proposes the same color (members are sorted, so each net is read
// only up to w).  Winners are listed.
template <bool D2>
__global__ void k_inc_conflict(Graph g, IncCtrl *ic, int par, const int *A, unsigned *aff_bits, const int *st,
                               int *win, Ctrl *ctrl)
{
    const int n = ic->n_a;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ic->n_d[par ^ 1] = 0;
        ic->n_cn = 0;
        ic->n_tcn = 0;
        ctrl->n_heavy = 0;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int w = A[i];
        clear_bit(aff_bits, w);
        int c = st[w] & COLOR_MASK;
        bool lost = false;
        int nn = Acc<D2>::nets_count(g, w);
        for (int j = 0; j < nn && !lost; j++) {
            int v = Acc<D2>::net_at(g, w, j);
            if (D2 && v < w) {
                int sv = st[v];
                if (is_tent(sv) && (sv & COLOR_MASK) == c) {
                    lost = true;
                    break;
                }
            }
            int b = g.b_off[v], e = g.b_off[v + 1];
            for (int k0 = b; k0 < e && !lost; k0 += 8) {
                int xs[8], ss[8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    int x = (k0 + q < e) ? g.b_idx[k0 + q] : 0x7fffffff;
                    xs[q] = x < w ? x : -1;
                }
#pragma unroll
                for (int q = 0; q < 8; q++) ss[q] = xs[q] >= 0 ? st[xs[q]] : -1;
#pragma unroll
                for (int q = 0; q < 8; q++)
                    if (is_tent(ss[q]) && (ss[q] & COLOR_MASK) == c) lost = true;
                if (xs[7] < 0) break;   // reached members >= w
            }
        }
        if (!lost) win[atomicAdd(&ic->n_win, 1)] = w;
    }
}

// Thread per winner: its proposal becomes its color; the masks of its nets
// take the color; its nets are queued for the next round's dirty set.
template <bool D2>
__global__ void k_inc_apply(Graph g, IncCtrl *ic, const int *win, int *st, uint64_t *mask0, unsigned *cn_bits,
                            int *cn, Ctrl *ctrl)
{
    const int n = ic->n_win;
    if (blockIdx.x == 0 && threadIdx.x == 0) ic->n_a = 0;
    int mx = -1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int w = win[i];
        int col = st[w] & COLOR_MASK;
        st[w] = col;
        mx = max(mx, col);
        int k = Acc<D2>::nets_count(g, w);
        for (int j = 0; j < k; j++) {
            int v = Acc<D2>::net_at(g, w, j);
            if (col < 64) atomicOr((unsigned long long *)&mask0[v], 1ull << col);
            if (set_once(cn_bits, v)) cn[atomicAdd(&ic->n_cn, 1)] = v;
        }
    }
    mx = wave_max(mx);
    if (lane_id() == 0 && mx >= 0) max_to(&ctrl->pad[0], mx);
}

// Over the worklist of a full round whose removal ran net-side: losers keep
// their proposal (lose flag cleared), winners are applied as in k_inc_apply.
template <bool D2>
__global__ void k_inc_apply_full(Graph g, IncCtrl *ic, Ctrl *ctrl, int par, const int *W, int *st, uint8_t *lose,
                                 uint64_t *mask0, unsigned *cn_bits, int *cn)
{
    const int n = ctrl->n_w[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->n_heavy = 0;
    int mx = -1, wins = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int w = W[i];
        if (lose[w]) {
            lose[w] = 0;
            continue;
        }
        int col = st[w] & COLOR_MASK;
        st[w] = col;
        mx = max(mx, col);
        wins++;
        int k = Acc<D2>::nets_count(g, w);
        for (int j = 0; j < k; j++) {
            int v = Acc<D2>::net_at(g, w, j);
            if (col < 64) atomicOr((unsigned long long *)&mask0[v], 1ull << col);
            if (set_once(cn_bits, v)) cn[atomicAdd(&ic->n_cn, 1)] = v;
        }
    }
    mx = wave_max(mx);
    wins = wave_sum(wins);
    if (lane_id() == 0) {
        if (mx >= 0) max_to(&ctrl->pad[0], mx);
        if (wins) atomicAdd(&ic->n_win, wins);
    }
}

// Closes an incremental round: worklist size, record, host mirror.
__global__ void k_inc_close(IncCtrl *ic, Ctrl *ctrl, int par, RoundRec *rec, int round, int *host)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int nw = ctrl->n_w[par];
    if (nw == 0) {
        ctrl->n_w[par ^ 1] = 0;
        return;
    }
    int next = nw - ic->n_win;
    ctrl->n_w[par ^ 1] = next;
    ctrl->rounds += 1;
    RoundRec &R = rec[round];
    R.mode = 0;
    R.w = nw;
    R.losers = next;
    R.max_color = ctrl->pad[0];
    if (host) {
        __atomic_store_n(&host[1], next, __ATOMIC_RELAXED);
        __atomic_store_n(&host[2], ctrl->error, __ATOMIC_RELAXED);
        __atomic_store_n(&host[3], ctrl->pad[0], __ATOMIC_RELAXED);
        __threadfence_system();
        __atomic_store_n(&host[0], round, __ATOMIC_RELAXED);
        __threadfence_system();
    }
}

// proposals still pending when the call stops become -1
__global__ void k_drop_proposals(int *st, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (is_tent(st[i])) st[i] = -1;
}

// ---------------------------------------------------------------------------
// color-set statistics

// Set cardinalities.  Up to HIST_LDS colors each block counts into its own
// LDS histogram and adds it to the global one once (many vertices share a
// few colors: per-vertex atomics on one global counter would serialize);
// beyond that, global atomics per vertex.
constexpr int HIST_LDS = 12288;
__global__ void k_hist(const int *colors, long n, int *count, int ncolors)
{
    __shared__ int s_cnt[HIST_LDS];
    const bool local = ncolors <= HIST_LDS;
    if (local) {
        for (int c = threadIdx.x; c < ncolors; c += blockDim.x) s_cnt[c] = 0;
        __syncthreads();
    }
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        int c = colors[i];
        if (c >= 0 && c < ncolors) atomicAdd(local ? &s_cnt[c] : &count[c], 1);
    }
    if (local) {
        __syncthreads();
        for (int c = threadIdx.x; c < ncolors; c += blockDim.x)
            if (s_cnt[c]) atomicAdd(&count[c], s_cnt[c]);
    }
}

__global__ void k_colors_max(const int *colors, long n, int *out)
{
    int local = -1;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        local = max(local, colors[i]);
    local = wave_max(local);
    if (lane_id() == 0) atomicMax(out, local);
}

// single block: reduce the histogram into the statistics
__global__ void k_hist_reduce(const int *count, int ncolors, long long *out_i, double *out_d)
{
    __shared__ long long s_nd[16], s_min[16], s_max[16], s_sum[16];
    __shared__ double s_sq[16];
    const int tid = threadIdx.x, wid = tid / WAVE, lane = lane_id(), nw = blockDim.x / WAVE;
    long long nd = 0, mn = 0x7fffffffffffffffll, mx = 0, sum = 0;
    for (int c = tid; c < ncolors; c += blockDim.x) {
        long long k = count[c];
        if (k == 0) continue;
        nd++;
        mn = k < mn ? k : mn;
        mx = k > mx ? k : mx;
        sum += k;
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        nd += __shfl_xor(nd, d);
        long long o = __shfl_xor(mn, d);
        mn = o < mn ? o : mn;
        o = __shfl_xor(mx, d);
        mx = o > mx ? o : mx;
        sum += __shfl_xor(sum, d);
    }
    if (lane == 0) {
        s_nd[wid] = nd;
        s_min[wid] = mn;
        s_max[wid] = mx;
        s_sum[wid] = sum;
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = 1; i < nw; i++) {
            s_nd[0] += s_nd[i];
            s_min[0] = s_min[i] < s_min[0] ? s_min[i] : s_min[0];
            s_max[0] = s_max[i] > s_max[0] ? s_max[i] : s_max[0];
            s_sum[0] += s_sum[i];
        }
    }
    __syncthreads();
    const double mean = s_nd[0] ? (double)s_sum[0] / (double)s_nd[0] : 0.0;
    double sq = 0.0;
    for (int c = tid; c < ncolors; c += blockDim.x) {
        long long k = count[c];
        if (k == 0) continue;
        double d = (double)k - mean;
        sq += d * d;
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) sq += __shfl_xor(sq, d);
    if (lane == 0) s_sq[wid] = sq;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int i = 0; i < nw; i++) tot += s_sq[i];
        long long ndist = s_nd[0];
        double var = ndist ? tot / (double)ndist : 0.0;
        out_i[0] = ndist;
        out_i[1] = ncolors - 1;
        out_i[2] = ndist ? s_min[0] : 0;
        out_i[3] = s_max[0];
        out_i[4] = (long long)ncolors - ndist;
        out_d[0] = mean;
        out_d[1] = sqrt(var);
    }
}

}  // namespace bgpc
