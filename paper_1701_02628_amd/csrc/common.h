// Device-side vocabulary shared by the coloring kernels (gfx950, wave64).
//
// State word per vertex (st[u], int32):
//   -1                 uncolored
//   col (>= 0)         colored
//   TENT | col         proposed this round (still uncolored in the snapshot)
// A vertex's snapshot color (what the round's coloring phase may read) is
// col for a plain colored word and -1 otherwise; its current color (what the
// removal step compares) is col for both colored and proposed words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bgpc {

constexpr int TENT = 0x40000000;
constexpr int COLOR_MASK = 0x3fffffff;
constexpr int WAVE = 64;

__device__ __forceinline__ int snap_color(int s) { return (s >= 0 && !(s & TENT)) ? s : -1; }
__device__ __forceinline__ int cur_color(int s) { return s < 0 ? -1 : (s & COLOR_MASK); }

// Device view of the bipartite graph.  a_* lists nets(u) per vertex, b_*
// lists vtxs(v) per net.  In distance-2 mode both are the adjacency of a
// symmetric graph and every vertex v is, in addition, the first member of its
// own net N[v] (the closed neighbourhood).
struct Graph {
    int n_a, n_b;
    const int *a_off, *a_idx;
    const int *b_off, *b_idx;
};

template <bool D2>
struct Acc {
    __device__ __forceinline__ static int nets_count(const Graph &g, int u)
    {
        return g.a_off[u + 1] - g.a_off[u] + (D2 ? 1 : 0);
    }
    // k-th net of u; distance-2: N[u] first, then N[x] for x in nbor(u)
    __device__ __forceinline__ static int net_at(const Graph &g, int u, int k)
    {
        if (D2) {
            if (k == 0) return u;
            k -= 1;
        }
        return g.a_idx[g.a_off[u] + k];
    }
    __device__ __forceinline__ static int size(const Graph &g, int v)
    {
        return g.b_off[v + 1] - g.b_off[v] + (D2 ? 1 : 0);
    }
    // k-th member of net v in adjacency order; distance-2: the center first
    __device__ __forceinline__ static int member(const Graph &g, int v, int k)
    {
        if (D2) {
            if (k == 0) return v;
            k -= 1;
        }
        return g.b_idx[g.b_off[v] + k];
    }
};

// Control block in device memory, one per call.
struct Ctrl {
    int n_w[2];          // worklist length, double-buffered by round parity
    int n_heavy;         // vertices deferred to the wide coloring path this round
    int max_color;       // upper bound of every color present (max ever assigned)
    int rounds;          // rounds that started with a non-empty worklist
    int error;           // device-side invariant violations (bit set)
    int pad[2];
    // front-driven first-fit rounds
    int fl_n[2];         // front list lengths, double-buffered by round parity
    int zl_n[2];         // nets that gained color 0, double-buffered by round parity
    int win;             // winners of the round so far
    unsigned done_blocks;   // blocks of the closing kernel that have finished
    int dl_n;            // nets listed for this round's removal
    int z0n[2];          // winners of color 0 listed for the zf marking, by round parity
    int pad2[1];
};

// per-round record written by the compaction kernel
struct RoundRec {
    int mode;
    int w;
    int losers;
    int evicted;
    int max_color;
    int pad[3];
};

// Profiling counters of one round (opts->prof only), 64 slots each so that
// concurrent waves rarely hit the same address: per slot (nets walked by the
// small-net removal scan, memberships walked by it, nets(w) entries walked by
// first-fit coloring).
constexpr int PROF_SLOTS = 64;
constexpr int PROF_ROUNDS = 8192;

enum : int {
    ERR_COLOR_CAP = 1,      // a color needed more bitmap capacity than reserved
    ERR_NET_DUP = 2,        // two colored members of one net share a color at round start
    ERR_REVERSE_NEG = 4,    // reverse first-fit ran below color 0
    ERR_NET_TOO_BIG = 8
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    int lo = __shfl((int)(uint32_t)v, src);
    int hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// inclusive scan over the 64 lanes of a wave
__device__ __forceinline__ int wave_incl_scan(int v)
{
    int lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d));
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v = min(v, __shfl_xor(v, d));
    return v;
}

// block-wide exclusive scan for blockDim.x <= 1024 (multiple of 64);
// `scratch` holds at least blockDim.x / 64 + 1 ints.  Returns the exclusive
// prefix; *total receives the block sum.
// orders one wave's LDS writes before its later LDS reads (no block barrier)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int block_excl_scan(int v, int *scratch, int *total)
{
    int lane = lane_id();
    int wid = threadIdx.x / WAVE;
    int nw = blockDim.x / WAVE;
    int incl = wave_incl_scan(v);
    if (lane == WAVE - 1) scratch[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int s = lane < nw ? scratch[lane] : 0;
        int si = wave_incl_scan(s);
        if (lane < nw) scratch[lane] = si - s;
        if (lane == nw - 1) scratch[nw] = si;
    }
    __syncthreads();
    int res = scratch[wid] + incl - v;
    *total = scratch[nw];
    __syncthreads();
    return res;
}

__device__ __forceinline__ int block_sum(int v, int *scratch)
{
    int t;
    block_excl_scan(v, scratch, &t);
    return t;
}

__device__ __forceinline__ int block_max(int v, int *scratch)
{
    int lane = lane_id();
    int wid = threadIdx.x / WAVE;
    int nw = blockDim.x / WAVE;
    v = wave_max(v);
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    int r = scratch[0];
    for (int i = 1; i < nw; i++) r = max(r, scratch[i]);
    __syncthreads();
    return r;
}

}  // namespace bgpc
