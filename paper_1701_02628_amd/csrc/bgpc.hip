// Host driver and C ABI of the speculative coloring library (see bgpc.h).
//
// Every round is a fixed chain of launches on the caller's stream; the
// kernels read the worklist length from device memory, so rounds are queued
// without waiting.  The chain of round r ends with a one-thread kernel that
// copies (rounds done, worklist length) into pinned host memory; the host
// keeps at most LOOKAHEAD rounds queued beyond what it has seen completed and
// stops queueing as soon as it sees an empty worklist.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <thread>
#include <vector>

#include "bgpc.h"
#include "kernels.h"

namespace bgpc {
constexpr int DENSE_ROUTE_N = 4096;   // same bound as the batch kernel's dense mode
int color_one_workgroup(const Graph &g, int *colors, int max_rounds, hipStream_t s, int log_cap,
                        std::vector<int> *log, int *rounds_out);
}  // namespace bgpc

using namespace bgpc;

namespace {

constexpr int LOOKAHEAD = 4;

struct DevInfo {
    int cus = 256;
    int lds_max = 65536;
};

DevInfo dev_info()
{
    static std::mutex mu;
    static std::vector<DevInfo> cache;
    static std::vector<bool> have;
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev) {
        cache.resize(dev + 1);
        have.resize(dev + 1, false);
    }
    if (!have[dev]) {
        DevInfo d;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) d.cus = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            d.lds_max = v;
        cache[dev] = d;
        have[dev] = true;
    }
    return cache[dev];
}

#define HIP_TRY(x)                                  \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return BGPC_E_HIP;    \
    } while (0)

#define LAUNCH_CHECK()                              \
    do {                                            \
        if (hipGetLastError() != hipSuccess) {      \
            st_code = BGPC_E_HIP;                   \
            goto finish;                            \
        }                                           \
    } while (0)

int grid_for(long n, int block, int cap)
{
    long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// stream-ordered device workspace carved from one allocation
struct Arena {
    char *base = nullptr;
    size_t used = 0, cap = 0;
    hipStream_t s = nullptr;
    bool async = true;
    char *ext = nullptr;      // caller-provided memory (the allocation-free entry point)
    size_t ext_cap = 0;
    int reserve(size_t bytes, hipStream_t stream)
    {
        s = stream;
        cap = bytes;
        if (ext) {
            if (bytes > ext_cap) return BGPC_E_UNSUPPORTED;
            base = ext;
            return BGPC_OK;
        }
        hipError_t e = hipMallocAsync((void **)&base, bytes, stream);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            async = false;
            e = hipMalloc((void **)&base, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                base = nullptr;
                return BGPC_E_OOM;
            }
        }
        return BGPC_OK;
    }
    template <class T>
    T *take(size_t count)
    {
        size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        T *p = (T *)(base + used);
        used += bytes;
        return p;
    }
    void release()
    {
        if (!base) return;
        if (ext) {
            base = nullptr;
            return;
        }
        if (async) hipFreeAsync(base, s);
        else {
            hipStreamSynchronize(s);
            hipFree(base);
        }
        base = nullptr;
    }
};

size_t aligned(size_t count, size_t elem) { return (count * elem + 255) & ~(size_t)255; }

// pinned host mirror of the device progress counters, one per thread
struct HostProgress {
    volatile int *h = nullptr;
    int *d = nullptr;
    explicit HostProgress(std::nullptr_t) {}   // none: rounds are checked with plain copies
    HostProgress()
    {
        void *p = nullptr;
        if (hipHostMalloc(&p, 64, hipHostMallocMapped) == hipSuccess) {
            h = (volatile int *)p;
            void *dp = nullptr;
            if (hipHostGetDevicePointer(&dp, p, 0) == hipSuccess) d = (int *)dp;
        } else {
            (void)hipGetLastError();
        }
    }
};

// HIP events bracketing the launches of one kernel (opts->prof)
struct EventPool {
    std::vector<hipEvent_t> ev;
    int used = 0;
    hipEvent_t next()
    {
        if (used == (int)ev.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev.push_back(e);
        }
        return ev[used++];
    }
};

// per-thread state of the round driver (pinned progress mirror, event pool);
// created on a thread's first call and kept: freeing it at thread exit could
// run after the HIP runtime has shut down.  Worker threads that end while the
// runtime is up give it back with release_thread_state().
thread_local HostProgress *t_prog = nullptr;
thread_local EventPool *t_evpool = nullptr;

struct RunArgs {
    Graph g;
    long nnz;
    bool d2;
    const bgpc_opts *o;
    int *st;
    hipStream_t s;
    char *ext = nullptr;   // non-null: the workspace lives here and nothing is allocated
    size_t ext_cap = 0;
};

// workgroups of k_vcolor_ff resident per compute unit (occupancy query, once)
template <bool D2>
int resident_per_cu()
{
    static std::atomic<int> cached{0};
    int v = cached.load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_vcolor_ff<D2>, 64, 0) != hipSuccess || v <= 0) {
            (void)hipGetLastError();
            v = 32;
        }
        cached.store(v, std::memory_order_relaxed);
    }
    return v;
}

// workgroups of the standing-proposal removal kernel resident per compute unit
template <bool D2>
int resident_sp_per_cu()
{
    static std::atomic<int> cached{0};
    int v = cached.load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_conflict_small<D2, true>, 64, 0) != hipSuccess || v <= 0) {
            (void)hipGetLastError();
            v = 32;
        }
        cached.store(v, std::memory_order_relaxed);
    }
    return v;
}

// Choices cached by bgpc_autotune, keyed by the shape of the graph and the
// class of the schedule.
struct TuneKey {
    int d2, cls, la, lb, ld;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(d2, cls, la, lb, ld) < std::tie(o.d2, o.cls, o.la, o.lb, o.ld);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, bgpc_tuning> g_tune_cache;

int ilog2l(long v) { int r = 0; while (v > 1) { v >>= 1; r++; } return r; }

TuneKey tune_key(const Graph &g, long nnz, bool d2, const bgpc_opts &o)
{
    // schedule class: first-fit vertex rounds, first-fit with net rounds, a balancing policy
    const int cls = o.policy != BGPC_FIRST_FIT ? 2 : (o.net_color_mask ? 1 : 0);
    return TuneKey{d2 ? 1 : 0, cls, ilog2l(g.n_a), ilog2l(g.n_b), ilog2l(g.n_a ? nnz / g.n_a : 0)};
}

bgpc_tuning tune_default() { return bgpc_tuning{-1, -1, -1, 0, 0, 0}; }

// the choices for this call: the caller's, else the cached ones, else the rules
bgpc_tuning tune_for(const Graph &g, long nnz, bool d2, const bgpc_opts &o)
{
    if (o.tuning) return *o.tuning;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(g, nnz, d2, o));
    return it == g_tune_cache.end() ? tune_default() : it->second;
}

template <bool D2>
int run(const RunArgs &a)
{
    const Graph g = a.g;
    const bgpc_opts &o = *a.o;
    hipStream_t s = a.s;
    int *st = a.st;
    const int n_a = g.n_a, n_b = g.n_b;
    const DevInfo di = dev_info();
    const bool resume = (o.flags & BGPC_RESUME) != 0;
    const int policy = o.policy;
    const int chunk = o.chunk;
    int max_rounds = o.max_rounds > 0 ? o.max_rounds : n_a + 65;
    const int start_round = o.start_round;

    if (o.rounds_out) *o.rounds_out = 0;
    if (o.log) o.log->n = 0;
    if (n_a == 0) return BGPC_OK;

    // ---- workspace
    const int max_tiles = (n_a + TILE - 1) / TILE + 1;
    const int rec_cap = std::min(max_rounds, 65536) + 2;   // the round log keeps 65,536 rounds
    const int prof_rounds = o.prof ? std::min(max_rounds, PROF_ROUNDS) : 0;
    bool any_net_round = false;
    for (int r = 0; r < max_rounds && start_round + r < 64; r++)
        if (start_round + r >= 0 && ((o.net_color_mask >> (start_round + r)) & 1ull)) any_net_round = true;
    const size_t sp_words = (size_t)((a.nnz + (D2 ? n_b : 0)) / 64 + 4);
    // front-driven first-fit rounds (see k_front_apply) may run: their lists
    // (two front lists, winner candidates, stamps, front flags)
    const bgpc_tuning tune = tune_for(g, a.nnz, D2, o);
    // standing proposals pay where a coloring front sweeps many nets round
    // after round (on 2^21 stencil nets: 12% per call); on graphs of 10^4-10^5
    // nets the bookkeeping costs about as much as it saves
    const bool sp_on = !(o.flags & BGPC_INCREMENTAL) && o.net_conflict_mask == ~0ull &&
                       (tune.standing == 1 || (tune.standing < 0 && n_b >= (1 << 20)));
    // front-driven rounds do less work per round but append to shared lists,
    // and same-address atomics serialize: on the 128^3 stencil they measured
    // 82 ms per call against 24 ms for the worklist rounds, so they run only
    // when chosen (bgpc_tuning.front = 1)
    const bool front_possible = policy == BGPC_FIRST_FIT && !resume && !(o.flags & BGPC_INCREMENTAL) &&
                                !any_net_round && sp_on && tune.front == 1;
    const long fr_a = front_possible ? n_a : 0, fr_b = front_possible ? n_b : 0;
    const long n_huge_cap = std::min<long>(n_b, (a.nnz + (D2 ? n_b : 0)) / (HASH_MAX + 1) + 1) + 1;
    const bool inc_flag = (o.flags & BGPC_INCREMENTAL) != 0;
    const long inc_a = inc_flag ? n_a : 0, inc_b = inc_flag ? n_b : 0;   // incremental lists and bit sets
    size_t bytes = aligned(n_a + 1, 4) * 4            // W[0], W[1], heavy, first-fit cursors
                   + aligned(n_a + 1, 1)              // lose
                   + aligned(n_b + 1, 8)              // mask0
                   + aligned(n_b + 1, 4)              // big net list
                   + aligned(n_huge_cap, 4)           // nets above HASH_MAX members
                   + aligned(n_b + 1, 1)              // done nets
                   + aligned(max_tiles, 4)            // tile counts
                   + aligned(1, sizeof(Ctrl))         //
                   + aligned(8, 4)                    // shape figures
                   + aligned(rec_cap, sizeof(RoundRec))
                   + aligned((size_t)prof_rounds * PROF_SLOTS * 4 + 1, 8)
                   + (any_net_round ? aligned(n_a + 1, 4) : 0)
                   + aligned(1, sizeof(IncCtrl))
                   + aligned(inc_a + 1, 4) * 4        // incremental lists D0, D1, A, winners
                   + aligned(inc_b + 1, 4) * 2        // nets with a changed proposal / a winner
                   + aligned(inc_a / 32 + 2, 4) * 2   // dirty, affected bit sets
                   + aligned(inc_b / 32 + 2, 4) * 2   // net bit sets
                   + aligned(sp_words, 8)             // standing proposals: verdict bits
                   + aligned(n_a + 1, 4)              //   loss counts
                   + aligned(n_b + 1, 1)              //   dirty nets
                   + aligned(n_a + 1, 1)              //   vertices with a net holding color 0
                   + aligned(n_a + 1, 4)              //   winners of color 0 of the round
                   + aligned(fr_a + 1, 4) * 3         // front lists, front flags
                   + aligned(fr_b + 1, 4) * 4;        //   dirty-net list, its stamps, two zero-net lists
    const bool noalloc = a.ext != nullptr;
    Arena ar;
    ar.ext = a.ext;
    ar.ext_cap = a.ext_cap;
    int rc = ar.reserve(bytes, s);
    if (rc != BGPC_OK) return rc;
    int *W0 = ar.take<int>(n_a + 1);
    int *W1 = ar.take<int>(n_a + 1);
    int *heavy = ar.take<int>(n_a + 1);
    int *ffc = ar.take<int>(n_a + 1);
    uint8_t *lose = ar.take<uint8_t>(n_a + 1);
    uint64_t *mask0 = ar.take<uint64_t>(n_b + 1);
    int *big = ar.take<int>(n_b + 1);
    int *huge = ar.take<int>(n_huge_cap);
    uint8_t *done_net = ar.take<uint8_t>(n_b + 1);
    int *tile_count = ar.take<int>(max_tiles);
    Ctrl *ctrl = ar.take<Ctrl>(1);
    int *shape = ar.take<int>(8);
    RoundRec *rec = ar.take<RoundRec>(rec_cap);
    unsigned long long *pcnt = ar.take<unsigned long long>((size_t)prof_rounds * PROF_SLOTS * 4 + 1);
    int *owner = any_net_round ? ar.take<int>(n_a + 1) : nullptr;
    IncCtrl *ic = ar.take<IncCtrl>(1);
    int *Dl[2] = {ar.take<int>(inc_a + 1), ar.take<int>(inc_a + 1)};
    int *Al = ar.take<int>(inc_a + 1);
    int *WINl = ar.take<int>(inc_a + 1);
    int *TCNl = ar.take<int>(inc_b + 1);
    int *CNl = ar.take<int>(inc_b + 1);
    unsigned *dirty_bits = ar.take<unsigned>(inc_a / 32 + 2);
    unsigned *aff_bits = ar.take<unsigned>(inc_a / 32 + 2);
    unsigned *tchg_bits = ar.take<unsigned>(inc_b / 32 + 2);
    unsigned *cn_bits = ar.take<unsigned>(inc_b / 32 + 2);
    // clears the incremental rounds' bit sets (opt-in)
    auto clear_inc_bits = [&]() {
        if (!inc_flag) return;
        k_fill_i32<<<grid_for(n_a / 32 + 2, 256, 1024), 256, 0, s>>>((int *)dirty_bits, 0, n_a / 32 + 2);
        k_fill_i32<<<grid_for(n_a / 32 + 2, 256, 1024), 256, 0, s>>>((int *)aff_bits, 0, n_a / 32 + 2);
        k_fill_i32<<<grid_for(n_b / 32 + 2, 256, 1024), 256, 0, s>>>((int *)tchg_bits, 0, n_b / 32 + 2);
        k_fill_i32<<<grid_for(n_b / 32 + 2, 256, 1024), 256, 0, s>>>((int *)cn_bits, 0, n_b / 32 + 2);
    };
    unsigned long long *sp_bits = ar.take<unsigned long long>(sp_words);
    int *sp_cnt = ar.take<int>(n_a + 1);
    uint8_t *sp_dirty = ar.take<uint8_t>(n_b + 1);
    uint8_t *zf = ar.take<uint8_t>(n_a + 1);
    int *z0l = ar.take<int>(n_a + 1);
    int *FL[2] = {ar.take<int>(fr_a + 1), ar.take<int>(fr_a + 1)};
    int *infront = ar.take<int>(fr_a + 1);
    int *DL = ar.take<int>(fr_b + 1);
    int *dstamp = ar.take<int>(fr_b + 1);
    int *ZL[2] = {ar.take<int>(fr_b + 1), ar.take<int>(fr_b + 1)};
    int *Wb[2] = {W0, W1};

    int st_code = BGPC_OK;
    int h_shape[8] = {0};
    Ctrl h_ctrl;
    std::vector<RoundRec> h_rec;
    int issued = 0;
    const int nthr = 256;
    const int g_a = grid_for(n_a, nthr, di.cus * 8);
    const int g_b = grid_for(n_b, nthr, di.cus * 8);
    // higher color words (colors >= 64), net-major, grown as the largest
    // possible color grows; at most half of the free device memory
    uint64_t *hw = nullptr;
    int PH = 0;
    // balancing policies: rows of color words of the vertices of many nets,
    // precomputed per round (F, H rows of PH + 1 words)
    int *hv_id = nullptr, *hv_list = nullptr, *hv_counts = nullptr;
    HeavySlice *hv_slices = nullptr;
    uint64_t *hv_F = nullptr;
    int hv_H = 0, hv_stride = 0;
    // column-major copy of the nets' first members for the standing-proposal
    // removal scan (distance-1 graphs; skipped without room, or without
    // allocation)
    int *ell = nullptr;
    int ell_w = 0;
    // pending lists of the nets above SMALL_NET (standing proposals)
    int *pend_l = nullptr, *pend_n = nullptr;
    long mc_ub = -1;   // upper bound of every color present before the next round
    // (decided from the graph's shape below)
    bool planes_ok = !(o.flags & BGPC_INCREMENTAL) && !noalloc;   // the words are allocated as colors grow
    long max_PH = 0;
    {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) max_PH = (long)(fr / 2 / (8 * ((size_t)n_b + 1)));
        else (void)hipGetLastError();
        max_PH = std::min<long>(max_PH, (long)n_a / 64 + 2);
    }
    // standing proposals (sp_on, above) in vertex-based rounds; their state
    // is reset after every net-based round
    // removal form of round r: the vertex form (Algorithm 5) where its bit is
    // clear and it is exact -- a vertex-based round, or a net-based first
    // round that starts with nothing colored -- else the net form
    auto vertex_form = [&](int r, bool net_mode) {
        const int bit = std::min(start_round + r, 63);
        if ((o.net_conflict_mask >> bit) & 1ull) return false;
        return !net_mode || (r == 0 && !resume);
    };
    const bool net_bal = (o.flags & BGPC_NET_BALANCE) != 0;
    // diagnostics of the round log: FNV-1a hashes (rounds wait for the host)
    // and per-round event times
    const bool hash_mode = o.log && o.log->cap > 0 && (o.log->hash_t || o.log->hash_c);
    int *h_states = nullptr;
    std::vector<hipEvent_t> round_ev;
    const bool time_rounds = o.log && o.log->cap > 0 && o.log->round_ms;
    bool sp_reset = true, sp_used = false;
    const SPState sp_none = {nullptr, nullptr, nullptr, nullptr, nullptr};
    SPState sp_state = {sp_bits, sp_cnt, sp_dirty, nullptr, nullptr};   // pending lists added below
    auto ensure_planes = [&](long bound) {
        const long need = bound < 64 ? 0 : (bound >> 6);
        if (need <= PH || PH >= max_PH) return;
        long np = std::min<long>(std::max<long>(need + 2, 2L * PH), max_PH);
        if (np <= PH) return;
        uint64_t *nh = nullptr;
        if (hipMallocAsync((void **)&nh, (size_t)np * ((size_t)n_b + 1) * 8, s) != hipSuccess) {
            (void)hipGetLastError();
            max_PH = PH;   // no room: colors past the words take the neighbourhood walk
            return;
        }
        k_grow_planes<<<grid_for((long)np * n_b, nthr, di.cus * 16), nthr, 0, s>>>(hw, PH, nh, (int)np, n_b);
        if (hw) (void)hipFreeAsync(hw, s);
        hw = nh;
        PH = (int)np;
    };
    // pinned counters live for the thread's lifetime (never freed: freeing at
    // thread exit could run after the HIP runtime has shut down)
    // (none without allocation: rounds are then checked by plain copies)
    HostProgress no_prog(nullptr);
    EventPool no_events;
    if (!noalloc && !t_prog) t_prog = new HostProgress();
    HostProgress *prog_p = noalloc ? &no_prog : t_prog;
    HostProgress &prog = *prog_p;
    if (!noalloc && !t_evpool) t_evpool = new EventPool();
    EventPool *evpool_p = noalloc ? &no_events : t_evpool;
    EventPool &evpool = *evpool_p;
    evpool.used = 0;
    const int prof_kernel = o.prof ? o.prof->kernel : -1;
    if (o.prof) {
        o.prof->launches = 0;
        o.prof->ms = 0.0;
        o.prof->bytes = 0.0;
        o.prof->bytes_scanned = 0.0;
        o.prof->bytes_states = 0.0;
    }
#define PCNT(r) ((r) < prof_rounds ? pcnt + (size_t)(r) * PROF_SLOTS * 4 : nullptr)
    if (prof_rounds)
        k_fill_i32<<<grid_for((long)prof_rounds * PROF_SLOTS * 8, nthr, di.cus * 4), nthr, 0, s>>>(
            (int *)pcnt, 0, (long)prof_rounds * PROF_SLOTS * 8);
#define LAUNCH_PROF(kid, launch)                                  \
    do {                                                          \
        hipEvent_t e0_ = nullptr, e1_ = nullptr;                  \
        if (prof_kernel == (kid)) {                               \
            e0_ = evpool.next();                                  \
            if (e0_) hipEventRecord(e0_, s);                      \
        }                                                         \
        launch;                                                   \
        if (prof_kernel == (kid) && e0_) {                        \
            e1_ = evpool.next();                                  \
            if (e1_) hipEventRecord(e1_, s);                      \
        }                                                         \
    } while (0)

    // FNV-1a-64 of the int32 colors implied by the states: tentative (every
    // proposal counts as a color) or snapshot (proposals count as -1)
    auto hash_states = [&](int r, bool tentative) -> bool {
        if (!hash_mode || r >= o.log->cap) return true;
        uint64_t *dst = tentative ? o.log->hash_t : o.log->hash_c;
        if (!dst) return true;
        if (hipMemcpyAsync(h_states, st, sizeof(int) * (size_t)n_a, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return false;
        uint64_t h = 0xcbf29ce484222325ull;
        for (int i = 0; i < n_a; i++) {
            const int v = h_states[i];
            const int c = tentative ? (v < 0 ? -1 : (v & COLOR_MASK)) : ((v >= 0 && !(v & TENT)) ? v : -1);
            const uint32_t u = (uint32_t)c;
            for (int b = 0; b < 4; b++) {
                h ^= (u >> (8 * b)) & 0xffu;
                h *= 0x100000001b3ull;
            }
        }
        dst[r] = h;
        return true;
    };
    auto mark_round = [&]() {
        if (!time_rounds || (int)round_ev.size() > o.log->cap) return;
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) == hipSuccess && hipEventRecord(e, s) == hipSuccess) round_ev.push_back(e);
        else (void)hipGetLastError();
    };
    if (hash_mode && hipHostMalloc((void **)&h_states, sizeof(int) * ((size_t)n_a + 1)) != hipSuccess) {
        (void)hipGetLastError();
        h_states = nullptr;
        st_code = BGPC_E_OOM;
        goto finish;
    }

    // ---- shape of the graph: largest net, big nets, distance-2 bound
    k_fill_i32<<<1, 64, 0, s>>>(shape, 0, 8);
    k_fill_i32<<<grid_for(rec_cap * (long)sizeof(RoundRec) / 4, nthr, di.cus * 4), nthr, 0, s>>>(
        (int *)rec, 0, rec_cap * (long)sizeof(RoundRec) / 4);
    k_net_shape<D2><<<g_b, nthr, 0, s>>>(g, &shape[0], big, &shape[1], (unsigned long long *)&shape[4], &shape[2],
                                         huge, &shape[3]);
    LAUNCH_CHECK();
    if (hipMemcpyAsync(h_shape, shape, sizeof(h_shape), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        st_code = BGPC_E_HIP;
        goto finish;
    }
    {
        const int max_net = h_shape[0];
        const int n_big = h_shape[1];
        const int n_huge = h_shape[3];
        // front-driven rounds need every net on the small-net removal path
        // (its candidate listing) and standing proposals
        const bool front = front_possible && n_big == 0 && n_huge == 0 && max_net <= SMALL_NET &&
                           !(o.flags & BGPC_NET_BALANCE);
        if (!D2 && sp_on && !noalloc && max_net >= 2 && n_big == 0 && (long)std::min(max_net, ELL_W) * n_b < (1L << 31)) {
            ell_w = std::min(max_net, ELL_W);
            if (hipMallocAsync((void **)&ell, (size_t)ell_w * (size_t)n_b * 4, s) != hipSuccess) {
                (void)hipGetLastError();
                ell = nullptr;
                ell_w = 0;
            } else {
                k_build_ell<<<grid_for(n_b, ELL_BLOCK, di.cus * 8), ELL_BLOCK, 0, s>>>(g, ell_w, ell);
            }
        }
        if (sp_on && !noalloc && n_big > 0) {
            if (hipMallocAsync((void **)&pend_l, (size_t)(a.nnz + (D2 ? n_b : 0) + 1) * 4, s) != hipSuccess ||
                hipMallocAsync((void **)&pend_n, ((size_t)n_b + 1) * 4, s) != hipSuccess) {
                (void)hipGetLastError();
                if (pend_l) (void)hipFreeAsync(pend_l, s);
                pend_l = pend_n = nullptr;
            }
            sp_state.pl = pend_l;
            sp_state.pn = pend_n;
        }
        // distance-2 degree bound: most nets of a vertex x largest net
        const long two_hop = std::min<long>((long)h_shape[2] * (long)max_net, 1L << 30);
        unsigned long long walk;
        std::memcpy(&walk, &h_shape[4], sizeof(walk));
        // small dense graphs under plain first-fit vertex rounds: one workgroup
        // with an explicit conflict bit matrix (the batch kernel's dense mode)
        if (!D2 && !any_net_round && policy == BGPC_FIRST_FIT && !resume && !(o.flags & BGPC_INCREMENTAL) &&
            !o.prof && !noalloc && n_a <= DENSE_ROUTE_N && (double)walk > 4.0 * (double)n_a * (double)n_a) {
            std::vector<int> lg;
            int rounds = 0;
            const int lcap = o.log ? std::min(o.log->cap, max_rounds) : 0;
            st_code = color_one_workgroup(g, st, max_rounds, s, lcap, &lg, &rounds);
            if (st_code == BGPC_OK || st_code == BGPC_E_NOT_CONVERGED) {
                if (o.rounds_out) *o.rounds_out = rounds;
                if (o.log) {
                    int k = (int)lg.size() / 3;
                    for (int i = 0; i < k; i++) {
                        if (o.log->mode) o.log->mode[i] = 0;
                        if (o.log->w_size) o.log->w_size[i] = lg[3 * i];
                        if (o.log->losers) o.log->losers[i] = lg[3 * i + 1];
                        if (o.log->evicted) o.log->evicted[i] = 0;
                        if (o.log->max_color) o.log->max_color[i] = lg[3 * i + 2];
                    }
                    o.log->n = k;
                }
            }
            ar.release();
            hipStreamSynchronize(s);
            return st_code;
        }
        const int lds_total = std::min(di.lds_max, 65536);
        const int lds_budget = lds_total - 10240;   // beside the kernels' static LDS
        // bitmap capacity of the wide vertex paths, in bits
        long need_bits = std::max<long>(two_hop + 2, max_net + 1) + chunk + 66;
        const int lds_bits = (int)std::min<long>(((need_bits + 31) / 32) * 32, (long)lds_budget * 8);
        // per-net color words past 63 where the distance-2 walk is costly
        // (nets of more than SMALL_NET members) or cannot hold every color
        // (bound past the LDS bitmap); elsewhere the walk is cheaper
        planes_ok = planes_ok && (tune.planes == 1 || (tune.planes < 0 && (n_big > 0 || need_bits > lds_bits)) ||
                                  need_bits > lds_bits);
        const int wide_bytes = lds_bits / 8;
        // net-based rounds: bitmap + suffix counts of the largest net
        const int ncolor_words = std::min(lds_budget / 4, 2 * ((max_net + 31) / 32) + 2);
        if (any_net_round && 2 * ((max_net + 31) / 32) + 1 > lds_budget / 4) {
            st_code = BGPC_E_UNSUPPORTED;
            goto finish;
        }
        const int conflict_bytes = (int)(WIN_COLORS * sizeof(int));
        // nets above HASH_MAX members in vertex-based rounds: block per net, a
        // proposal list as long as the LDS allows (7 ints per proposal)
        int huge_list = 0;
        const int huge_lds = std::min(di.lds_max, 163840) - 1024;
        if (n_huge > 0 && huge_lds >= conflict_bytes) {
            huge_list = 64;
            while (7 * 4 * (2 * huge_list) <= huge_lds) huge_list <<= 1;
        }
        const int huge_bytes = std::max(7 * 4 * huge_list, conflict_bytes);
        if (huge_list && huge_bytes > 65536 &&
            hipFuncSetAttribute((const void *)k_conflict_huge<D2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                huge_bytes) != hipSuccess) {
            (void)hipGetLastError();
            huge_list = 0;   // the block-per-net kernel takes them as well
        }
        const int huge_on = huge_list > 0 ? 1 : 0;
        const int g_huge = std::max(1, std::min(n_huge, di.cus * 2));
        if (lds_total < conflict_bytes) {
            st_code = BGPC_E_UNSUPPORTED;
            goto finish;
        }

        if (any_net_round) k_owner<D2><<<g_a, nthr, 0, s>>>(g, owner);
        if (policy != BGPC_FIRST_FIT && planes_ok) {
            // vertices of more than HEAVY_NETS nets (fewer than incidences / HEAVY_NETS)
            const long inc = a.nnz + (D2 ? n_a : 0);
            const long cap_h = std::min<long>(n_a, inc / (HEAVY_NETS + 1) + 1);
            const long cap_s = inc / HEAVY_SLICE + cap_h + 1;
            int h_counts[2] = {0, 0};
            bool ok = hipMallocAsync((void **)&hv_id, sizeof(int) * ((size_t)n_a + 1), s) == hipSuccess &&
                      hipMallocAsync((void **)&hv_list, sizeof(int) * (size_t)cap_h, s) == hipSuccess &&
                      hipMallocAsync((void **)&hv_slices, sizeof(HeavySlice) * (size_t)cap_s, s) == hipSuccess &&
                      hipMallocAsync((void **)&hv_counts, 64, s) == hipSuccess;
            if (ok) {
                k_fill_i32<<<1, 64, 0, s>>>(hv_counts, 0, 2);
                k_heavy_mark<D2><<<g_a, nthr, 0, s>>>(g, hv_id, hv_list, hv_slices, hv_counts);
                ok = hipMemcpyAsync(h_counts, hv_counts, sizeof(h_counts), hipMemcpyDeviceToHost, s) == hipSuccess &&
                     hipStreamSynchronize(s) == hipSuccess;
            }
            if (!ok) (void)hipGetLastError();
            hv_H = ok ? h_counts[0] : 0;   // none (or no room): every vertex walks its own nets
        }

        // ---- initial state
        k_fill_u8<<<g_a, nthr, 0, s>>>(lose, 0, n_a + 1);
        k_fill_i32<<<g_a, nthr, 0, s>>>(ffc, 0, n_a + 1);
        k_fill_u8<<<g_b, nthr, 0, s>>>(done_net, 0, n_b + 1);
        clear_inc_bits();
        if (!resume) {
            // front-driven rounds start every vertex on its standing proposal 0
            // (first-fit with nothing colored)
            k_fill_i32<<<g_a, nthr, 0, s>>>(st, front ? TENT : -1, n_a);
            if (front) {
                k_fill_i32<<<g_a, nthr, 0, s>>>(infront, 0, n_a + 1);
                k_fill_i32<<<g_b, nthr, 0, s>>>(dstamp, 0, n_b + 1);
                k_iota<<<g_b, nthr, 0, s>>>(DL, n_b);   // the first round rescans every net
            }
            k_iota<<<g_a, nthr, 0, s>>>(W0, n_a);
            k_fill_u64<<<g_b, nthr, 0, s>>>(mask0, 0ull, n_b + 1);
            k_init_ctrl<<<1, 64, 0, s>>>(ctrl, n_a, -1);
            if (front) k_fill_i32<<<1, 64, 0, s>>>(&ctrl->dl_n, n_b, 1);
        } else {
            k_init_ctrl<<<1, 64, 0, s>>>(ctrl, 0, -1);
            k_check_colors<<<g_a, nthr, 0, s>>>(st, n_a, 1 << 29, &ctrl->error);
            if (hipMemcpyAsync(&h_ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st_code = BGPC_E_HIP;
                goto finish;
            }
            if (h_ctrl.error) {
                st_code = BGPC_E_INVALID;
                goto finish;
            }
            k_max_color<<<g_a, nthr, 0, s>>>(st, n_a, ctrl);
            {
                // colors present: size the higher color words before the rebuild
                if (hipMemcpyAsync(&h_ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    st_code = BGPC_E_HIP;
                    goto finish;
                }
                mc_ub = h_ctrl.max_color;
                if (planes_ok) ensure_planes(mc_ub + 1);
            }
            k_mask_rebuild<D2><<<g_b, nthr, 0, s>>>(g, st, mask0, hw, PH);
            const int gt = grid_for(max_tiles, 1, di.cus * (tune.apply_grid > 0 ? tune.apply_grid : 4));
            k_count_uncolored<<<gt, TILE_BLOCK, 0, s>>>(st, n_a, tile_count);
            // identity compaction: the uncolored vertices in id order become W0
            k_compact<<<gt, TILE_BLOCK, 0, s>>>(nullptr, n_a, ctrl, 1, st, tile_count, W0, rec, 0, 0, 0, nullptr);
        }
        LAUNCH_CHECK();

        if (prog.h) {
            prog.h[0] = -1;
            prog.h[1] = -1;
            prog.h[2] = 0;
            prog.h[3] = -1;
        }

        // ---- rounds
        const int gt = grid_for(max_tiles, 1, di.cus * (tune.apply_grid > 0 ? tune.apply_grid : 4));
        const int g_big = std::max(1, std::min(n_big, di.cus * 4));
        const int g_chunk = grid_for((n_a + chunk - 1) / chunk, 1, di.cus * 16);
        // first-fit vertex rounds after the last net-based round run
        // incrementally (graphs whose nets all run thread-per-net)
        const bool inc_ok = (o.flags & BGPC_INCREMENTAL) && policy == BGPC_FIRST_FIT && n_big == 0 &&
                            max_net <= SMALL_NET;
        int last_net = -1;
        for (int r = 0; r < max_rounds && start_round + r < 64; r++)
            if ((o.net_color_mask >> (start_round + r)) & 1ull) last_net = r;
        const int inc_start = inc_ok ? last_net + 1 : 0x7fffffff;
        const int g_inc = di.cus * 4;
        bool done = false;
        bool use_prog = prog.h && prog.d;
        bool inc_used = false;
        int net_round_issued = -1;   // last net-based round queued
        bool zf_valid = false;       // zf matches the masks (kept by the rounds that pass it)
        // one wave per 64 items, grids a multiple of 8 (XCD-aware remap)
        auto grid64 = [&](long items) {
            long gsz = (items + 63) / 64;
            gsz = std::min<long>(gsz, (long)di.cus * 32);
            gsz = std::max<long>(8, (gsz + 7) / 8 * 8);
            return (int)gsz;
        };
        // first-fit: one resident pass of workgroups (the LDS staging buffer
        // limits residency; a second partial pass of workgroups costs more than
        // the longer per-wave loop)
        const int g_w64a = std::min(grid64(n_a), std::max(8, di.cus * (tune.color_grid > 0 ? tune.color_grid
                                                                                  : resident_per_cu<D2>()) / 8 * 8));
        const int g_w64b = tune.removal_grid > 0 ? std::min(grid64(n_b), std::max(8, di.cus * tune.removal_grid / 8 * 8))
                                                 : grid64(n_b);
        // standing-proposal removal: one resident pass of workgroups
        const int g_sp = std::min(grid64(n_b), std::max(8, di.cus * (tune.removal_grid > 0 ? tune.removal_grid
                                                                           : resident_sp_per_cu<D2>()) / 8 * 8));
        const int g_list = di.cus * (tune.removal_grid > 0 ? tune.removal_grid : 8);
        const int g_fa = grid_for(((long)n_a + 3) / 4, APPLY_BLOCK, di.cus * (tune.apply_grid > 0 ? tune.apply_grid : 8));
        // balanced net rounds: a wave per chunk of net ids, an LDS bitmap of
        // 16 bits per member of the largest net (at least 16 KB), within the budget
        const int bal_bytes = (int)std::min<long>(lds_budget, std::max<long>(16384, (16L * max_net + 64) / 8 + 64) / 4 * 4);
        const int g_nbal = std::max(1, std::min((n_b + chunk - 1) / chunk, di.cus * 16));
        mark_round();
        while (!done && issued < max_rounds) {
            // keep at most LOOKAHEAD rounds in flight beyond the last one seen
            if (use_prog) {
                long spins = 0;
                for (;;) {
                    int seen = prog.h[0];
                    std::atomic_thread_fence(std::memory_order_acquire);
                    int nw = prog.h[1];
                    if ((seen >= 0 && nw == 0) || prog.h[2] != 0) {
                        done = true;
                        break;
                    }
                    if (issued - (seen + 1) < LOOKAHEAD) break;
                    if ((++spins & 1023) == 0) {
                        hipError_t q = hipStreamQuery(s);
                        if (q == hipSuccess) {
                            // all queued work is complete but not seen: stop
                            // relying on the host mapping and read the device
                            if (hipMemcpy(&h_ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) {
                                st_code = BGPC_E_HIP;
                                goto finish;
                            }
                            use_prog = false;
                            if (h_ctrl.n_w[issued & 1] == 0 || h_ctrl.error) done = true;
                            break;
                        }
                        if (q != hipErrorNotReady) {
                            st_code = BGPC_E_HIP;
                            goto finish;
                        }
                    }
                    std::this_thread::yield();
                }
                if (done) break;
            } else if (issued > 0 && issued % LOOKAHEAD == 0) {
                if (hipMemcpyAsync(&h_ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    st_code = BGPC_E_HIP;
                    goto finish;
                }
                if (h_ctrl.n_w[issued & 1] == 0 || h_ctrl.error) break;
            }
            const int r = issued;
            const int rr = std::min(r, rec_cap - 2);   // record slot
            const int par = r & 1;
            const int rid = start_round + r;
            const bool net_mode = rid >= 0 && rid < 64 && ((o.net_color_mask >> rid) & 1ull);
            int *Wc = Wb[par], *Wn = Wb[par ^ 1];
            int *host = use_prog ? prog.d : nullptr;
            if (planes_ok) {
                // a vertex-based round raises the largest color by at most one;
                // a net-based round colors below the largest net
                if (use_prog) {
                    int seen = prog.h[0], mc = prog.h[3];
                    if (seen >= 0 && net_round_issued <= seen) mc_ub = std::min(mc_ub, (long)mc + (r - 1 - seen));
                }
                mc_ub = net_mode ? std::max<long>(mc_ub, max_net - 1) : mc_ub + 1;
                ensure_planes(mc_ub);
            }
            if (net_mode && sp_used && !sp_reset) {
                // losers of the previous vertex-based round hold their
                // proposals: a net-based round starts from them uncolored
                k_drop_proposals<<<g_a, nthr, 0, s>>>(st, n_a);
                sp_reset = true;
            }
            if (!net_mode && r < inc_start && sp_on && sp_reset) {
                k_fill_i32<<<grid_for((long)sp_words * 2, nthr, di.cus * 8), nthr, 0, s>>>((int *)sp_bits, 0,
                                                                                           (long)sp_words * 2);
                k_fill_i32<<<g_a, nthr, 0, s>>>(sp_cnt, 0, n_a + 1);
                k_fill_u8<<<g_b, nthr, 0, s>>>(sp_dirty, 1, n_b + 1);
                if (pend_l) k_pending_init<D2><<<g_big, 256, 0, s>>>(g, big, &shape[1], pend_l, pend_n);
                if (pend_l && !ell) k_pending_init_small<D2><<<g_b, nthr, 0, s>>>(g, pend_l, pend_n);
                sp_reset = false;
            }
            const bool spr = !net_mode && r < inc_start && sp_on;   // this round keeps standing proposals
            if (spr) sp_used = true;
            if (net_mode) {
                if (net_bal) {
                    k_ncolor_balanced<D2><<<g_nbal, 64, bal_bytes, s>>>(g, st, owner, ctrl, policy, chunk,
                                                                        bal_bytes * 8);
                } else {
                    k_ncolor_small<D2><<<g_b, nthr, 0, s>>>(g, st, owner, ctrl, o.net_alg);
                    if (n_big)
                        k_ncolor_big<D2><<<g_big, NBIG_BLOCK, ncolor_words * 4, s>>>(g, st, owner, big, &shape[1],
                                                                                     ctrl, ncolor_words, o.net_alg);
                }
                if (!D2) k_ncolor_isolated<<<g_a, nthr, 0, s>>>(g, Wc, ctrl, par, st);
                if (!hash_states(r, true)) {
                    st_code = BGPC_E_HIP;
                    goto finish;
                }
                if (vertex_form(r, true)) {
                    k_conflict_vertex<D2><<<g_a, nthr, 0, s>>>(g, Wc, ctrl, par, st, lose);
                } else {
                    LAUNCH_PROF(BGPC_PROF_CONFLICT, (k_conflict_small<D2><<<g_w64b, 64, 0, s>>>(g, st, lose, done_net, 0, PCNT(r), sp_none)));
                    if (n_big)
                        k_conflict_big<D2><<<g_big, BIG_BLOCK, conflict_bytes, s>>>(g, st, lose, done_net, big, &shape[1],
                                                                                   ctrl, 0, sp_none, 0);
                }
                const bool full = r > 0 || resume;
                if (full) {
                    k_set_max_final<<<1, 64, 0, s>>>(ctrl, -1);
                    k_apply<D2><<<gt, TILE_BLOCK, 0, s>>>(g, nullptr, ctrl, par, st, lose, mask0, tile_count, rec, rr, 0,
                                                          hw, PH, nullptr);
                    k_compact<<<gt, TILE_BLOCK, 0, s>>>(nullptr, n_a, ctrl, par, st, tile_count, Wn, rec, rr, 1, 1, host);
                    k_mask_rebuild<D2><<<g_b, nthr, 0, s>>>(g, st, mask0, hw, PH);
                    k_fill_i32<<<g_a, nthr, 0, s>>>(ffc, 0, n_a + 1);
                    k_fill_u8<<<g_b, nthr, 0, s>>>(done_net, 0, n_b + 1);
                    clear_inc_bits();
                } else {
                    k_apply<D2><<<gt, TILE_BLOCK, 0, s>>>(g, Wc, ctrl, par, st, lose, mask0, tile_count, rec, rr, 1, hw, PH,
                                                          nullptr);
                    k_compact<<<gt, TILE_BLOCK, 0, s>>>(Wc, n_a, ctrl, par, st, tile_count, Wn, rec, rr, 1, 1, host);
                }
                net_round_issued = r;
                zf_valid = false;
            } else if (r >= inc_start) {
                zf_valid = false;
                // the wide path can only be needed once colors 0..63 all exist
                bool need_wide = true;
                if (use_prog) {
                    int seen = prog.h[0], mc = prog.h[3];
                    if (seen >= 0 && net_round_issued <= seen) need_wide = (long)mc + (r - 1 - seen) >= 63;
                    else if (seen < 0 && !resume && net_round_issued < 0) need_wide = r >= 63;
                }
                if (r == inc_start) {
                    // full round whose losers keep their proposals
                    k_inc_reset<<<1, 64, 0, s>>>(ic);
                    LAUNCH_PROF(BGPC_PROF_COLOR, (k_vcolor_ff<D2><<<g_w64a, 64, 0, s>>>(g, Wc, ctrl, par, st, mask0, heavy, PCNT(r), hw, PH, ffc, nullptr)));
                    if (need_wide)
                        k_vcolor_wide<D2><<<di.cus * 2, 256, wide_bytes, s>>>(g, heavy, ctrl, st, lds_bits, nullptr,
                                                                               nullptr, nullptr, nullptr, nullptr,
                                                                               hw, PH, ffc, nullptr);
                    if (!hash_states(r, true)) {
                        st_code = BGPC_E_HIP;
                        goto finish;
                    }
                    LAUNCH_PROF(BGPC_PROF_CONFLICT, (k_conflict_small<D2><<<g_w64b, 64, 0, s>>>(g, st, lose, done_net, 1, PCNT(r), sp_none)));
                    k_inc_apply_full<D2><<<g_inc, nthr, 0, s>>>(g, ic, ctrl, par, Wc, st, lose, mask0, cn_bits, CNl);
                } else {
                    k_inc_color<D2><<<g_inc, nthr, 0, s>>>(g, ic, par, Dl[par], dirty_bits, st, mask0, aff_bits, Al,
                                                           tchg_bits, TCNl, heavy, ctrl);
                    if (need_wide)
                        k_vcolor_wide<D2><<<di.cus * 2, 256, wide_bytes, s>>>(g, heavy, ctrl, st, lds_bits, ic,
                                                                               aff_bits, Al, tchg_bits, TCNl,
                                                                               nullptr, 0, nullptr, nullptr);
                    if (!hash_states(r, true)) {
                        st_code = BGPC_E_HIP;
                        goto finish;
                    }
                    k_expand<D2><<<g_inc, nthr, 0, s>>>(g, TCNl, &ic->n_tcn, tchg_bits, st, aff_bits, Al, &ic->n_a);
                    k_inc_conflict<D2><<<g_inc, nthr, 0, s>>>(g, ic, par, Al, aff_bits, st, WINl, ctrl);
                    k_inc_apply<D2><<<g_inc, nthr, 0, s>>>(g, ic, WINl, st, mask0, cn_bits, CNl, ctrl);
                }
                k_expand<D2><<<g_inc, nthr, 0, s>>>(g, CNl, &ic->n_cn, cn_bits, st, dirty_bits, Dl[par ^ 1],
                                                    &ic->n_d[par ^ 1]);
                k_inc_close<<<1, 64, 0, s>>>(ic, ctrl, par, rec, rr, host);
                inc_used = true;
            } else {
                uint8_t *dty = spr ? sp_dirty : nullptr;
                const SPState &spx = spr ? sp_state : sp_none;
                // first-fit skips standing proposals 0 of vertices without a
                // net holding color 0 (zf, kept up to date by k_apply)
                const bool zfr = spr && policy == BGPC_FIRST_FIT && !front;
                if (front) {
                    const DirtyList dlr{DL, &ctrl->dl_n, dstamp, r};
                    LAUNCH_PROF(BGPC_PROF_COLOR, (k_vcolor_ff<D2, true><<<g_w64a, 64, 0, s>>>(g, FL[par], ctrl, par, st, mask0, heavy, PCNT(r), hw, PH, ffc, dty, &ctrl->fl_n[par], FL[par ^ 1], &ctrl->fl_n[par ^ 1], dlr)));
                    bool need_wide = true;
                    if (use_prog) {
                        int seen = prog.h[0], mc = prog.h[3];
                        if (seen >= 0) need_wide = (long)mc + (r - 1 - seen) >= 63;
                        else need_wide = r >= 63;
                    }
                    if (need_wide)
                        k_vcolor_wide<D2><<<di.cus * 2, 256, wide_bytes, s>>>(g, heavy, ctrl, st, lds_bits, nullptr,
                                                                               nullptr, nullptr, nullptr, nullptr,
                                                                               hw, PH, ffc, dty, dlr);
                } else if (policy == BGPC_FIRST_FIT) {
                    if (zfr && !zf_valid) {
                        // before any color exists nothing holds color 0
                        if (!resume && net_round_issued < 0) k_fill_u8<<<g_a, nthr, 0, s>>>(zf, 0, n_a + 1);
                        else k_zero_front_init<D2><<<g_a, nthr, 0, s>>>(g, mask0, zf);
                        zf_valid = true;
                    }
                    LAUNCH_PROF(BGPC_PROF_COLOR, (k_vcolor_ff<D2><<<g_w64a, 64, 0, s>>>(g, Wc, ctrl, par, st, mask0, heavy, PCNT(r), hw, PH, ffc, dty, nullptr, nullptr, nullptr, DirtyList{nullptr, nullptr, nullptr, 0}, zfr ? zf : nullptr)));
                    // the wide path can only be needed once colors 0..63 all exist:
                    // a vertex-based first-fit round raises the largest color by at
                    // most one, a net-based round keeps it below the largest net
                    bool need_wide = true;
                    if (use_prog) {
                        int seen = prog.h[0], mc = prog.h[3];
                        if (seen >= 0 && net_round_issued <= seen) {
                            long bound = (long)mc + (r - 1 - seen);
                            need_wide = bound >= 63;
                        } else if (seen < 0 && !resume && net_round_issued < 0) {
                            need_wide = r >= 63;
                        }
                    }
                    if (need_wide)
                        k_vcolor_wide<D2><<<di.cus * 2, 256, wide_bytes, s>>>(g, heavy, ctrl, st, lds_bits, nullptr,
                                                                               nullptr, nullptr, nullptr, nullptr,
                                                                               hw, PH, ffc, dty);
                } else {
                    const uint64_t *Fp = nullptr;
                    if (hv_H > 0 && PH > 0) {
                        if (hv_stride != PH + 1) {
                            // rows follow the number of color words (rewritten every round)
                            if (hv_F) (void)hipFreeAsync(hv_F, s);
                            hv_F = nullptr;
                            hv_stride = 0;
                            if (hipMallocAsync((void **)&hv_F, (size_t)hv_H * (PH + 1) * 8, s) != hipSuccess) {
                                (void)hipGetLastError();
                                hv_F = nullptr;
                                hv_H = 0;
                            } else {
                                hv_stride = PH + 1;
                            }
                        }
                        if (hv_F) {
                            const long nw = (long)hv_H * (PH + 1);
                            k_fill_u64<<<grid_for(nw, nthr, di.cus * 8), nthr, 0, s>>>(hv_F, 0ull, nw);
                            k_heavy_words<D2><<<di.cus * 8, 256, 0, s>>>(g, st, hv_list, hv_slices, hv_counts, mask0,
                                                                        hw, PH, ctrl, hv_F);
                            Fp = hv_F;
                        }
                    }
                    k_vcolor_chunked<D2><<<g_chunk, 64, wide_bytes, s>>>(g, Wc, ctrl, par, st, mask0, policy, chunk,
                                                                          lds_bits, hw, PH, dty, Fp ? hv_id : nullptr,
                                                                          Fp);
                }
                if (!hash_states(r, true)) {
                    st_code = BGPC_E_HIP;
                    goto finish;
                }
                if (vertex_form(r, false)) {
                    k_conflict_vertex<D2><<<g_a, nthr, 0, s>>>(g, Wc, ctrl, par, st, lose);
                } else {
                    if (front)
                        LAUNCH_PROF(BGPC_PROF_CONFLICT, (k_conflict_list<D2><<<g_list, LIST_BLOCK, 0, s>>>(g, st, done_net, sp_state, DL, &ctrl->dl_n, PCNT(r))));
                    else if (spr && ell)
                        LAUNCH_PROF(BGPC_PROF_CONFLICT, (k_conflict_small<D2, true, !D2><<<g_sp, 64, 0, s>>>(g, st, lose, done_net, 1, PCNT(r), sp_state, ell, ell_w)));
                    else if (spr && pend_l)
                        LAUNCH_PROF(BGPC_PROF_CONFLICT, (k_conflict_small<D2, true, false, true><<<g_sp, 64, 0, s>>>(g, st, lose, done_net, 1, PCNT(r), sp_state)));
                    else if (spr)
                        LAUNCH_PROF(BGPC_PROF_CONFLICT, (k_conflict_small<D2, true><<<g_sp, 64, 0, s>>>(g, st, lose, done_net, 1, PCNT(r), sp_state)));
                    else
                        LAUNCH_PROF(BGPC_PROF_CONFLICT, (k_conflict_small<D2><<<g_w64b, 64, 0, s>>>(g, st, lose, done_net, 1, PCNT(r), sp_none)));
                    if (spr && prof_kernel == BGPC_PROF_CONFLICT && PCNT(r))
                        k_census<D2><<<g_b, nthr, 0, s>>>(g, st, PCNT(r));
                    if (n_big)
                        k_conflict_big<D2><<<g_big, BIG_BLOCK, conflict_bytes, s>>>(g, st, lose, done_net, big, &shape[1],
                                                                                   ctrl, 1, spx, huge_on);
                    if (huge_on)
                        k_conflict_huge<D2><<<g_huge, HUGE_BLOCK, huge_bytes, s>>>(g, st, lose, done_net, huge, &shape[3],
                                                                                 ctrl, 1, spx, huge_list);
                }
                if (front) {
                    // winners (all vertices streamed); closes the round; then
                    // the members of nets that gained color 0 join the front
                    k_front_apply<D2><<<g_fa, APPLY_BLOCK, 0, s>>>(g, sp_cnt, st, mask0, hw, PH, ZL[par],
                                                                  &ctrl->zl_n[par], ctrl, par, rec, rr, host,
                                                                  &ctrl->dl_n, &ctrl->fl_n[par], &ctrl->zl_n[par ^ 1]);
                    k_front_push<D2><<<di.cus * 8, 256, 0, s>>>(g, ZL[par], &ctrl->zl_n[par], st, infront,
                                                                 FL[par ^ 1], &ctrl->fl_n[par ^ 1]);
                } else {
                    k_apply<D2><<<gt, TILE_BLOCK, 0, s>>>(g, Wc, ctrl, par, st, lose, mask0, tile_count, rec, rr, 1, hw,
                                                          PH, spr ? sp_cnt : nullptr, zfr ? zf : nullptr, z0l);
                    k_compact<D2><<<gt, TILE_BLOCK, 0, s>>>(Wc, n_a, ctrl, par, st, tile_count, Wn, rec, rr, 0, 1, host,
                                                            g, z0l, zfr ? zf : nullptr);
                    if (!zfr) zf_valid = false;
                }
            }
            LAUNCH_CHECK();
            mark_round();
            if (!hash_states(r, false)) {
                st_code = BGPC_E_HIP;
                goto finish;
            }
            issued++;
        }
        if (inc_used || sp_used) k_drop_proposals<<<g_a, nthr, 0, s>>>(st, n_a);
        LAUNCH_CHECK();
    }

finish:
    if (hipMemcpyAsync(&h_ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        if (st_code == BGPC_OK) st_code = BGPC_E_HIP;
    }
    if (st_code == BGPC_OK) {
        if (h_ctrl.error & (ERR_COLOR_CAP | ERR_NET_TOO_BIG)) st_code = BGPC_E_UNSUPPORTED;
        else if (h_ctrl.error) st_code = BGPC_E_INTERNAL;
        else if (h_ctrl.n_w[issued & 1] != 0) st_code = BGPC_E_NOT_CONVERGED;
    }
    if (o.prof && evpool.used >= 2 && (st_code == BGPC_OK || st_code == BGPC_E_NOT_CONVERGED)) {
        double ms = 0.0;
        for (int i = 0; i + 1 < evpool.used; i += 2) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, evpool.ev[i], evpool.ev[i + 1]) == hipSuccess) ms += t;
        }
        o.prof->ms = ms;
        o.prof->launches = evpool.used / 2;
        // algorithmic bytes from the per-round counters
        int k = std::min(std::min(h_ctrl.rounds, rec_cap - 2), prof_rounds);
        std::vector<RoundRec> rr_h(std::max(k, 1));
        std::vector<unsigned long long> pc_h((size_t)std::max(k, 1) * PROF_SLOTS * 4);
        if (k > 0 && hipMemcpy(rr_h.data(), rec, sizeof(RoundRec) * k, hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(pc_h.data(), pcnt, sizeof(unsigned long long) * k * PROF_SLOTS * 4,
                      hipMemcpyDeviceToHost) == hipSuccess) {
            double bytes = 0.0, scanned = 0.0, alt = 0.0;
            for (int i = 0; i < k; i++) {
                double nets = 0, mem = 0, rows = 0, smem = 0;
                for (int q = 0; q < PROF_SLOTS; q++) {
                    nets += (double)pc_h[((size_t)i * PROF_SLOTS + q) * 4 + 0];
                    mem += (double)pc_h[((size_t)i * PROF_SLOTS + q) * 4 + 1];
                    rows += (double)pc_h[((size_t)i * PROF_SLOTS + q) * 4 + 2];
                    smem += (double)pc_h[((size_t)i * PROF_SLOTS + q) * 4 + 3];
                }
                if (prof_kernel == BGPC_PROF_CONFLICT) {
                    // net form of removal, per net of the round (a net with a
                    // member uncolored or proposing): two offsets, then per
                    // member its id and its state
                    bytes += 8.0 * nets + 8.0 * mem;
                    // the same over the nets actually read (their count is
                    // not kept: counted per member / average size)
                    const double snets = mem > 0 ? nets * smem / mem : 0.0;
                    scanned += 8.0 * snets + 8.0 * smem;
                    // per net one offset and the member ids, every member
                    // state read once per round (at most n_a distinct)
                    alt += 4.0 * nets + 4.0 * mem + 4.0 * std::min(mem, (double)n_a);
                } else if (prof_kernel == BGPC_PROF_COLOR && rr_h[i].mode == 0) {
                    // per entry: id, two row offsets, proposal; per incidence: net
                    // id; every net mask once (at most n_b distinct)
                    const double b = 16.0 * rr_h[i].w + 4.0 * rows + 8.0 * std::min(rows, (double)n_b);
                    bytes += b;
                    scanned += b;
                    alt += b;
                }
            }
            o.prof->bytes_scanned = scanned;
            o.prof->bytes = bytes;
            o.prof->bytes_states = alt;
        }
    }
    if (st_code == BGPC_OK || st_code == BGPC_E_NOT_CONVERGED) {
        if (o.rounds_out) *o.rounds_out = h_ctrl.rounds;
        if (o.log && o.log->cap > 0) {
            int k = std::min(o.log->cap, h_ctrl.rounds);
            h_rec.resize(std::max(k, 1));
            if (k > 0 && (hipMemcpyAsync(h_rec.data(), rec, sizeof(RoundRec) * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
                          hipStreamSynchronize(s) != hipSuccess)) {
                st_code = BGPC_E_HIP;
            } else {
                for (int i = 0; i < k; i++) {
                    if (o.log->mode) o.log->mode[i] = h_rec[i].mode;
                    if (o.log->w_size) o.log->w_size[i] = h_rec[i].w;
                    if (o.log->losers) o.log->losers[i] = h_rec[i].losers;
                    if (o.log->evicted) o.log->evicted[i] = h_rec[i].evicted;
                    if (o.log->max_color) o.log->max_color[i] = h_rec[i].max_color;
                }
                o.log->n = k;
            }
        }
    }
    if (time_rounds && (st_code == BGPC_OK || st_code == BGPC_E_NOT_CONVERGED)) {
        const int k = std::min(std::min(o.log->cap, h_ctrl.rounds), (int)round_ev.size() - 1);
        for (int i = 0; i < k; i++) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, round_ev[i], round_ev[i + 1]) != hipSuccess) t = -1.f;
            o.log->round_ms[i] = t;
        }
    }
    for (hipEvent_t e : round_ev) (void)hipEventDestroy(e);
    if (h_states) (void)hipHostFree(h_states);
    if (hw) (void)hipFreeAsync(hw, s);
    for (void *p : {(void *)hv_id, (void *)hv_list, (void *)hv_slices, (void *)hv_counts, (void *)hv_F, (void *)ell,
                    (void *)pend_l, (void *)pend_n})
        if (p) (void)hipFreeAsync(p, s);
    ar.release();
    if (!ar.async) (void)hipGetLastError();
    hipStreamSynchronize(s);
    return st_code;
}

// d_err_ext: a device int to use instead of allocating one
int validate_bipartite(const bgpc_csr *A, const bgpc_csr *B, hipStream_t s, int *d_err_ext = nullptr)
{
    int *d_err = d_err_ext;
    if (!d_err) HIP_TRY(hipMallocAsync((void **)&d_err, 256, s));
    const DevInfo di = dev_info();
    k_fill_i32<<<1, 64, 0, s>>>(d_err, 0, 1);
    k_check_sorted<<<grid_for(A->n_rows, 256, di.cus * 8), 256, 0, s>>>(A->offsets, A->indices, A->n_rows, A->n_cols,
                                                                          d_err);
    k_check_sorted<<<grid_for(B->n_rows, 256, di.cus * 8), 256, 0, s>>>(B->offsets, B->indices, B->n_rows, B->n_cols,
                                                                          d_err);
    int h_err = 0;
    hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
    HIP_TRY(hipStreamSynchronize(s));
    if (h_err == 0) {
        int ends[2] = {0, 0};
        hipMemcpyAsync(&ends[0], A->offsets + A->n_rows, sizeof(int), hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(&ends[1], B->offsets + B->n_rows, sizeof(int), hipMemcpyDeviceToHost, s);
        k_check_transpose<<<grid_for(A->n_rows, 256, di.cus * 8), 256, 0, s>>>(A->offsets, A->indices, A->n_rows,
                                                                                 B->offsets, B->indices, 0, d_err);
        hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
        HIP_TRY(hipStreamSynchronize(s));
        if (ends[0] != A->nnz || ends[1] != B->nnz) h_err |= 1;
    }
    if (!d_err_ext) hipFreeAsync(d_err, s);
    hipStreamSynchronize(s);
    if (h_err & 1) return BGPC_E_INVALID;
    if (h_err & 2) return BGPC_E_UNSORTED;
    if (h_err & 4) return BGPC_E_NOT_TRANSPOSE;
    return BGPC_OK;
}

int validate_symmetric(const bgpc_csr *adj, hipStream_t s)
{
    int *d_err = nullptr;
    HIP_TRY(hipMallocAsync((void **)&d_err, 256, s));
    const DevInfo di = dev_info();
    k_fill_i32<<<1, 64, 0, s>>>(d_err, 0, 1);
    k_check_sorted<<<grid_for(adj->n_rows, 256, di.cus * 8), 256, 0, s>>>(adj->offsets, adj->indices, adj->n_rows,
                                                                            adj->n_cols, d_err);
    int h_err = 0;
    hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
    HIP_TRY(hipStreamSynchronize(s));
    if (h_err == 0) {
        int end = 0;
        hipMemcpyAsync(&end, adj->offsets + adj->n_rows, sizeof(int), hipMemcpyDeviceToHost, s);
        k_check_transpose<<<grid_for(adj->n_rows, 256, di.cus * 8), 256, 0, s>>>(
            adj->offsets, adj->indices, adj->n_rows, adj->offsets, adj->indices, 1, d_err);
        hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
        HIP_TRY(hipStreamSynchronize(s));
        if (end != adj->nnz) h_err |= 1;
    }
    hipFreeAsync(d_err, s);
    hipStreamSynchronize(s);
    if (h_err & 1) return BGPC_E_INVALID;
    if (h_err & 2) return BGPC_E_UNSORTED;
    if (h_err & (4 | 8)) return BGPC_E_NOT_SYMMETRIC;
    return BGPC_OK;
}

bool csr_ok(const bgpc_csr *c)
{
    return c && c->n_rows >= 0 && c->n_cols >= 0 && c->nnz >= 0 && c->nnz < (1ll << 31) &&
           c->n_rows < (1 << 30) && c->n_cols < (1 << 30) && c->offsets && (c->nnz == 0 || c->indices);
}

bool opts_ok(const bgpc_opts &o)
{
    return o.policy >= 0 && o.policy <= BGPC_B1_GLOBAL && o.chunk >= 1 && o.max_rounds >= 0 && o.start_round >= 0 &&
           o.net_alg >= BGPC_NET_ALG8 && o.net_alg <= BGPC_NET_ALG6_REVERSE &&
           (!(o.flags & BGPC_NET_BALANCE) || o.net_alg == BGPC_NET_ALG8);
}

}  // namespace

namespace {

// ---- caller orders (ranks = positions in `order`): the graph is relabelled
// to ranks on the device, colored in natural order, and the colors mapped back

// inv[order[k]] = k; err set when order is not a permutation of [0, n)
__global__ void k_order_inverse(const int *order, int n, int *mark, int *inv, int *err)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        unsigned v = (unsigned)order[k];
        if (v >= (unsigned)n || atomicAdd(&mark[v], 1) != 0) {
            atomicOr(err, 1);
            continue;
        }
        inv[v] = k;
    }
}

// size of rank k's row (the row of vertex order[k])
__global__ void k_rank_degree(const int *off, const int *order, int n, int *deg)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
        deg[k] = off[order[k] + 1] - off[order[k]];
}

// rows copied in rank order, one wave per row; entries mapped through map (if given)
__global__ void k_rank_rows(const int *off, const int *idx, const int *order, int n, const int *noff,
                            const int *map, int *nidx)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE, nwv = gridDim.x * blockDim.x / WAVE;
    for (int k = wid; k < n; k += nwv) {
        const int src = off[order[k]], len = off[order[k] + 1] - src, dst = noff[k];
        for (int j = lane; j < len; j += WAVE) {
            int x = idx[src + j];
            nidx[dst + j] = map ? map[x] : x;
        }
    }
}

__global__ void k_map_ids(const int *idx, long n, const int *map, int *out)
{
    for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x)
        out[j] = map[idx[j]];
}

// out[i] = in[perm[i]]
__global__ void k_gather_i32(const int *in, const int *perm, int n, int *out)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = in[perm[i]];
}

// ---- largest-first orders: key(u) = sum over the nets of u of (size - 1),
// one wave per vertex (lanes over its nets); ids for the stable sort
template <bool D2>
__global__ void k_order_key(Graph g, unsigned long long *key, int *ids)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE, nwv = gridDim.x * blockDim.x / WAVE;
    for (int u = wid; u < g.n_a; u += nwv) {
        const int nn = Acc<D2>::nets_count(g, u);
        unsigned long long s = 0;
        for (int k = lane; k < nn; k += WAVE) s += (unsigned long long)(Acc<D2>::size(g, Acc<D2>::net_at(g, u, k)) - 1);
        for (int d = WAVE / 2; d > 0; d >>= 1) s += (unsigned long long)__shfl_xor((long long)s, d);
        if (lane == 0) {
            key[u] = s;
            ids[u] = u;
        }
    }
}

// ---- smallest-last orders, removed in steps: key(x) = sum over the nets v
// of x of (members of v still present - 1) = base(x) - sum over those nets of
// removed(v); every step removes all present vertices whose key is at most
// d + (d >> shift), d the smallest key, and adds one to removed(v) for each
// net of each removed vertex.  Keys are recomputed from removed() every step
// (work proportional to the memberships still present, whatever the net
// sizes).

// keys of the present vertices R[0..n) and their minimum (atomicMin into *dmin)
template <bool D2>
__global__ void k_sl_keys(Graph g, const int *R, const int *n_p, const unsigned long long *base, const int *removed,
                          unsigned long long *key, unsigned long long *dmin)
{
    const int n = *n_p;
    const int lane = lane_id();
    const int stride = gridDim.x * blockDim.x;
    unsigned long long m = ~0ull;
    // a lane per present vertex; rows of more than 256 nets summed by the
    // whole wave
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < n; i0 += stride) {
        const int i = i0 + lane;
        const int x = i < n ? R[i] : -1;
        const int nn = x >= 0 ? Acc<D2>::nets_count(g, x) : 0;
        const bool coop = nn > 4 * WAVE;
        unsigned long long r = 0;
        if (!coop)
            for (int k = 0; k < nn; k++) r += (unsigned long long)removed[Acc<D2>::net_at(g, x, k)];
        for (uint64_t bal = __ballot(coop); bal; bal &= bal - 1) {
            const int j = __builtin_ctzll(bal);
            const int xj = __shfl(x, j), nj = __shfl(nn, j);
            unsigned long long acc = 0;
            for (int k = lane; k < nj; k += WAVE) acc += (unsigned long long)removed[Acc<D2>::net_at(g, xj, k)];
            for (int o = WAVE / 2; o > 0; o >>= 1) acc += shfl64(acc, lane ^ o);
            if (lane == j) r = acc;
        }
        if (x >= 0) {
            const unsigned long long kx = base[x] - r;
            key[x] = kx;
            m = kx < m ? kx : m;
        }
    }
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)m, d);
        m = o < m ? o : m;
    }
    if (lane == 0 && m != ~0ull) atomicMin(dmin, m);
}

// flags of the step: present vertices at or below the threshold leave
__global__ void k_sl_flags(const int *R, const int *n_p, const unsigned long long *key, const unsigned long long *dmin,
                           int shift, uint8_t *take, uint8_t *keep)
{
    const int n = *n_p;
    const unsigned long long d = *dmin;
    const unsigned long long thr = shift >= 63 ? d : d + (d >> shift);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const bool t = key[R[i]] <= thr;
        take[i] = t;
        keep[i] = !t;
    }
}

// removed(v) += 1 for every net of every vertex removed in this step (rows
// of more than 256 nets by the whole wave)
template <bool D2>
__global__ void k_sl_remove(Graph g, const int *B, const int *nb_p, int *removed)
{
    const int n = *nb_p;
    const int lane = lane_id();
    const int stride = gridDim.x * blockDim.x;
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < n; i0 += stride) {
        const int i = i0 + lane;
        const int u = i < n ? B[i] : -1;
        const int nn = u >= 0 ? Acc<D2>::nets_count(g, u) : 0;
        const bool coop = nn > 4 * WAVE;
        if (!coop)
            for (int k = 0; k < nn; k++) atomicAdd(&removed[Acc<D2>::net_at(g, u, k)], 1);
        for (uint64_t bal = __ballot(coop); bal; bal &= bal - 1) {
            const int j = __builtin_ctzll(bal);
            const int uj = __shfl(u, j), nj = __shfl(nn, j);
            for (int k = lane; k < nj; k += WAVE) atomicAdd(&removed[Acc<D2>::net_at(g, uj, k)], 1);
        }
    }
}

// rank of removal position i: steps in reverse, a step's vertices in
// ascending id; step_end[s] = vertices removed after step s
__global__ void k_sl_ranks(const int *seq, int n, const int *step_end, int steps, int *order)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int lo = 0, hi = steps - 1;   // first step with step_end > i
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (step_end[mid] > i) hi = mid;
            else lo = mid + 1;
        }
        const int beg = lo ? step_end[lo - 1] : 0;
        order[(n - step_end[lo]) + (i - beg)] = seq[i];
    }
}

}  // namespace

namespace bgpc {

// Relabels the graph to ranks, runs the rounds there and maps the colors back.
// BGPC: vertex rows are reordered (net ids unchanged) and every net's members
// become ranks, sorted again; distance-2: rows reordered, entries mapped,
// each row sorted again.  The caller's arrays are not modified.
int run_ordered(const RunArgs &a, const int32_t *order)
{
    if (a.g.n_a == 0) return a.d2 ? run<true>(a) : run<false>(a);
    const Graph g = a.g;
    hipStream_t s = a.s;
    const int n_a = g.n_a, n_b = g.n_b;
    const long nnz = a.nnz;
    const DevInfo di = dev_info();
    const int nthr = 256;
    const int ga = grid_for(n_a, nthr, di.cus * 8);
    size_t sort_bytes = 0, scan_bytes = 0;
    const int nseg = a.d2 ? n_a : n_b;
    if (rocprim::segmented_radix_sort_keys(nullptr, sort_bytes, (const int *)nullptr, (int *)nullptr, (unsigned)nnz,
                                           (unsigned)nseg, (const int *)nullptr, (const int *)nullptr, 0u, 32u,
                                           s) != hipSuccess ||
        rocprim::inclusive_scan(nullptr, scan_bytes, (const int *)nullptr, (int *)nullptr, (size_t)n_a,
                                rocprim::plus<int>(), s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_HIP;
    }
    const size_t bytes = aligned(n_a + 1, 4) * 4 + aligned(nnz + 1, 4) * 3 + aligned(4, 4) + aligned(sort_bytes, 1) +
                         aligned(scan_bytes, 1);
    Arena ar;
    int rc = ar.reserve(bytes, s);
    if (rc != BGPC_OK) return rc;
    int *inv = ar.take<int>(n_a + 1);
    int *mark = ar.take<int>(n_a + 1);
    int *noff = ar.take<int>(n_a + 1);
    int *ncol = ar.take<int>(n_a + 1);
    int *nidx = ar.take<int>(nnz + 1);
    int *tmp = ar.take<int>(nnz + 1);
    int *nidx2 = ar.take<int>(nnz + 1);
    int *err = ar.take<int>(4);
    void *sort_tmp = ar.take<char>(sort_bytes);
    void *scan_tmp = ar.take<char>(scan_bytes);
    int h_err = 0;
    k_fill_i32<<<ga, nthr, 0, s>>>(mark, 0, n_a + 1);
    k_fill_i32<<<1, 64, 0, s>>>(err, 0, 4);
    k_order_inverse<<<ga, nthr, 0, s>>>(order, n_a, mark, inv, err);
    if (hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        ar.release();
        return BGPC_E_HIP;
    }
    if (h_err) {
        ar.release();
        (void)hipStreamSynchronize(s);
        return BGPC_E_INVALID;
    }
    // rank-ordered vertex rows
    int *deg = mark;   // free again after the permutation check
    k_rank_degree<<<ga, nthr, 0, s>>>(g.a_off, order, n_a, deg);
    k_fill_i32<<<1, 64, 0, s>>>(noff, 0, 1);
    bool ok = rocprim::inclusive_scan(scan_tmp, scan_bytes, (const int *)deg, noff + 1, (size_t)n_a,
                                      rocprim::plus<int>(), s) == hipSuccess;
    const int gw = grid_for((long)n_a * WAVE, nthr, di.cus * 16);
    Graph ng;
    if (!a.d2) {
        k_rank_rows<<<gw, nthr, 0, s>>>(g.a_off, g.a_idx, order, n_a, noff, nullptr, nidx);
        k_map_ids<<<grid_for(nnz, nthr, di.cus * 16), nthr, 0, s>>>(g.b_idx, nnz, inv, tmp);
        ok = ok && (nnz == 0 ||
                    rocprim::segmented_radix_sort_keys(sort_tmp, sort_bytes, (const int *)tmp, nidx2, (unsigned)nnz,
                                                      (unsigned)n_b, g.b_off, g.b_off + 1, 0u, 32u, s) == hipSuccess);
        ng = Graph{n_a, n_b, noff, nidx, g.b_off, nidx2};
    } else {
        k_rank_rows<<<gw, nthr, 0, s>>>(g.a_off, g.a_idx, order, n_a, noff, inv, tmp);
        ok = ok && (nnz == 0 ||
                    rocprim::segmented_radix_sort_keys(sort_tmp, sort_bytes, (const int *)tmp, nidx, (unsigned)nnz,
                                                      (unsigned)n_a, (const int *)noff, (const int *)noff + 1, 0u, 32u,
                                                      s) == hipSuccess);
        ng = Graph{n_a, n_a, noff, nidx, noff, nidx};
    }
    if (!ok) {
        (void)hipGetLastError();
        ar.release();
        (void)hipStreamSynchronize(s);
        return BGPC_E_HIP;
    }
    if (a.o->flags & BGPC_RESUME) k_gather_i32<<<ga, nthr, 0, s>>>(a.st, order, n_a, ncol);
    RunArgs ra = a;
    ra.g = ng;
    ra.st = ncol;
    rc = a.d2 ? run<true>(ra) : run<false>(ra);
    if (rc == BGPC_OK || rc == BGPC_E_NOT_CONVERGED) k_gather_i32<<<ga, nthr, 0, s>>>(ncol, inv, n_a, a.st);
    if (hipGetLastError() != hipSuccess && (rc == BGPC_OK || rc == BGPC_E_NOT_CONVERGED)) rc = BGPC_E_HIP;
    ar.release();
    (void)hipStreamSynchronize(s);
    return rc;
}

// Vertices by decreasing key, ties by increasing id (the radix sort is stable
// and the ids enter in increasing order).
int order_largest_first(const Graph &g, bool d2, hipStream_t s, int32_t *order_out)
{
    const int n = g.n_a;
    if (n == 0) return BGPC_OK;
    const DevInfo di = dev_info();
    size_t sort_bytes = 0;
    if (rocprim::radix_sort_pairs_desc(nullptr, sort_bytes, (const unsigned long long *)nullptr,
                                       (unsigned long long *)nullptr, (const int *)nullptr, (int *)nullptr,
                                       (size_t)n, 0u, 64u, s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_HIP;
    }
    Arena ar;
    int rc = ar.reserve(aligned(n, 8) * 2 + aligned(n, 4) + aligned(sort_bytes, 1), s);
    if (rc != BGPC_OK) return rc;
    unsigned long long *key = ar.take<unsigned long long>(n);
    unsigned long long *key_sorted = ar.take<unsigned long long>(n);
    int *ids = ar.take<int>(n);
    void *tmp = ar.take<char>(sort_bytes);
    const int blocks = grid_for((long)n * WAVE, 256, di.cus * 16);
    if (d2) k_order_key<true><<<blocks, 256, 0, s>>>(g, key, ids);
    else k_order_key<false><<<blocks, 256, 0, s>>>(g, key, ids);
    bool ok = hipGetLastError() == hipSuccess &&
              rocprim::radix_sort_pairs_desc(tmp, sort_bytes, (const unsigned long long *)key, key_sorted,
                                             (const int *)ids, order_out, (size_t)n, 0u, 64u, s) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    ar.release();
    if (hipStreamSynchronize(s) != hipSuccess) ok = false;
    return ok ? BGPC_OK : BGPC_E_HIP;
}

// Smallest-last order by steps (see k_sl_keys).  steps_out: optional, host.
int order_smallest_last(const Graph &g, bool d2, int shift, hipStream_t s, int32_t *order_out, int32_t *steps_out)
{
    const int n = g.n_a;
    if (steps_out) *steps_out = 0;
    if (n == 0) return BGPC_OK;
    const DevInfo di = dev_info();
    size_t sel_bytes = 0;
    if (rocprim::select(nullptr, sel_bytes, (const int *)nullptr, (const uint8_t *)nullptr, (int *)nullptr,
                        (int *)nullptr, (size_t)n, s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_HIP;
    }
    Arena ar;
    const size_t bytes = aligned(n, 8) * 2 + aligned(n, 4) * 4 + aligned(g.n_b + 1, 4) + aligned(n, 1) * 2 +
                         aligned(16, 8) + aligned(sel_bytes, 1);
    int rc = ar.reserve(bytes, s);
    if (rc != BGPC_OK) return rc;
    unsigned long long *base = ar.take<unsigned long long>(n);
    unsigned long long *key = ar.take<unsigned long long>(n);
    int *R[2] = {ar.take<int>(n), ar.take<int>(n)};
    int *seq = ar.take<int>(n);
    int *ids = ar.take<int>(n);
    int *removed = ar.take<int>(g.n_b + 1);
    uint8_t *take = ar.take<uint8_t>(n);
    uint8_t *keep = ar.take<uint8_t>(n);
    unsigned long long *ctl = ar.take<unsigned long long>(16);   // [0] min key; ints from [1]: counts
    int *cnt = (int *)(ctl + 1);                                 // cnt[0] present, cnt[1] taken, cnt[2] kept
    void *tmp = ar.take<char>(sel_bytes);
    const int nthr = 256;
    const int blocks_w = grid_for((long)n * WAVE, 256, di.cus * 16);
    const int ga = grid_for(n, nthr, di.cus * 8);
    bool ok = true;
    if (d2) k_order_key<true><<<blocks_w, 256, 0, s>>>(g, base, ids);
    else k_order_key<false><<<blocks_w, 256, 0, s>>>(g, base, ids);
    k_iota<<<ga, nthr, 0, s>>>(R[0], n);
    k_fill_i32<<<grid_for(g.n_b + 1, nthr, di.cus * 8), nthr, 0, s>>>(removed, 0, g.n_b + 1);
    ok = hipMemcpyAsync(cnt, &n, sizeof(int), hipMemcpyHostToDevice, s) == hipSuccess;
    std::vector<int> step_end;
    int present = n, removed_total = 0, cur = 0;
    while (ok && present > 0) {
        k_fill_u64<<<1, 64, 0, s>>>((uint64_t *)ctl, ~0ull, 1);
        if (d2) k_sl_keys<true><<<ga, nthr, 0, s>>>(g, R[cur], cnt, base, removed, key, ctl);
        else k_sl_keys<false><<<ga, nthr, 0, s>>>(g, R[cur], cnt, base, removed, key, ctl);
        k_sl_flags<<<ga, nthr, 0, s>>>(R[cur], cnt, key, ctl, shift, take, keep);
        ok = hipGetLastError() == hipSuccess &&
             rocprim::select(tmp, sel_bytes, (const int *)R[cur], (const uint8_t *)take, seq + removed_total,
                             cnt + 1, (size_t)present, s) == hipSuccess &&
             rocprim::select(tmp, sel_bytes, (const int *)R[cur], (const uint8_t *)keep, R[cur ^ 1], cnt + 2,
                             (size_t)present, s) == hipSuccess;
        if (!ok) break;
        if (d2) k_sl_remove<true><<<ga, nthr, 0, s>>>(g, seq + removed_total, cnt + 1, removed);
        else k_sl_remove<false><<<ga, nthr, 0, s>>>(g, seq + removed_total, cnt + 1, removed);
        int h[3] = {0, 0, 0};
        ok = hipMemcpyAsync(cnt, cnt + 2, sizeof(int), hipMemcpyDeviceToDevice, s) == hipSuccess &&
             hipMemcpyAsync(h, cnt, 3 * sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
             hipStreamSynchronize(s) == hipSuccess;
        if (!ok || h[1] <= 0) {   // a step always removes the vertices at the minimum
            ok = false;
            break;
        }
        removed_total += h[1];
        present = h[2];
        step_end.push_back(removed_total);
        cur ^= 1;
    }
    int *d_steps = nullptr;
    if (ok) {
        // the step boundaries go where the keys were (no longer needed)
        d_steps = (int *)key;
        ok = (size_t)step_end.size() <= (size_t)n * 2 &&
             hipMemcpyAsync(d_steps, step_end.data(), sizeof(int) * step_end.size(), hipMemcpyHostToDevice, s) ==
                 hipSuccess;
    }
    if (ok) {
        k_sl_ranks<<<ga, nthr, 0, s>>>(seq, n, d_steps, (int)step_end.size(), order_out);
        ok = hipGetLastError() == hipSuccess;
    }
    if (!ok) (void)hipGetLastError();
    ar.release();
    if (hipStreamSynchronize(s) != hipSuccess) ok = false;
    if (ok && steps_out) *steps_out = (int32_t)step_end.size();
    return ok ? BGPC_OK : BGPC_E_HIP;
}

}  // namespace bgpc

namespace bgpc {

void release_thread_state()
{
    if (t_prog) {
        if (t_prog->h) (void)hipHostFree((void *)t_prog->h);
        delete t_prog;
        t_prog = nullptr;
    }
    if (t_evpool) {
        for (hipEvent_t e : t_evpool->ev) (void)hipEventDestroy(e);
        delete t_evpool;
        t_evpool = nullptr;
    }
}

}  // namespace bgpc

extern "C" {

// ---- allocation-free entry point: the workspace is one static device array
// per GPU (held until the process ends); host code reaches it only through
// the address hipGetSymbolAddress returns on that device.
namespace {
__device__ __align__(256) unsigned char scratch[BGPC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
char *g_scratch_ptr[64] = {};

// address of this device's scratch array (looked up once per device, with
// the device current); null when the lookup fails
char *scratch_of_current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = (char *)ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" BGPC_API int bgpc_color_noalloc(const bgpc_csr *csr_A, const bgpc_csr *csr_B, const bgpc_opts *opts,
                                           int32_t *colors_out)
{
    bgpc_opts o;
    if (opts) o = *opts;
    else bgpc_opts_default(&o);
    if (!csr_ok(csr_A) || !csr_ok(csr_B) || !colors_out || !opts_ok(o)) return BGPC_E_INVALID;
    if (csr_A->n_rows != csr_B->n_cols || csr_A->n_cols != csr_B->n_rows || csr_A->nnz != csr_B->nnz)
        return BGPC_E_INVALID;
    // sizes past the documented limits, and the options that need memory of
    // their own (events, pinned buffers), are refused before any device call
    if (csr_A->n_rows > BGPC_NOALLOC_MAX_VERTICES || csr_B->n_rows > BGPC_NOALLOC_MAX_NETS ||
        csr_A->nnz > BGPC_NOALLOC_MAX_NNZ || (o.flags & BGPC_INCREMENTAL) || o.prof ||
        (o.log && (o.log->hash_t || o.log->hash_c || o.log->round_ms)))
        return BGPC_E_UNSUPPORTED;
    char *base = scratch_of_current_device();
    if (!base) return BGPC_E_HIP;
    hipStream_t s = (hipStream_t)o.stream;
    if (o.flags & BGPC_STRICT) {
        int v = validate_bipartite(csr_A, csr_B, s, (int *)base);
        if (v != BGPC_OK) return v;
    }
    RunArgs a;
    a.g = Graph{csr_A->n_rows, csr_B->n_rows, csr_A->offsets, csr_A->indices, csr_B->offsets, csr_B->indices};
    a.nnz = csr_B->nnz;
    a.d2 = false;
    a.o = &o;
    a.st = colors_out;
    a.s = s;
    a.ext = base;
    a.ext_cap = BGPC_NOALLOC_SCRATCH_BYTES;
    return run<false>(a);
}

// ---- autotuner (see bgpc.h)
extern "C" BGPC_API int bgpc_autotune(const bgpc_csr *csr_A, const bgpc_csr *csr_B, const bgpc_opts *opts,
                                      int32_t trials, bgpc_tuning *best, double *ms_default, double *ms_best)
{
    bgpc_opts o;
    if (opts) o = *opts;
    else bgpc_opts_default(&o);
    const bool d2 = csr_B == nullptr;
    if (!csr_ok(csr_A) || !opts_ok(o) || !best || trials < 1 || (o.flags & BGPC_RESUME)) return BGPC_E_INVALID;
    if (d2 ? csr_A->n_rows != csr_A->n_cols
           : (!csr_ok(csr_B) || csr_A->n_rows != csr_B->n_cols || csr_A->n_cols != csr_B->n_rows ||
              csr_A->nnz != csr_B->nnz))
        return BGPC_E_INVALID;
    hipStream_t s = (hipStream_t)o.stream;
    o.log = nullptr;
    o.prof = nullptr;
    o.flags &= ~(uint32_t)BGPC_STRICT;
    int32_t rounds = 0;
    o.rounds_out = &rounds;
    const int n = csr_A->n_rows;
    RunArgs a;
    a.g = d2 ? Graph{n, n, csr_A->offsets, csr_A->indices, csr_A->offsets, csr_A->indices}
             : Graph{csr_A->n_rows, csr_B->n_rows, csr_A->offsets, csr_A->indices, csr_B->offsets, csr_B->indices};
    a.nnz = csr_A->nnz;
    a.d2 = d2;
    a.o = &o;
    a.s = s;
    int32_t *colors = nullptr;
    if (hipMallocAsync((void **)&colors, sizeof(int32_t) * ((size_t)n + 1), s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_OOM;
    }
    a.st = colors;
    std::vector<int32_t> ref(n), got(n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = BGPC_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = BGPC_E_HIP;
    // one configuration: the fastest of `trials` calls, its colors and rounds
    auto measure = [&](const bgpc_tuning &t, std::vector<int32_t> &out, int32_t *r_out, double *ms) -> int {
        o.tuning = &t;
        double bestms = 1e30;
        for (int k = 0; k < trials; k++) {
            if (hipEventRecord(e0, s) != hipSuccess) return BGPC_E_HIP;
            int st = d2 ? run<true>(a) : run<false>(a);
            if (st != BGPC_OK && st != BGPC_E_NOT_CONVERGED) return st;
            float t_ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess)
                return BGPC_E_HIP;
            bestms = std::min(bestms, (double)t_ms);
        }
        *r_out = rounds;
        *ms = bestms;
        if (n && (hipMemcpyAsync(out.data(), colors, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
                  hipStreamSynchronize(s) != hipSuccess))
            return BGPC_E_HIP;
        return BGPC_OK;
    };
    bgpc_tuning cur = tune_default();
    double cur_ms = 0.0, base_ms = 0.0;
    int32_t ref_rounds = 0;
    if (rc == BGPC_OK) rc = measure(cur, ref, &ref_rounds, &cur_ms);
    base_ms = cur_ms;
    // candidates per field, tried one field at a time
    struct Field {
        int32_t bgpc_tuning::*f;
        std::vector<int32_t> values;
    };
    const std::vector<Field> fields = {{&bgpc_tuning::front, {0, 1}},
                                       {&bgpc_tuning::standing, {0, 1}},
                                       {&bgpc_tuning::planes, {0, 1}},
                                       {&bgpc_tuning::color_grid, {8, 16, 32, 64}},
                                       {&bgpc_tuning::removal_grid, {2, 4, 16, 32}},
                                       {&bgpc_tuning::apply_grid, {2, 8, 16}}};
    for (const Field &fd : fields) {
        for (int32_t v : fd.values) {
            if (rc != BGPC_OK) break;
            bgpc_tuning cand = cur;
            cand.*(fd.f) = v;
            double ms = 0.0;
            int32_t r2 = 0;
            rc = measure(cand, got, &r2, &ms);
            if (rc != BGPC_OK) break;
            if (r2 != ref_rounds || got != ref) {   // a choice that changes a result is a library fault
                rc = BGPC_E_INTERNAL;
                break;
            }
            if (ms < cur_ms) {
                cur = cand;
                cur_ms = ms;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFreeAsync(colors, s);
    (void)hipStreamSynchronize(s);
    if (rc != BGPC_OK) return rc;
    *best = cur;
    if (ms_default) *ms_default = base_ms;
    if (ms_best) *ms_best = cur_ms;
    {
        bgpc_opts ko = o;
        ko.tuning = nullptr;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[tune_key(a.g, a.nnz, d2, ko)] = cur;
    }
    return BGPC_OK;
}

BGPC_API void bgpc_opts_default(bgpc_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->policy = BGPC_FIRST_FIT;
    o->chunk = 64;
    o->net_conflict_mask = ~0ull;
    o->net_alg = BGPC_NET_ALG8;
}

BGPC_API int bgpc_color(const bgpc_csr *csr_A, const bgpc_csr *csr_B, const int32_t *order, const bgpc_opts *opts,
                        int32_t *colors_out)
{
    bgpc_opts o;
    if (opts) o = *opts;
    else bgpc_opts_default(&o);
    if (!csr_ok(csr_A) || !csr_ok(csr_B) || !colors_out || !opts_ok(o)) return BGPC_E_INVALID;
    if (csr_A->n_rows != csr_B->n_cols || csr_A->n_cols != csr_B->n_rows || csr_A->nnz != csr_B->nnz)
        return BGPC_E_INVALID;
    hipStream_t s = (hipStream_t)o.stream;
    if (o.flags & BGPC_STRICT) {
        int v = validate_bipartite(csr_A, csr_B, s);
        if (v != BGPC_OK) return v;
    }
    RunArgs a;
    a.g = Graph{csr_A->n_rows, csr_B->n_rows, csr_A->offsets, csr_A->indices, csr_B->offsets, csr_B->indices};
    a.nnz = csr_B->nnz;
    a.d2 = false;
    a.o = &o;
    a.st = colors_out;
    a.s = s;
    return order ? run_ordered(a, order) : run<false>(a);
}

BGPC_API int d2gc_color(const bgpc_csr *adj, const int32_t *order, const bgpc_opts *opts, int32_t *colors_out)
{
    bgpc_opts o;
    if (opts) o = *opts;
    else bgpc_opts_default(&o);
    if (!csr_ok(adj) || !colors_out || !opts_ok(o) || adj->n_rows != adj->n_cols) return BGPC_E_INVALID;
    hipStream_t s = (hipStream_t)o.stream;
    if (o.flags & BGPC_STRICT) {
        int v = validate_symmetric(adj, s);
        if (v != BGPC_OK) return v;
    }
    RunArgs a;
    a.g = Graph{adj->n_rows, adj->n_rows, adj->offsets, adj->indices, adj->offsets, adj->indices};
    a.nnz = adj->nnz;
    a.d2 = true;
    a.o = &o;
    a.st = colors_out;
    a.s = s;
    return order ? run_ordered(a, order) : run<true>(a);
}

BGPC_API int bgpc_order_largest_first(const bgpc_csr *csr_A, const bgpc_csr *csr_B, void *stream,
                                      int32_t *order_out)
{
    if (!csr_ok(csr_A) || !csr_ok(csr_B) || (csr_A->n_rows > 0 && !order_out)) return BGPC_E_INVALID;
    if (csr_A->n_rows != csr_B->n_cols || csr_A->n_cols != csr_B->n_rows || csr_A->nnz != csr_B->nnz)
        return BGPC_E_INVALID;
    const Graph g{csr_A->n_rows, csr_B->n_rows, csr_A->offsets, csr_A->indices, csr_B->offsets, csr_B->indices};
    return order_largest_first(g, false, (hipStream_t)stream, order_out);
}

BGPC_API int d2gc_order_largest_first(const bgpc_csr *adj, void *stream, int32_t *order_out)
{
    if (!csr_ok(adj) || adj->n_rows != adj->n_cols || (adj->n_rows > 0 && !order_out)) return BGPC_E_INVALID;
    const Graph g{adj->n_rows, adj->n_rows, adj->offsets, adj->indices, adj->offsets, adj->indices};
    return order_largest_first(g, true, (hipStream_t)stream, order_out);
}

BGPC_API int bgpc_order_smallest_last(const bgpc_csr *csr_A, const bgpc_csr *csr_B, int32_t slack_shift, void *stream,
                                      int32_t *order_out, int32_t *steps_out)
{
    if (!csr_ok(csr_A) || !csr_ok(csr_B) || csr_A->n_rows != csr_B->n_cols || csr_A->n_cols != csr_B->n_rows ||
        csr_A->nnz != csr_B->nnz || (csr_A->n_rows > 0 && !order_out) || slack_shift < 0)
        return BGPC_E_INVALID;
    Graph g{csr_A->n_rows, csr_B->n_rows, csr_A->offsets, csr_A->indices, csr_B->offsets, csr_B->indices};
    return order_smallest_last(g, false, slack_shift, (hipStream_t)stream, order_out, steps_out);
}

BGPC_API int d2gc_order_smallest_last(const bgpc_csr *adj, int32_t slack_shift, void *stream, int32_t *order_out,
                                      int32_t *steps_out)
{
    if (!csr_ok(adj) || adj->n_rows != adj->n_cols || (adj->n_rows > 0 && !order_out) || slack_shift < 0)
        return BGPC_E_INVALID;
    Graph g{adj->n_rows, adj->n_rows, adj->offsets, adj->indices, adj->offsets, adj->indices};
    return order_smallest_last(g, true, slack_shift, (hipStream_t)stream, order_out, steps_out);
}

BGPC_API int color_stats(const int32_t *colors, int64_t n, void *stream, bgpc_stats *out)
{
    if (!out || n < 0 || (n > 0 && !colors)) return BGPC_E_INVALID;
    std::memset(out, 0, sizeof(*out));
    out->max_color = -1;
    if (n == 0) return BGPC_OK;
    hipStream_t s = (hipStream_t)stream;
    const DevInfo di = dev_info();
    int *d_max = nullptr;
    HIP_TRY(hipMallocAsync((void **)&d_max, 256, s));
    k_fill_i32<<<1, 64, 0, s>>>(d_max, -1, 1);
    k_colors_max<<<grid_for(n, 256, di.cus * 8), 256, 0, s>>>(colors, n, d_max);
    int h_max = -1;
    hipMemcpyAsync(&h_max, d_max, sizeof(int), hipMemcpyDeviceToHost, s);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hipFreeAsync(d_max, s);
        return BGPC_E_HIP;
    }
    if (h_max < 0) {
        hipFreeAsync(d_max, s);
        hipStreamSynchronize(s);
        return BGPC_OK;
    }
    const int ncol = h_max + 1;
    int *d_count = nullptr;
    long long *d_i = nullptr;
    double *d_d = nullptr;
    char *blk = nullptr;
    size_t bytes = aligned(ncol, 4) + aligned(5, 8) + aligned(2, 8);
    if (hipMallocAsync((void **)&blk, bytes, s) != hipSuccess) {
        hipFreeAsync(d_max, s);
        return BGPC_E_OOM;
    }
    d_count = (int *)blk;
    d_i = (long long *)(blk + aligned(ncol, 4));
    d_d = (double *)(blk + aligned(ncol, 4) + aligned(5, 8));
    k_fill_i32<<<grid_for(ncol, 256, di.cus * 8), 256, 0, s>>>(d_count, 0, ncol);
    // with LDS histograms, few enough blocks that each one's flush (ncol
    // atomics at most) stays below the atomics it saves
    const int g_hist = ncol <= HIST_LDS ? (int)std::max<long>(1, std::min<long>(di.cus * 8, n / (8L * ncol)))
                                        : grid_for(n, 256, di.cus * 8);
    k_hist<<<g_hist, 256, 0, s>>>(colors, n, d_count, ncol);
    k_hist_reduce<<<1, 1024, 0, s>>>(d_count, ncol, d_i, d_d);
    long long hi[5];
    double hd[2];
    hipMemcpyAsync(hi, d_i, sizeof(hi), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(hd, d_d, sizeof(hd), hipMemcpyDeviceToHost, s);
    e = hipStreamSynchronize(s);
    hipFreeAsync(blk, s);
    hipFreeAsync(d_max, s);
    hipStreamSynchronize(s);
    if (e != hipSuccess) return BGPC_E_HIP;
    out->n_distinct = hi[0];
    out->max_color = hi[1];
    out->card_min = hi[2];
    out->card_max = hi[3];
    out->n_empty_below_max = hi[4];
    out->card_mean = hd[0];
    out->card_std = hd[1];
    return BGPC_OK;
}

BGPC_API const char *bgpc_status_string(int status)
{
    switch (status) {
    case BGPC_OK: return "ok";
    case BGPC_E_INVALID: return "invalid argument";
    case BGPC_E_UNSORTED: return "member list not strictly ascending";
    case BGPC_E_NOT_TRANSPOSE: return "csr_A is not the transpose of csr_B";
    case BGPC_E_NOT_SYMMETRIC: return "adjacency not symmetric or has a self loop";
    case BGPC_E_OOM: return "device workspace allocation failed";
    case BGPC_E_NOT_CONVERGED: return "worklist not empty after max_rounds rounds";
    case BGPC_E_HIP: return "HIP runtime error";
    case BGPC_E_UNSUPPORTED: return "size beyond the library's limits";
    case BGPC_E_INTERNAL: return "device-side invariant violated";
    default: return "unknown status";
    }
}

}  // extern "C"
