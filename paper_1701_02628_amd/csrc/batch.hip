// Batched coloring (bgpc_color_batch): many graphs, one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "batch.h"
#include "bgpc.h"

using namespace bgpc;

namespace bgpc {
// frees the calling thread's round-driver state (bgpc.hip)
void release_thread_state();
}  // namespace bgpc

namespace {

int device_cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 256;
    return v;
}

// Streams per device for the graphs that take the whole-device path while
// the persistent launch runs (default priority, created once): each is driven
// by a host thread of its own, since a bgpc_color call waits for its rounds.
constexpr int SIDE_STREAMS = 3;
hipStream_t side_stream(int i)
{
    static std::mutex mu;
    static hipStream_t streams[64][SIDE_STREAMS] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || i < 0 || i >= SIDE_STREAMS) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!streams[dev][i] && hipStreamCreateWithFlags(&streams[dev][i], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        streams[dev][i] = nullptr;
    }
    return streams[dev][i];
}

// Serving: graphs of at least this many memberships take an idle
// whole-device thread when one is free (see bgpc_session::loop).
constexpr long long LIGHT_LOAD_NNZ = 50000;

// Graphs that one workgroup would color far slower than the whole device:
// many nets to rescan every round and colors past the net masks, or simply
// many memberships.  They take bgpc_color (same rounds, same colors).
bool whole_device(const BatchItem &b)
{
    return b.mode != MODE_DENSE && ((b.mode == MODE_FORB && b.nnz > 50000) || b.nnz > 1000000);
}

bool item_ok(const bgpc_batch_item &it)
{
    const bgpc_csr &A = it.csr_A, &B = it.csr_B;
    const bool a_ok = A.n_rows >= 0 && A.n_cols >= 0 && A.n_rows < (1 << 30) && A.n_cols < (1 << 30) && A.nnz >= 0 &&
                      A.nnz < (1ll << 31) && A.offsets && (A.nnz == 0 || A.indices) && (A.n_rows == 0 || it.colors_out);
    if (it.d2gc) return a_ok && A.n_rows == A.n_cols;
    return a_ok && A.n_rows == B.n_cols && A.n_cols == B.n_rows && A.nnz == B.nnz && B.offsets &&
           (B.nnz == 0 || B.indices);
}

// the persistent launch runs the default schedule only: vertex-based
// first-fit rounds from scratch, net-side removal
bool default_schedule(const bgpc_opts &o)
{
    return o.policy == BGPC_FIRST_FIT && o.net_color_mask == 0 && !(o.flags & ~(uint32_t)BGPC_STRICT) &&
           o.start_round == 0 && o.net_alg == BGPC_NET_ALG8 && o.net_conflict_mask == ~0ull;
}

int route_of(int mode)
{
    return mode == MODE_DENSE ? BGPC_ROUTE_DENSE : mode == MODE_FORB ? BGPC_ROUTE_BITMAPS : BGPC_ROUTE_NET_MASKS;
}

}  // namespace

namespace bgpc {

// One graph on one workgroup (bgpc_color's route for small dense graphs):
// the batch kernel with a single item and its own scratch.  Fills the round
// log (|W|, losers, largest color per round) when log is non-null.
int color_one_workgroup(const Graph &g, int *colors, int max_rounds, hipStream_t s, int log_cap,
                        std::vector<int> *log, int *rounds_out)
{
    const long long scr = batch_scratch_bytes(MODE_DENSE, g.n_a, g.n_b, g.n_a + 1);
    const size_t o_tbl = 0, o_ord = 256, o_next = 512, o_log = 768;
    const size_t o_scr = o_log + (((size_t)3 * log_cap * 4 + 255) & ~(size_t)255);
    char *base = nullptr;
    if (hipMallocAsync((void **)&base, o_scr + (size_t)scr, s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_OOM;
    }
    BatchItem h = {};
    h.n_a = g.n_a;
    h.n_b = g.n_b;
    h.a_off = g.a_off;
    h.a_idx = g.a_idx;
    h.b_off = g.b_off;
    h.b_idx = g.b_idx;
    h.colors = colors;
    h.scratch = base + o_scr;
    h.log = log_cap ? (int *)(base + o_log) : nullptr;
    h.log_cap = log_cap;
    h.max_rounds = max_rounds;
    h.mode = MODE_DENSE;
    h.cap = g.n_a + 1;
    h.status = -1;
    int zero[2] = {0, 0};
    int rc = BGPC_OK;
    if (hipMemcpyAsync(base + o_tbl, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(base + o_ord, zero, 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(base + o_next, zero, 4, hipMemcpyHostToDevice, s) != hipSuccess) {
        rc = BGPC_E_HIP;
    } else {
        k_batch<<<1, BATCH_BLOCK, 0, s>>>((BatchItem *)(base + o_tbl), (const int *)(base + o_ord), 1,
                                          (int *)(base + o_next));
        if (hipGetLastError() != hipSuccess) rc = BGPC_E_HIP;
        else if (hipMemcpyAsync(&h, base + o_tbl, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
                 hipStreamSynchronize(s) != hipSuccess)
            rc = BGPC_E_HIP;
    }
    if (rc == BGPC_OK && log && log_cap) {
        int k = std::min(h.rounds, log_cap);
        log->assign(3 * (size_t)std::max(k, 1), 0);
        if (k > 0 && (hipMemcpyAsync(log->data(), base + o_log, 12 * (size_t)k, hipMemcpyDeviceToHost, s) !=
                          hipSuccess ||
                      hipStreamSynchronize(s) != hipSuccess))
            rc = BGPC_E_HIP;
        log->resize(3 * (size_t)k);
    }
    (void)hipFreeAsync(base, s);
    (void)hipStreamSynchronize(s);
    if (rc != BGPC_OK) return rc;
    *rounds_out = h.rounds;
    return h.status == 0 ? BGPC_OK : BGPC_E_NOT_CONVERGED;
}

}  // namespace bgpc

extern "C" BGPC_API int bgpc_color_batch(bgpc_batch_item *items, int32_t n_items, const bgpc_opts *opts)
{
    bgpc_opts o;
    if (opts) o = *opts;
    else bgpc_opts_default(&o);
    if (n_items < 0 || (n_items > 0 && !items)) return BGPC_E_INVALID;
    if (o.policy < 0 || o.policy > BGPC_B1_GLOBAL || o.chunk < 1 || o.max_rounds < 0 || o.start_round < 0 ||
        o.net_alg < BGPC_NET_ALG8 || o.net_alg > BGPC_NET_ALG6_REVERSE)
        return BGPC_E_INVALID;
    for (int i = 0; i < n_items; i++)
        if (!item_ok(items[i])) return BGPC_E_INVALID;
    if (n_items == 0) return BGPC_OK;
    hipStream_t s = (hipStream_t)o.stream;
    // items the persistent launch cannot run (another schedule, a caller
    // order, distance-2) take the whole-device route as they are
    const bool dflt = default_schedule(o);
    std::vector<char> forced(n_items);
    for (int i = 0; i < n_items; i++) forced[i] = !dflt || items[i].order || items[i].d2gc;

    std::vector<BatchItem> h(n_items);
    for (int i = 0; i < n_items; i++) {
        const bgpc_batch_item &it = items[i];
        BatchItem &b = h[i];
        b = BatchItem{};
        b.colors = it.colors_out;
        b.status = -1;
        if (forced[i]) {
            // measured by nobody: an empty graph for the shape pass
            b.a_off = b.b_off = it.csr_A.offsets;
            continue;
        }
        b.n_a = it.csr_A.n_rows;
        b.n_b = it.csr_B.n_rows;
        b.a_off = it.csr_A.offsets;
        b.a_idx = it.csr_A.indices;
        b.b_off = it.csr_B.offsets;
        b.b_idx = it.csr_B.indices;
        b.max_rounds = o.max_rounds > 0 ? o.max_rounds : b.n_a + 65;
        b.nnz = (int)it.csr_A.nnz;
    }
    // largest graphs first
    std::vector<int> order(n_items);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return items[x].csr_A.nnz + items[x].csr_A.n_rows > items[y].csr_A.nnz + items[y].csr_A.n_rows;
    });
    const int cus = device_cus();
    const size_t tbl = al256((long long)n_items * sizeof(BatchItem));
    const size_t ord = al256(4ll * n_items);
    char *meta = nullptr;
    if (hipMallocAsync((void **)&meta, tbl + ord + 256 * (size_t)(n_items + 1), s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_OOM;
    }
    BatchItem *d_items = (BatchItem *)meta;
    int *d_order = (int *)(meta + tbl);
    char *d_next = meta + tbl + ord;   // one queue counter per launch, 256 bytes apart
    int rc = BGPC_OK;
    // shape pass: the mode and scratch of each graph depend on its net sizes
    if (hipMemcpyAsync(d_items, h.data(), sizeof(BatchItem) * n_items, hipMemcpyHostToDevice, s) != hipSuccess)
        rc = BGPC_E_HIP;
    if (rc == BGPC_OK) {
        k_batch_shape<<<std::max(1, std::min(n_items, cus * 4)), BATCH_BLOCK, 0, s>>>(d_items, n_items);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h.data(), d_items, sizeof(BatchItem) * n_items, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = BGPC_E_HIP;
    }
    for (int i = 0; i < n_items && rc == BGPC_OK; i++)
        if (!forced[i] && h[i].walk < 0) {
            items[i].status = BGPC_E_INVALID;
            rc = BGPC_E_INVALID;
        }
    std::vector<long long> need(n_items);
    for (int i = 0; i < n_items && rc == BGPC_OK; i++) {
        h[i].mode = batch_mode(h[i].n_a, h[i].walk, h[i].walk_max, &h[i].cap);
        need[i] = batch_scratch_bytes(h[i].mode, h[i].n_a, h[i].n_b, h[i].cap);
    }
    // the persistent launch takes the graphs in `order` minus the whole-device ones
    std::vector<int> big, queue;
    for (int k = 0; k < n_items; k++)
        (forced[order[k]] || whole_device(h[order[k]]) ? big : queue).push_back(order[k]);
    for (int i = 0; i < n_items; i++) items[i].route = route_of(h[i].mode);
    for (int i : big) items[i].route = BGPC_ROUTE_WHOLE_DEVICE;
    const int nq = (int)queue.size();
    // launches over consecutive runs of the (largest-first) queue whose
    // scratch fits the budget; each launch reuses the one scratch buffer
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 8ull << 30;
    long long budget = std::max<long long>(1ll << 28, (long long)(free_b / 2));
    std::vector<std::pair<int, int>> runs;
    long long biggest = 0;
    for (int k = 0; k < nq && rc == BGPC_OK;) {
        long long sum = 0;
        int e = k;
        while (e < nq && (e == k || sum + need[queue[e]] <= budget)) sum += need[queue[e++]];
        runs.push_back({k, e});
        biggest = std::max(biggest, sum);
        k = e;
    }
    char *scr = nullptr;
    if (rc == BGPC_OK && !runs.empty() &&
        hipMallocAsync((void **)&scr, (size_t)std::max(biggest, 256ll), s) != hipSuccess) {
        (void)hipGetLastError();
        rc = BGPC_E_OOM;
    }
    for (size_t r = 0; r < runs.size() && rc == BGPC_OK; r++) {
        long long off = 0;
        for (int k = runs[r].first; k < runs[r].second; k++) {
            h[queue[k]].scratch = scr + off;
            off += need[queue[k]];
        }
    }
    if (rc == BGPC_OK &&
        (hipMemcpyAsync(d_items, h.data(), sizeof(BatchItem) * n_items, hipMemcpyHostToDevice, s) != hipSuccess ||
         (nq && hipMemcpyAsync(d_order, queue.data(), 4 * (size_t)nq, hipMemcpyHostToDevice, s) != hipSuccess)))
        rc = BGPC_E_HIP;
    std::vector<int> zeros(64 * (runs.size() + 1), 0);
    if (rc == BGPC_OK && !runs.empty() &&
        hipMemcpyAsync(d_next, zeros.data(), 256 * runs.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        rc = BGPC_E_HIP;
    // whole-device graphs on the side streams, after the caller's prior work on s
    const int nside = (int)std::min<size_t>(SIDE_STREAMS, big.size());
    hipStream_t side[SIDE_STREAMS] = {};
    hipEvent_t ev_in = nullptr, ev_out[SIDE_STREAMS] = {};
    if (rc == BGPC_OK && nside > 0) {
        if (hipEventCreateWithFlags(&ev_in, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev_in, s) != hipSuccess)
            rc = BGPC_E_HIP;
        for (int t = 0; t < nside && rc == BGPC_OK; t++) {
            side[t] = side_stream(t);
            if (!side[t] || hipStreamWaitEvent(side[t], ev_in, 0) != hipSuccess ||
                hipEventCreateWithFlags(&ev_out[t], hipEventDisableTiming) != hipSuccess)
                rc = BGPC_E_HIP;
        }
    }
    for (size_t r = 0; r < runs.size() && rc == BGPC_OK; r++) {
        const int n = runs[r].second - runs[r].first;
        const int grid = std::max(1, std::min(n, cus * 2));
        k_batch<<<grid, BATCH_BLOCK, 0, s>>>(d_items, d_order + runs[r].first, n, (int *)(d_next + 256 * r));
        if (hipGetLastError() != hipSuccess) rc = BGPC_E_HIP;
    }
    std::vector<std::pair<int, int>> big_res(big.size(), {BGPC_OK, 0});
    if (rc == BGPC_OK && nside > 0) {
        // largest first (the order of `big`), taken by the threads as they free up
        std::atomic<size_t> next_big(0);
        std::atomic<int> side_rc(BGPC_OK);
        int dev = 0;
        (void)hipGetDevice(&dev);
        auto worker = [&](int t) {
            (void)hipSetDevice(dev);
            for (size_t j = next_big++; j < big.size(); j = next_big++) {
                const bgpc_batch_item &it = items[big[j]];
                bgpc_opts po = o;
                po.stream = side[t];
                po.log = nullptr;
                po.prof = nullptr;
                int32_t rr = 0;
                po.rounds_out = &rr;
                int st = it.d2gc ? d2gc_color(&it.csr_A, it.order, &po, it.colors_out)
                                 : bgpc_color(&it.csr_A, &it.csr_B, it.order, &po, it.colors_out);
                if (st != BGPC_OK && st != BGPC_E_NOT_CONVERGED) side_rc = st;
                big_res[j] = {st, rr};
            }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nside; t++)
            pool.emplace_back([&worker, t] {
                worker(t);
                release_thread_state();
            });
        worker(0);
        for (auto &th : pool) th.join();
        if (side_rc != BGPC_OK) rc = side_rc;
        for (int t = 0; t < nside; t++)
            if (hipEventRecord(ev_out[t], side[t]) != hipSuccess || hipStreamWaitEvent(s, ev_out[t], 0) != hipSuccess)
                rc = BGPC_E_HIP;
    }
    if (rc == BGPC_OK &&
        (hipMemcpyAsync(h.data(), d_items, sizeof(BatchItem) * n_items, hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        rc = BGPC_E_HIP;
    for (size_t j = 0; j < big.size(); j++) {
        h[big[j]].status = big_res[j].first;
        h[big[j]].rounds = big_res[j].second;
    }
    for (int t = 0; t < nside; t++) {
        if (side[t]) (void)hipStreamSynchronize(side[t]);
        if (ev_out[t]) (void)hipEventDestroy(ev_out[t]);
    }
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (scr) (void)hipFreeAsync(scr, s);
    (void)hipFreeAsync(meta, s);
    (void)hipStreamSynchronize(s);
    if (rc != BGPC_OK) return rc;
    for (int i = 0; i < n_items; i++) {
        items[i].status = h[i].status;
        items[i].rounds = h[i].rounds;
        if (h[i].status != 0 && rc == BGPC_OK) rc = h[i].status;
    }
    return rc;
}

// ---------------------------------------------------------------------------
// Serving: continuous batching of coloring requests.
//
// A worker thread owns a device pool of `mem_budget` bytes and a pinned host
// staging area of the same size (same offsets).  Each pass it (1) retires
// every request whose done word (pinned host memory, written by the
// workgroup that colored it, after the colors) is set, and every group whose
// completion event fired (its table), (2) admits waiting requests in arrival
// order while a slot is free and the pool has room for the request's CSR
// arrays, colors and scratch, and (3) launches the admitted group on the next
// of four compute streams: uploads, one k_batch launch (one workgroup per
// graph).  Requests that arrive while other groups run join the next group,
// whose work overlaps the running ones on the device, and each request
// completes as soon as its own graph is done.  Graphs that one workgroup
// would color far slower than the whole device go to three more threads that
// run bgpc_color for them, each on a stream of its own (their arrays are
// allocated outside the pool).  A request's colors depend on its graph
// only.

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

// first-fit allocator over [0, cap) with coalescing; 256-byte granules
class RangeAlloc {
public:
    explicit RangeAlloc(size_t cap) { free_[0] = cap & ~(size_t)255; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (size_t)al256((long long)bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (size_t)al256((long long)bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

struct Req {
    bgpc_request r;
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t off = 0, bytes = 0;
    int status = 0, rounds = 0;
    int mode = MODE_MASKS, cap = 128;
    bool device = false;                 // whole-device path
    int slot = -1;                       // ring slot once published
    volatile long long *done = nullptr;  // pinned done word (batched path)
    // layout inside the request's pool block: uploaded arrays first, then
    // colors, then scratch; the done word sits at o_done in the staging area
    size_t o_aoff = 0, o_aidx = 0, o_boff = 0, o_bidx = 0, o_col = 0, o_scr = 0, o_done = 0;
};

// mode of a request's graph from its host arrays (the shape pass of the
// batched path, on the submitting thread); false if the arrays are malformed
bool host_mode(Req *q)
{
    const bgpc_request &r = q->r;
    const long long nnz = r.nnz;
    if (r.a_off[0] != 0 || r.a_off[r.n_a] != nnz || r.b_off[0] != 0 || r.b_off[r.n_b] != nnz) return false;
    double walk = 0.0;
    for (int v = 0; v < r.n_b; v++) {
        if (r.b_off[v + 1] < r.b_off[v] || r.b_off[v + 1] > nnz) return false;
        double sz = (double)(r.b_off[v + 1] - r.b_off[v]);
        walk += sz * sz;
    }
    for (long long j = 0; j < nnz; j++)
        if ((unsigned)r.b_idx[j] >= (unsigned)r.n_a) return false;
    long long wmax = 0;
    for (int u = 0; u < r.n_a; u++) {
        if (r.a_off[u + 1] < r.a_off[u] || r.a_off[u + 1] > nnz) return false;
        long long sum = 0;
        for (int k = r.a_off[u]; k < r.a_off[u + 1]; k++) {
            unsigned v = (unsigned)r.a_idx[k];
            if (v >= (unsigned)r.n_b) return false;
            sum += r.b_off[v + 1] - r.b_off[v];
        }
        wmax = std::max(wmax, std::min(sum, 0x3fffffffll));
    }
    q->mode = batch_mode(r.n_a, walk, wmax, &q->cap);
    BatchItem b = {};
    b.mode = q->mode;
    b.nnz = (int)nnz;
    q->device = whole_device(b);
    return true;
}

void layout(Req *q)
{
    const bgpc_request &r = q->r;
    size_t o = 0;
    q->o_aoff = o;
    o += al256(4 * ((long long)r.n_a + 1));
    q->o_aidx = o;
    o += al256(4 * (long long)r.nnz + 4);
    q->o_boff = o;
    o += al256(4 * ((long long)r.n_b + 1));
    q->o_bidx = o;
    o += al256(4 * (long long)r.nnz + 4);
    q->o_col = o;
    o += al256(4 * ((long long)r.n_a + 1));
    q->o_done = o;
    o += 256;
    q->o_scr = o;
    o += (size_t)batch_scratch_bytes(q->mode, r.n_a, r.n_b, q->cap);
    q->bytes = o;
}

}  // namespace

struct bgpc_session {
    int device = 0;
    size_t budget = 0;
    int max_slots = 0, max_group = 0, max_rounds = 0;
    char *dpool = nullptr;
    char *hpool = nullptr;
    char *hpool_dev = nullptr;      // device view of hpool
    RangeAlloc *alloc = nullptr;
    std::vector<hipStream_t> streams;   // uploads
    std::vector<hipEvent_t> events;     // free upload events
    static constexpr int KSTREAMS = 6;  // most serving-kernel launches that may run at once
    int nk = 1;                         // launches allowed at once (from the hardware queues)
    hipStream_t kstream[KSTREAMS] = {}; // one per launch in flight
    hipEvent_t kdone[KSTREAMS] = {};    // recorded after each launch
    bool klaunched[KSTREAMS] = {};
    std::chrono::steady_clock::time_point klast;   // last launch
    ServeRing *ring = nullptr, *ring_dev = nullptr;
    int cap = 0;                        // ring slots
    std::vector<Req *> slot_owner;      // request in each ring slot until it is done
    int *head = nullptr;                // device: descriptors claimed
    int tail = 0;                       // descriptors published
    int cus = 256;
    std::vector<hipStream_t> dev_streams;   // one per whole-device thread
    int rr = 0;
    int slots_used = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_dev;
    std::deque<Req *> submitted;    // guarded by mu
    std::vector<Req *> completed;   // guarded by mu
    std::deque<Req *> dev_queue;    // guarded by mu: graphs that need the whole device
    std::deque<Req *> dev_light;    // guarded by mu: graphs sent to idle whole-device threads under light load
    std::deque<Req *> pending;      // worker only: waiting for admission
    std::deque<std::pair<Req *, hipEvent_t>> uploading;   // worker only: arrays on their way
    std::vector<Req *> running;     // worker only: published, done word not yet seen
    std::thread worker;
    std::vector<std::thread> dev_workers;
    bool stop = false;              // guarded by mu
    bool kernels_stopped = false;   // worker only: after an error, the serving kernels have left
    bool dev_stop = false;          // guarded by mu: set once the worker has handed over every request
    int dev_busy = 0;               // guarded by mu: whole-device threads running a request
    int error = 0;

    bool upload(Req *q);
    bool publish(Req *q);
    void finish(Req *q);
    void loop();
    void dev_loop(int t);
    void dev_run(Req *q, hipStream_t s);
};

// copies a request's arrays into its pool block (staged through pinned
// memory unless they are pinned already) and queues the copies' event
bool bgpc_session::upload(Req *q)
{
    const bgpc_request &r = q->r;
    hipStream_t s = streams[rr++ % streams.size()];
    hipEvent_t ev = nullptr;
    if (!events.empty()) {
        ev = events.back();
        events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    char *hb = hpool + q->off, *db = dpool + q->off;
    bool ok = true;
    if (r.flags & BGPC_REQ_PINNED) {
        ok = ok && hipMemcpyAsync(db + q->o_aoff, r.a_off, 4 * ((size_t)r.n_a + 1), hipMemcpyHostToDevice, s) ==
                       hipSuccess;
        ok = ok && (!r.nnz || hipMemcpyAsync(db + q->o_aidx, r.a_idx, 4 * (size_t)r.nnz, hipMemcpyHostToDevice, s) ==
                                  hipSuccess);
        ok = ok && hipMemcpyAsync(db + q->o_boff, r.b_off, 4 * ((size_t)r.n_b + 1), hipMemcpyHostToDevice, s) ==
                       hipSuccess;
        ok = ok && (!r.nnz || hipMemcpyAsync(db + q->o_bidx, r.b_idx, 4 * (size_t)r.nnz, hipMemcpyHostToDevice, s) ==
                                  hipSuccess);
    } else {
        std::memcpy(hb + q->o_aoff, r.a_off, 4 * ((size_t)r.n_a + 1));
        if (r.nnz) std::memcpy(hb + q->o_aidx, r.a_idx, 4 * (size_t)r.nnz);
        std::memcpy(hb + q->o_boff, r.b_off, 4 * ((size_t)r.n_b + 1));
        if (r.nnz) std::memcpy(hb + q->o_bidx, r.b_idx, 4 * (size_t)r.nnz);
        ok = ok && hipMemcpyAsync(db, hb, q->o_col, hipMemcpyHostToDevice, s) == hipSuccess;
    }
    ok = ok && hipEventRecord(ev, s) == hipSuccess;
    if (!ok) {
        error = BGPC_E_HIP;
        (void)hipStreamSynchronize(s);
    }
    q->done = (volatile long long *)(hb + q->o_done);
    *q->done = 0;
    uploading.push_back({q, ev});
    return true;
}

// writes the request's descriptor into the next ring slot and raises tail;
// false while that slot still belongs to a request that is not done
bool bgpc_session::publish(Req *q)
{
    const int slot = tail % cap;
    if (slot_owner[slot]) return false;
    const bgpc_request &r = q->r;
    char *db = dpool + q->off, *hb_dev = hpool_dev + q->off;
    BatchItem b = {};
    b.n_a = r.n_a;
    b.n_b = r.n_b;
    b.a_off = (const int *)(db + q->o_aoff);
    b.a_idx = (const int *)(db + q->o_aidx);
    b.b_off = (const int *)(db + q->o_boff);
    b.b_idx = (const int *)(db + q->o_bidx);
    b.colors = (int *)(db + q->o_col);
    b.scratch = db + q->o_scr;
    b.max_rounds = max_rounds > 0 ? max_rounds : r.n_a + 65;
    b.mode = q->mode;
    b.cap = q->cap;
    b.status = -1;
    b.nnz = (int)r.nnz;
    void *user_dev = nullptr;
    if ((r.flags & BGPC_REQ_PINNED) && r.n_a && hipHostGetDevicePointer(&user_dev, r.colors_out, 0) != hipSuccess) {
        (void)hipGetLastError();
        error = BGPC_E_HIP;
    }
    b.host_colors = (r.flags & BGPC_REQ_PINNED) ? (int *)user_dev : (int *)(hb_dev + q->o_col);
    b.host_done = (long long *)(hb_dev + q->o_done);
    std::memcpy((void *)&ring->items[slot], &b, sizeof(b));
    std::atomic_thread_fence(std::memory_order_release);
    __atomic_store_n(&ring->tail, tail + 1, __ATOMIC_RELEASE);
    tail++;
    slot_owner[slot] = q;
    q->slot = slot;
    running.push_back(q);
    return true;
}

// a request whose done word is set: colors to the caller, memory back
void bgpc_session::finish(Req *q)
{
    const long long d = *q->done;
    if (q->r.n_a && !(q->r.flags & BGPC_REQ_PINNED))
        std::memcpy(q->r.colors_out, hpool + q->off + q->o_col, 4 * (size_t)q->r.n_a);
    q->status = error ? error : (int)(d & 0xffffffffll) - 256;
    q->rounds = (int)(d >> 32);
    q->t_done = now_s();
    alloc->release(q->off, q->bytes);
    if (q->slot >= 0) slot_owner[q->slot] = nullptr;
    slots_used--;
    {
        std::lock_guard<std::mutex> lk(mu);
        completed.push_back(q);
    }
    cv_done.notify_all();
}

void bgpc_session::loop()
{
    (void)hipSetDevice(device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (submitted.empty() && pending.empty() && uploading.empty() && running.empty()) {
                if (stop) break;
                cv_work.wait(lk, [&] { return stop || !submitted.empty(); });
                if (stop && submitted.empty()) break;
            }
            while (!submitted.empty()) {
                Req *q = submitted.front();
                submitted.pop_front();
                // light load: a graph that one workgroup of the serving
                // kernel would color slowly takes an idle whole-device
                // thread instead (same colors, far lower latency); under
                // load those threads stay busy and graphs go to the kernel
                if (!q->device && q->mode != MODE_DENSE && q->r.nnz >= LIGHT_LOAD_NNZ &&
                    dev_busy + (int)(dev_queue.size() + dev_light.size()) < (int)dev_streams.size()) {
                    dev_light.push_back(q);
                    cv_dev.notify_one();
                } else if (q->device) {
                    dev_queue.push_back(q);
                    cv_dev.notify_one();
                } else {
                    pending.push_back(q);
                }
            }
        }
        bool progress = false;
        if (error && !kernels_stopped) {
            // a failed call: nothing more is published, and no workgroup may
            // still read a request's arrays when its pool range is released
            __atomic_store_n(&ring->stop, 1, __ATOMIC_RELEASE);
            for (int k = 0; k < nk; k++)
                if (klaunched[k]) (void)hipEventSynchronize(kdone[k]);
            for (auto &u : uploading) (void)hipEventSynchronize(u.second);
            kernels_stopped = true;
        }
        // requests whose graphs are done
        for (size_t i = 0; i < running.size();) {
            if (*running[i]->done != 0 || error) {
                Req *q = running[i];
                running[i] = running.back();
                running.pop_back();
                finish(q);
                progress = true;
            } else {
                i++;
            }
        }
        // uploaded requests go on the ring, in admission order (after an
        // error they are retired instead)
        while (!uploading.empty() && error) {
            events.push_back(uploading.front().second);
            running.push_back(uploading.front().first);
            uploading.pop_front();
            progress = true;
        }
        while (!uploading.empty()) {
            hipError_t e = hipEventQuery(uploading.front().second);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) error = BGPC_E_HIP;
            if (!publish(uploading.front().first)) break;
            events.push_back(uploading.front().second);
            uploading.pop_front();
            progress = true;
        }
        // the serving kernel runs while published work is not done: a launch
        // when none is in flight, and another (on a free stream) when requests
        // wait unclaimed while fewer than one workgroup per CU is left (the
        // others having left after their idle polls); at most one launch per
        // millisecond
        if (!running.empty() && !error) {
            int in_flight = 0, free_k = -1;
            for (int k = 0; k < nk; k++) {
                bool alive = false;
                if (klaunched[k]) {
                    hipError_t e = hipEventQuery(kdone[k]);
                    if (e == hipErrorNotReady) alive = true;
                    else if (e != hipSuccess) error = BGPC_E_HIP;
                    else klaunched[k] = false;
                }
                if (alive) in_flight++;
                else if (free_k < 0) free_k = k;
            }
            const int active = __atomic_load_n(&ring->active, __ATOMIC_ACQUIRE);
            const int claimed = __atomic_load_n(&ring->claimed, __ATOMIC_ACQUIRE);
            const bool starved = tail > claimed && active < cus &&
                                 std::chrono::steady_clock::now() - klast > std::chrono::milliseconds(1);
            if (free_k >= 0 && !error && (in_flight == 0 || starved)) {
                // about 20 ms of empty polls (1,500 polls 14 us apart) before a workgroup leaves; an
                // extra launch brings only as many workgroups as requests
                // wait, so that idle polling does not crowd the device
                const int grid = in_flight == 0 ? std::max(1, cus * 2)
                                                : std::max(8, std::min(cus * 2, tail - claimed));
                k_serve<<<grid, BATCH_BLOCK, 0, kstream[free_k]>>>(ring_dev, cap, head, 1500);
                if (hipGetLastError() != hipSuccess || hipEventRecord(kdone[free_k], kstream[free_k]) != hipSuccess)
                    error = BGPC_E_HIP;
                klaunched[free_k] = true;
                klast = std::chrono::steady_clock::now();
                progress = true;
            }
        }
        // admit in arrival order while a slot and pool room are free
        int admitted = 0;
        while (!error && !pending.empty() && slots_used < max_slots && admitted < max_group) {
            Req *q = pending.front();
            if (!alloc->alloc(q->bytes, &q->off)) break;
            q->t_admit = now_s();
            pending.pop_front();
            slots_used++;
            admitted++;
            if (!upload(q)) {
                error = BGPC_E_HIP;
                q->done = (volatile long long *)(hpool + q->off + q->o_done);
                *q->done = 0;
                running.push_back(q);   // retired through the error path
            }
            progress = true;
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// one whole-device request: arrays in stream-ordered allocations, bgpc_color
void bgpc_session::dev_run(Req *q, hipStream_t s)
{
    const bgpc_request &r = q->r;
    const size_t b_aoff = 4 * ((size_t)r.n_a + 1), b_boff = 4 * ((size_t)r.n_b + 1), b_idx = 4 * (size_t)r.nnz + 4;
    const size_t b_col = 4 * ((size_t)r.n_a + 1);
    const size_t o1 = al256(b_aoff), o2 = o1 + al256(b_idx), o3 = o2 + al256(b_boff), o4 = o3 + al256(b_idx);
    char *d = nullptr;
    int st = BGPC_OK;
    int32_t rounds = 0;
    if (hipMallocAsync((void **)&d, o4 + al256(b_col), s) != hipSuccess) {
        (void)hipGetLastError();
        st = BGPC_E_OOM;
    }
    if (st == BGPC_OK) {
        bool ok = hipMemcpyAsync(d, r.a_off, b_aoff, hipMemcpyHostToDevice, s) == hipSuccess &&
                  (!r.nnz || hipMemcpyAsync(d + o1, r.a_idx, 4 * (size_t)r.nnz, hipMemcpyHostToDevice, s) ==
                                 hipSuccess) &&
                  hipMemcpyAsync(d + o2, r.b_off, b_boff, hipMemcpyHostToDevice, s) == hipSuccess &&
                  (!r.nnz || hipMemcpyAsync(d + o3, r.b_idx, 4 * (size_t)r.nnz, hipMemcpyHostToDevice, s) ==
                                 hipSuccess);
        if (!ok) st = BGPC_E_HIP;
    }
    if (st == BGPC_OK) {
        bgpc_csr A = {r.n_a, r.n_b, r.nnz, (const int32_t *)d, (const int32_t *)(d + o1)};
        bgpc_csr B = {r.n_b, r.n_a, r.nnz, (const int32_t *)(d + o2), (const int32_t *)(d + o3)};
        bgpc_opts o;
        bgpc_opts_default(&o);
        o.stream = s;
        o.max_rounds = max_rounds;
        o.rounds_out = &rounds;
        st = bgpc_color(&A, &B, nullptr, &o, (int32_t *)(d + o4));
        if ((st == BGPC_OK || st == BGPC_E_NOT_CONVERGED) && r.n_a &&
            (hipMemcpyAsync(r.colors_out, d + o4, 4 * (size_t)r.n_a, hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess))
            st = BGPC_E_HIP;
    }
    if (d) (void)hipFreeAsync(d, s);
    (void)hipStreamSynchronize(s);
    q->status = st;
    q->rounds = rounds;
    q->t_done = now_s();
}

void bgpc_session::dev_loop(int t)
{
    (void)hipSetDevice(device);
    for (;;) {
        Req *q = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_dev.wait(lk, [&] { return dev_stop || !dev_queue.empty() || !dev_light.empty(); });
            if (dev_queue.empty() && dev_light.empty()) {   // dev_stop and nothing left
                lk.unlock();
                release_thread_state();
                break;
            }
            // graphs that need the whole device first
            std::deque<Req *> &from = dev_queue.empty() ? dev_light : dev_queue;
            q = from.front();
            from.pop_front();
            dev_busy++;
        }
        q->t_admit = now_s();
        dev_run(q, dev_streams[t]);
        {
            std::lock_guard<std::mutex> lk(mu);
            dev_busy--;
            completed.push_back(q);
        }
        cv_done.notify_all();
    }
}

extern "C" {

BGPC_API bgpc_session *bgpc_session_create(size_t mem_budget, int32_t max_slots, int32_t max_group,
                                           int32_t max_rounds)
{
    if (mem_budget < (1u << 20) || max_slots < 1 || max_group < 1 || max_rounds < 0) return nullptr;
    bgpc_session *S = new bgpc_session();
    S->budget = mem_budget & ~(size_t)255;
    S->max_slots = max_slots;
    S->max_group = max_group;
    S->max_rounds = max_rounds;
    bool ok = hipGetDevice(&S->device) == hipSuccess;
    ok = ok && hipMalloc((void **)&S->dpool, S->budget) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&S->hpool, S->budget, hipHostMallocMapped) == hipSuccess;
    ok = ok && hipHostGetDevicePointer((void **)&S->hpool_dev, S->hpool, 0) == hipSuccess;
    for (int i = 0; i < 4 && ok; i++) {
        hipStream_t st;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) S->streams.push_back(st);
    }
    for (int i = 0; i < SIDE_STREAMS && ok; i++) {
        hipStream_t st;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) S->dev_streams.push_back(st);
    }
    // kernels on one hardware queue run in order: a second serving launch
    // only helps when its stream can have a queue of its own (HIP gives a
    // process GPU_MAX_HW_QUEUES queues, 4 unless set; the session's upload,
    // whole-device and kernel streams then share them)
    {
        const char *e = std::getenv("GPU_MAX_HW_QUEUES");
        const int hwq = e ? std::atoi(e) : 4;
        S->nk = hwq >= 16 ? bgpc_session::KSTREAMS : 1;
    }
    for (int k = 0; k < S->nk; k++) {
        ok = ok && hipStreamCreateWithFlags(&S->kstream[k], hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&S->kdone[k], hipEventDisableTiming) == hipSuccess;
    }
    // ring: a few times the slots, so that a slot is normally free again long
    // before its index comes round
    S->cap = std::max(64, 4 * max_slots);
    const size_t ring_bytes = sizeof(ServeRing) + sizeof(BatchItem) * (size_t)S->cap;
    ok = ok && hipHostMalloc((void **)&S->ring, ring_bytes, hipHostMallocMapped | hipHostMallocCoherent) ==
                   hipSuccess;
    ok = ok && hipHostGetDevicePointer((void **)&S->ring_dev, S->ring, 0) == hipSuccess;
    ok = ok && hipMalloc((void **)&S->head, 256) == hipSuccess;
    if (ok) {
        std::memset(S->ring, 0, ring_bytes);
        const int zero = 0;
        ok = hipMemcpy(S->head, &zero, sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        for (auto st : S->streams) (void)hipStreamDestroy(st);
        for (auto st : S->dev_streams) (void)hipStreamDestroy(st);
        for (int k = 0; k < bgpc_session::KSTREAMS; k++) {
            if (S->kstream[k]) (void)hipStreamDestroy(S->kstream[k]);
            if (S->kdone[k]) (void)hipEventDestroy(S->kdone[k]);
        }
        if (S->ring) (void)hipHostFree(S->ring);
        if (S->head) (void)hipFree(S->head);
        if (S->dpool) (void)hipFree(S->dpool);
        if (S->hpool) (void)hipHostFree(S->hpool);
        delete S;
        return nullptr;
    }
    S->slot_owner.assign(S->cap, nullptr);
    S->cus = device_cus();
    S->alloc = new RangeAlloc(S->budget);
    S->worker = std::thread([S] { S->loop(); });
    for (int t = 0; t < (int)S->dev_streams.size(); t++) S->dev_workers.emplace_back([S, t] { S->dev_loop(t); });
    return S;
}

BGPC_API int bgpc_session_submit(bgpc_session *S, const bgpc_request *r)
{
    if (!S || !r || r->n_a < 0 || r->n_b < 0 || r->nnz < 0 || r->nnz >= (1ll << 31) || !r->a_off || !r->b_off ||
        (r->nnz && (!r->a_idx || !r->b_idx)) || (r->n_a && !r->colors_out))
        return BGPC_E_INVALID;
    Req *q = new Req();
    q->r = *r;
    if (!host_mode(q)) {
        delete q;
        return BGPC_E_INVALID;
    }
    layout(q);
    if (!q->device && q->bytes + 4096 > S->budget) {
        delete q;
        return BGPC_E_OOM;   // could never be admitted
    }
    q->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->submitted.push_back(q);
    }
    S->cv_work.notify_one();
    return BGPC_OK;
}

BGPC_API int bgpc_session_poll(bgpc_session *S, bgpc_completion *out, int32_t cap, int32_t *n_out, int32_t wait_ms)
{
    if (!S || !n_out || cap < 0 || (cap > 0 && !out)) return BGPC_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->completed.empty() && wait_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->completed.empty(); });
    int k = 0;
    while (k < cap && !S->completed.empty()) {
        Req *q = S->completed.front();
        S->completed.erase(S->completed.begin());
        out[k].tag = q->r.tag;
        out[k].status = q->status;
        out[k].rounds = q->rounds;
        out[k].t_submit = q->t_submit;
        out[k].t_admit = q->t_admit;
        out[k].t_done = q->t_done;
        delete q;
        k++;
    }
    *n_out = k;
    return S->error;
}

BGPC_API void bgpc_session_destroy(bgpc_session *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    // every request is done: the serving kernel's workgroups leave
    __atomic_store_n(&S->ring->stop, 1, __ATOMIC_RELEASE);
    for (int k = 0; k < S->nk; k++) (void)hipStreamSynchronize(S->kstream[k]);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->dev_stop = true;
    }
    S->cv_dev.notify_all();
    for (auto &th : S->dev_workers)
        if (th.joinable()) th.join();
    for (auto st : S->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto st : S->dev_streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (int k = 0; k < S->nk; k++) {
        (void)hipStreamDestroy(S->kstream[k]);
        (void)hipEventDestroy(S->kdone[k]);
    }
    for (auto e : S->events) (void)hipEventDestroy(e);
    (void)hipHostFree(S->ring);
    (void)hipFree(S->head);
    for (Req *q : S->completed) delete q;
    for (Req *q : S->pending) delete q;
    for (Req *q : S->submitted) delete q;
    (void)hipFree(S->dpool);
    (void)hipHostFree(S->hpool);
    delete S->alloc;
    delete S;
}

}  // extern "C"
