// Batched coloring (bgpc_color_batch): many graphs, one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "batch.h"
#include "bgpc.h"

using namespace bgpc;

namespace {

const int kZero = 0;

int device_cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 256;
    return v;
}

bool item_ok(const bgpc_batch_item &it)
{
    const bgpc_csr &A = it.csr_A, &B = it.csr_B;
    return A.n_rows >= 0 && A.n_cols >= 0 && A.n_rows < (1 << 30) && A.n_cols < (1 << 30) && A.nnz >= 0 &&
           A.nnz < (1ll << 31) && A.n_rows == B.n_cols && A.n_cols == B.n_rows && A.nnz == B.nnz && A.offsets &&
           B.offsets && (A.nnz == 0 || (A.indices && B.indices)) && (A.n_rows == 0 || it.colors_out);
}

}  // namespace

namespace bgpc {

// One graph on one workgroup (bgpc_color's route for small dense graphs):
// the batch kernel with a single item and its own scratch.  Fills the round
// log (|W|, losers, largest color per round) when log is non-null.
int color_one_workgroup(const Graph &g, int *colors, int max_rounds, hipStream_t s, int log_cap,
                        std::vector<int> *log, int *rounds_out)
{
    const long long scr = batch_slot_bytes(g.n_a, g.n_b);
    const size_t o_tbl = 0, o_ord = 256, o_next = 512, o_log = 768;
    const size_t o_scr = o_log + (((size_t)3 * log_cap * 4 + 255) & ~(size_t)255);
    char *base = nullptr;
    if (hipMallocAsync((void **)&base, o_scr + (size_t)scr, s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_OOM;
    }
    BatchItem h;
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
    h.status = -1;
    h.rounds = 0;
    h.dense = 0;
    int zero[2] = {0, 0};
    int rc = BGPC_OK;
    if (hipMemcpyAsync(base + o_tbl, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(base + o_ord, zero, 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(base + o_next, zero, 4, hipMemcpyHostToDevice, s) != hipSuccess) {
        rc = BGPC_E_HIP;
    } else {
        k_batch<<<1, BATCH_BLOCK, 0, s>>>((BatchItem *)(base + o_tbl), (const int *)(base + o_ord), 1,
                                          (int *)(base + o_next), nullptr, 0, 0, 0);
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
    if (o.policy != BGPC_FIRST_FIT || o.net_color_mask != 0 || (o.flags & ~(uint32_t)BGPC_STRICT) ||
        o.start_round != 0)
        return BGPC_E_UNSUPPORTED;   // the batched path runs vertex-based first-fit rounds
    for (int i = 0; i < n_items; i++)
        if (!item_ok(items[i])) return BGPC_E_INVALID;
    if (n_items == 0) return BGPC_OK;
    hipStream_t s = (hipStream_t)o.stream;

    std::vector<BatchItem> h(n_items);
    int cap_a = 1, cap_b = 1;
    for (int i = 0; i < n_items; i++) {
        const bgpc_batch_item &it = items[i];
        BatchItem &b = h[i];
        b.n_a = it.csr_A.n_rows;
        b.n_b = it.csr_B.n_rows;
        b.a_off = it.csr_A.offsets;
        b.a_idx = it.csr_A.indices;
        b.b_off = it.csr_B.offsets;
        b.b_idx = it.csr_B.indices;
        b.colors = it.colors_out;
        b.scratch = nullptr;
        b.log = nullptr;
        b.log_cap = 0;
        b.max_rounds = o.max_rounds > 0 ? o.max_rounds : b.n_a + 65;
        b.status = -1;
        b.rounds = 0;
        b.dense = 0;
        cap_a = std::max(cap_a, b.n_a);
        cap_b = std::max(cap_b, b.n_b);
    }
    // largest graphs first
    std::vector<int> order(n_items);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return items[x].csr_A.nnz + items[x].csr_A.n_rows > items[y].csr_A.nnz + items[y].csr_A.n_rows;
    });
    const int grid = std::max(1, std::min(n_items, device_cus() * 2));
    const long long slot = batch_slot_bytes(cap_a, cap_b);
    const size_t tbl = ((size_t)n_items * sizeof(BatchItem) + 255) & ~(size_t)255;
    const size_t ord = ((size_t)n_items * 4 + 255) & ~(size_t)255;
    const size_t bytes = tbl + ord + 256 + (size_t)grid * slot;
    char *base = nullptr;
    if (hipMallocAsync((void **)&base, bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        return BGPC_E_OOM;
    }
    BatchItem *d_items = (BatchItem *)base;
    int *d_order = (int *)(base + tbl);
    int *d_next = (int *)(base + tbl + ord);
    char *slots = base + tbl + ord + 256;
    int rc = BGPC_OK;
    if (hipMemcpyAsync(d_items, h.data(), sizeof(BatchItem) * n_items, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_order, order.data(), 4 * (size_t)n_items, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_next, &kZero, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) {
        rc = BGPC_E_HIP;
    } else {
        k_batch<<<grid, BATCH_BLOCK, 0, s>>>(d_items, d_order, n_items, d_next, slots, slot, cap_a, cap_b);
        if (hipGetLastError() != hipSuccess) rc = BGPC_E_HIP;
        else if (hipMemcpyAsync(h.data(), d_items, sizeof(BatchItem) * n_items, hipMemcpyDeviceToHost, s) !=
                     hipSuccess ||
                 hipStreamSynchronize(s) != hipSuccess)
            rc = BGPC_E_HIP;
    }
    (void)hipFreeAsync(base, s);
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
// groups whose completion event has fired, (2) admits waiting requests in
// arrival order while a slot is free and the pool has room for the request's
// CSR arrays, colors and scratch, and (3) launches the admitted group on the
// next of four compute streams: uploads, one k_batch launch (one workgroup
// per graph), downloads of colors and statuses, completion event.  Requests
// that arrive while other groups run join the next group, whose work overlaps
// the running ones on the device.  A request's colors depend on its graph
// only.

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// first-fit allocator over [0, cap) with coalescing; 256-byte granules
class RangeAlloc {
public:
    explicit RangeAlloc(size_t cap) { free_[0] = cap & ~(size_t)255; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = al256(bytes);
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
        bytes = al256(bytes);
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
    // layout inside the request's pool block: uploaded arrays first, then
    // colors, then scratch
    size_t o_aoff = 0, o_aidx = 0, o_boff = 0, o_bidx = 0, o_col = 0, o_scr = 0;
};

void layout(Req *q)
{
    const bgpc_request &r = q->r;
    size_t o = 0;
    q->o_aoff = o;
    o += al256(4 * ((size_t)r.n_a + 1));
    q->o_aidx = o;
    o += al256(4 * (size_t)r.nnz + 4);
    q->o_boff = o;
    o += al256(4 * ((size_t)r.n_b + 1));
    q->o_bidx = o;
    o += al256(4 * (size_t)r.nnz + 4);
    q->o_col = o;
    o += al256(4 * ((size_t)r.n_a + 1));
    q->o_scr = o;
    o += (size_t)batch_slot_bytes(r.n_a, r.n_b);
    q->bytes = o;
}

struct Group {
    std::vector<Req *> reqs;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    size_t tbl_off = 0, tbl_bytes = 0;
};

}  // namespace

struct bgpc_session {
    int device = 0;
    size_t budget = 0;
    int max_slots = 0, max_group = 0, max_rounds = 0;
    char *dpool = nullptr;
    char *hpool = nullptr;
    RangeAlloc *alloc = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    int rr = 0;
    int slots_used = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> submitted;    // guarded by mu
    std::vector<Req *> completed;   // guarded by mu
    std::deque<Req *> pending;      // worker only
    std::vector<Group *> inflight;  // worker only
    std::thread worker;
    bool stop = false;              // guarded by mu
    int error = 0;

    bool launch(std::vector<Req *> &grp);
    void retire(Group *g);
    void loop();
};

bool bgpc_session::launch(std::vector<Req *> &grp)
{
    const int n = (int)grp.size();
    Group *g = new Group();
    g->reqs = grp;
    const size_t o_ord = al256(sizeof(BatchItem) * n), o_next = o_ord + al256(4 * (size_t)n);
    g->tbl_bytes = o_next + 256;
    if (!alloc->alloc(g->tbl_bytes, &g->tbl_off)) {
        delete g;
        return false;
    }
    g->stream = streams[rr++ % streams.size()];
    if (!events.empty()) {
        g->done = events.back();
        events.pop_back();
    } else if (hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess) {
        alloc->release(g->tbl_off, g->tbl_bytes);
        delete g;
        error = BGPC_E_HIP;
        return false;
    }
    char *ht = hpool + g->tbl_off, *dt = dpool + g->tbl_off;
    BatchItem *h_items = (BatchItem *)ht;
    int *h_order = (int *)(ht + o_ord);
    hipStream_t s = g->stream;
    bool ok = true;
    for (int i = 0; i < n; i++) {
        Req *q = grp[i];
        const bgpc_request &r = q->r;
        char *hb = hpool + q->off, *db = dpool + q->off;
        std::memcpy(hb + q->o_aoff, r.a_off, 4 * ((size_t)r.n_a + 1));
        if (r.nnz) std::memcpy(hb + q->o_aidx, r.a_idx, 4 * (size_t)r.nnz);
        std::memcpy(hb + q->o_boff, r.b_off, 4 * ((size_t)r.n_b + 1));
        if (r.nnz) std::memcpy(hb + q->o_bidx, r.b_idx, 4 * (size_t)r.nnz);
        ok = ok && hipMemcpyAsync(db, hb, q->o_col, hipMemcpyHostToDevice, s) == hipSuccess;
        BatchItem &b = h_items[i];
        b.n_a = r.n_a;
        b.n_b = r.n_b;
        b.a_off = (const int *)(db + q->o_aoff);
        b.a_idx = (const int *)(db + q->o_aidx);
        b.b_off = (const int *)(db + q->o_boff);
        b.b_idx = (const int *)(db + q->o_bidx);
        b.colors = (int *)(db + q->o_col);
        b.scratch = db + q->o_scr;
        b.log = nullptr;
        b.log_cap = 0;
        b.max_rounds = max_rounds > 0 ? max_rounds : r.n_a + 65;
        b.status = -1;
        b.rounds = 0;
        b.dense = 0;
        h_order[i] = i;
    }
    *(int *)(ht + o_next) = 0;
    ok = ok && hipMemcpyAsync(dt, ht, g->tbl_bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok) {
        k_batch<<<n, BATCH_BLOCK, 0, s>>>((BatchItem *)dt, (const int *)(dt + o_ord), n, (int *)(dt + o_next),
                                          nullptr, 0, 0, 0);
        ok = hipGetLastError() == hipSuccess;
    }
    for (int i = 0; i < n && ok; i++) {
        Req *q = grp[i];
        ok = hipMemcpyAsync(hpool + q->off + q->o_col, dpool + q->off + q->o_col, 4 * (size_t)q->r.n_a,
                            hipMemcpyDeviceToHost, s) == hipSuccess;
    }
    ok = ok && hipMemcpyAsync(ht, dt, sizeof(BatchItem) * n, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipEventRecord(g->done, s) == hipSuccess;
    if (!ok) {
        error = BGPC_E_HIP;
        (void)hipStreamSynchronize(s);
    }
    inflight.push_back(g);
    return true;
}

void bgpc_session::retire(Group *g)
{
    const double t = now_s();
    const BatchItem *h_items = (const BatchItem *)(hpool + g->tbl_off);
    std::vector<Req *> done;
    for (size_t i = 0; i < g->reqs.size(); i++) {
        Req *q = g->reqs[i];
        if (q->r.n_a) std::memcpy(q->r.colors_out, hpool + q->off + q->o_col, 4 * (size_t)q->r.n_a);
        q->status = error ? error : h_items[i].status;
        q->rounds = h_items[i].rounds;
        q->t_done = t;
        alloc->release(q->off, q->bytes);
        done.push_back(q);
    }
    slots_used -= (int)g->reqs.size();
    alloc->release(g->tbl_off, g->tbl_bytes);
    events.push_back(g->done);
    delete g;
    {
        std::lock_guard<std::mutex> lk(mu);
        completed.insert(completed.end(), done.begin(), done.end());
    }
    cv_done.notify_all();
}

void bgpc_session::loop()
{
    (void)hipSetDevice(device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (submitted.empty() && pending.empty() && inflight.empty()) {
                if (stop) break;
                cv_work.wait(lk, [&] { return stop || !submitted.empty(); });
                if (stop && submitted.empty()) break;
            }
            while (!submitted.empty()) {
                pending.push_back(submitted.front());
                submitted.pop_front();
            }
        }
        bool progress = false;
        // retire finished groups
        for (size_t i = 0; i < inflight.size();) {
            hipError_t q = hipEventQuery(inflight[i]->done);
            if (q == hipSuccess) {
                Group *g = inflight[i];
                inflight.erase(inflight.begin() + i);
                retire(g);
                progress = true;
            } else {
                if (q != hipErrorNotReady) error = BGPC_E_HIP;
                i++;
            }
        }
        // admit in arrival order while a slot and pool room are free
        std::vector<Req *> grp;
        while (!pending.empty() && slots_used + (int)grp.size() < max_slots && (int)grp.size() < max_group) {
            Req *q = pending.front();
            if (!alloc->alloc(q->bytes, &q->off)) break;
            q->t_admit = now_s();
            grp.push_back(q);
            pending.pop_front();
        }
        if (!grp.empty()) {
            if (launch(grp)) {
                slots_used += (int)grp.size();
                progress = true;
            } else {
                for (auto it = grp.rbegin(); it != grp.rend(); ++it) {
                    alloc->release((*it)->off, (*it)->bytes);
                    pending.push_front(*it);
                }
            }
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
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
    ok = ok && hipHostMalloc((void **)&S->hpool, S->budget, hipHostMallocDefault) == hipSuccess;
    for (int i = 0; i < 4 && ok; i++) {
        hipStream_t st;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) S->streams.push_back(st);
    }
    if (!ok) {
        (void)hipGetLastError();
        for (auto st : S->streams) (void)hipStreamDestroy(st);
        if (S->dpool) (void)hipFree(S->dpool);
        if (S->hpool) (void)hipHostFree(S->hpool);
        delete S;
        return nullptr;
    }
    S->alloc = new RangeAlloc(S->budget);
    S->worker = std::thread([S] { S->loop(); });
    return S;
}

BGPC_API int bgpc_session_submit(bgpc_session *S, const bgpc_request *r)
{
    if (!S || !r || r->n_a < 0 || r->n_b < 0 || r->nnz < 0 || r->nnz >= (1ll << 31) || !r->a_off || !r->b_off ||
        (r->nnz && (!r->a_idx || !r->b_idx)) || (r->n_a && !r->colors_out))
        return BGPC_E_INVALID;
    Req *q = new Req();
    q->r = *r;
    layout(q);
    if (q->bytes + 4096 > S->budget) {
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
    for (auto st : S->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto e : S->events) (void)hipEventDestroy(e);
    for (Req *q : S->completed) delete q;
    for (Req *q : S->pending) delete q;
    for (Req *q : S->submitted) delete q;
    (void)hipFree(S->dpool);
    (void)hipHostFree(S->hpool);
    delete S->alloc;
    delete S;
}

}  // extern "C"
