// hm_serve.hip -- serving loop: several compressed matrices resident in HBM,
// requests Y = K~_m W of any width submitted without blocking, continuous
// batching on the device.
//
// A server thread keeps, per resident matrix, a FIFO of pending requests, and
// owns max_slots slots.  A slot is a stream with its own workspaces (W and Y
// in tree order, the skeleton weights and potentials), dependency counters,
// queue head and error flag, sized when matrices are added for the largest of
// them at the widest sweep.  Whenever a slot is free and the HBM budget
// allows it, the server takes the matrix next in round-robin order that has
// pending requests, coalesces them column-wise into one sweep (up to
// kServeMaxCols columns), and enqueues on the slot's stream:
//   - a wait for each request's submit-time event (work the caller enqueued
//     on W or Y before submitting finishes first),
//   - a gather of every request's columns into the slot's W (tree order),
//   - one persistent task-graph launch of the matrix's plan for that width,
//   - a scatter of the result columns into every request's Y,
//   - a copy of the launch's error flag to host memory, and an event.
// Requests that arrive while sweeps run are admitted as soon as a slot frees
// up, also for a matrix that already has a sweep in flight (each slot has its
// own workspaces), so the sweeps of one or several matrices overlap on the
// device.  Column j of Y depends only on column j of W, and a column's
// arithmetic does not depend on which columns share its sweep or on the
// slot, so a result is bitwise the same alone and in the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>

#include "hm_internal.h"

namespace {

using hm::kServeMaxCols;
constexpr size_t kMaxPending = 1 << 16;

double now_us() {
    return std::chrono::duration<double, std::micro>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    hm_ticket ticket = 0;
    int mat = 0;
    const void *W = nullptr;
    void *Y = nullptr;
    int64_t ldw = 0, ldy = 0, Q = 0;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream
    double t_submit = 0, latency_us = 0;
    int done = 0;
    hm_status status = HM_OK;
};

// Plans of one resident matrix, one per (column tile, padded columns) shape a
// sweep of 1..kServeMaxCols columns can take.
struct Resident {
    hm_matrix h = nullptr;
    std::deque<Req *> pending;
    std::map<std::pair<int, int>, hm::GraphPlan> plans;
};

struct Slot {
    hipStream_t stream = nullptr;
    void *ws[hm::BUF_COUNT] = {nullptr};
    size_t ws_bytes[hm::BUF_COUNT] = {0};
    int32_t *counters = nullptr;
    int64_t n_counters = 0;
    int32_t *head = nullptr;            // queue head, error flag
    hm::MatDesc *mats = nullptr;        // one descriptor per resident matrix (this slot's workspaces)
    int n_mats = 0;
    hm::ReqDesc *d_reqs = nullptr;      // the sweep's request table
    int16_t *d_col2req = nullptr;
    hm::ReqDesc *h_reqs = nullptr;      // pinned staging of the same
    int16_t *h_col2req = nullptr;
    int32_t *h_err = nullptr;           // pinned copy of the error flag after the sweep
    hipEvent_t done = nullptr;
    bool busy = false;
    int mat = -1;
    std::vector<Req *> reqs;
    size_t bytes = 0;
};

}  // namespace

struct hm_server_s {
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    hm_dtype dtype = HM_F32;
    hm_prec prec = HM_PREC_FP32;
    int es = 4;
    std::vector<Resident> mats;
    std::vector<Slot> slots;
    int64_t max_N = 0, max_R = 0;       // workspace rows the slots hold
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> incoming;
    std::unordered_map<hm_ticket, Req *> reqs;
    hm_ticket next_ticket = 1;
    std::thread th;
    std::atomic<bool> stop{false};
    size_t inflight_bytes = 0;
    int inflight = 0;
    int rr = 0;                        // round-robin start over matrices
    // statistics
    int64_t completed = 0, sweeps = 0, columns = 0, failed = 0;
    size_t peak_bytes = 0;
    int peak_inflight = 0;
};

namespace hm {
namespace {

#define HM_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? HM_ERR_NOMEM : HM_ERR_DEVICE,     \
                        std::string(#call ": ") + hipGetErrorString(e_));            \
    } while (0)

// Column tile and padded columns of a sweep of `cols` columns (in 256-column
// launches the last tile no wider than it needs, except with a symmetric
// store).
std::pair<int, int> sweep_shape(hm_server S, hm_matrix h, int64_t cols) {
    const int bn = graph_bn(cols, S->es, false, h->task_k);
    return {bn, (int)padded_columns(cols, bn, !h->symmetric && bn == 256)};
}

void finish(hm_server S, Req *r, hm_status st, double t) {
    r->status = st;
    r->latency_us = t - r->t_submit;
    r->done = 1;
    if (r->ready) {
        (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
    }
    if (st == HM_OK)
        S->completed++;
    else
        S->failed++;
}

// Start one sweep of matrix m on slot `si` (mutex held by the caller).
// Returns false when nothing was started.
bool try_launch(hm_server S, int m, int si) {
    Resident &R = S->mats[m];
    Slot &sl = S->slots[si];
    if (R.pending.empty() || sl.busy) return false;
    // coalesce pending requests, oldest first
    std::vector<Req *> take;
    int64_t cols = 0;
    for (Req *r : R.pending) {
        if (cols + r->Q > kServeMaxCols) break;
        take.push_back(r);
        cols += r->Q;
    }
    const size_t need = 2 * (size_t)R.h->N * (size_t)cols * S->es;
    if (S->inflight_bytes + need > S->budget && S->inflight > 0) return false;  // wait for memory
    for (size_t i = 0; i < take.size(); i++) R.pending.pop_front();
    const std::pair<int, int> shape = sweep_shape(S, R.h, cols);
    const GraphPlan &plan = R.plans.at(shape);
    const int64_t width = shape.second;
    // request table (pinned staging, copied on the slot's stream)
    int64_t off = 0;
    for (size_t i = 0; i < take.size(); i++) {
        Req *r = take[i];
        sl.h_reqs[i] = ReqDesc{r->W, r->ldw, r->Y, r->ldy, off, r->Q};
        for (int64_t c = 0; c < r->Q; c++) sl.h_col2req[off + c] = (int16_t)i;
        off += r->Q;
    }
    hipStream_t st = sl.stream;
    hipError_t e = hipSuccess;
    for (Req *r : take)
        if (e == hipSuccess && r->ready) e = hipStreamWaitEvent(st, r->ready, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.d_reqs, sl.h_reqs, sizeof(ReqDesc) * take.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.d_col2req, sl.h_col2req, sizeof(int16_t) * (size_t)cols, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_gather_in(sl.d_reqs, sl.d_col2req, cols, width, sl.ws[BUF_WT], kServeMaxCols, R.h->d_perm,
                             R.h->N, S->es, st);
    if (e == hipSuccess) {
        const int workers =
            std::max(1, persistent_occupancy(S->es, shape.first, false, R.h->symmetric, plan.narrow) * R.h->n_cu);
        e = launch_persistent(plan, S->es, sl.mats + m, sl.head, std::min(plan.n_tasks, workers), st,
                              OutScatter{}, sl.counters);
    }
    if (e == hipSuccess)
        e = launch_scatter_out(sl.d_reqs, sl.d_col2req, cols, sl.ws[BUF_YT], kServeMaxCols, R.h->d_perm, R.h->N,
                               S->es, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sl.h_err, sl.head + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(sl.done, st);
    if (e != hipSuccess) {
        // fail these requests, keep serving the others
        (void)hipStreamSynchronize(st);
        const double t = now_us();
        for (Req *r : take) finish(S, r, HM_ERR_DEVICE, t);
        return false;
    }
    sl.busy = true;
    sl.mat = m;
    sl.reqs = std::move(take);
    sl.bytes = need;
    S->inflight++;
    S->inflight_bytes += need;
    S->peak_bytes = std::max(S->peak_bytes, S->inflight_bytes);
    S->peak_inflight = std::max(S->peak_inflight, S->inflight);
    S->sweeps++;
    S->columns += cols;
    return true;
}

void server_loop(hm_server S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->stop.load()) {
        // route new requests
        while (!S->incoming.empty()) {
            Req *r = S->incoming.front();
            S->incoming.pop_front();
            S->mats[r->mat].pending.push_back(r);
        }
        // retire finished sweeps
        for (Slot &sl : S->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            hm_status st = q == hipSuccess ? HM_OK : HM_ERR_DEVICE;
            if (st == HM_OK && *sl.h_err) {
                // a bounded dependency wait expired: this sweep's results are invalid
                st = HM_ERR_INTERNAL;
                const int32_t zero = 0;
                (void)hipMemcpy(sl.head + 1, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
                *sl.h_err = 0;
            }
            const double t = now_us();
            for (Req *r : sl.reqs) finish(S, r, st, t);
            sl.reqs.clear();
            sl.busy = false;
            S->inflight--;
            S->inflight_bytes -= sl.bytes;
        }
        // start sweeps on free slots, round robin over the matrices
        const int nm = (int)S->mats.size();
        for (int si = 0; si < (int)S->slots.size() && nm > 0; si++) {
            if (S->slots[si].busy) continue;
            for (int k = 0; k < nm; k++) {
                const int m = (S->rr + k) % nm;
                if (try_launch(S, m, si)) {
                    S->rr = (m + 1) % nm;
                    break;
                }
            }
        }
        S->cv.wait_for(lk, std::chrono::microseconds(S->inflight > 0 ? 20 : 500));
    }
}

void free_slot(Slot &sl) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    for (void *&p : sl.ws)
        if (p) (void)hipFree(p), p = nullptr;
    if (sl.counters) (void)hipFree(sl.counters);
    if (sl.head) (void)hipFree(sl.head);
    if (sl.mats) (void)hipFree(sl.mats);
    if (sl.d_reqs) (void)hipFree(sl.d_reqs);
    if (sl.d_col2req) (void)hipFree(sl.d_col2req);
    if (sl.h_reqs) (void)hipHostFree(sl.h_reqs);
    if (sl.h_col2req) (void)hipHostFree(sl.h_col2req);
    if (sl.h_err) (void)hipHostFree(sl.h_err);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    sl = Slot{};
}

void destroy_server(hm_server S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop.store(true);
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    (void)hipSetDevice(S->device);
    for (Slot &sl : S->slots) free_slot(sl);
    for (Resident &R : S->mats)
        for (auto &kv : R.plans) free_plan(kv.second);
    for (auto &kv : S->reqs) {
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    delete S;
}

// Per-slot resources that do not depend on the resident matrices.
hm_status init_slot(Slot &sl) {
    HM_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    HM_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    HM_HIP(hipMalloc(&sl.head, 2 * sizeof(int32_t)));
    HM_HIP(hipMemset(sl.head, 0, 2 * sizeof(int32_t)));
    HM_HIP(hipMalloc(&sl.d_reqs, sizeof(ReqDesc) * kServeMaxCols));
    HM_HIP(hipMalloc(&sl.d_col2req, sizeof(int16_t) * kServeMaxCols));
    HM_HIP(hipHostMalloc(&sl.h_reqs, sizeof(ReqDesc) * kServeMaxCols, hipHostMallocDefault));
    HM_HIP(hipHostMalloc(&sl.h_col2req, sizeof(int16_t) * kServeMaxCols, hipHostMallocDefault));
    HM_HIP(hipHostMalloc(&sl.h_err, sizeof(int32_t), hipHostMallocDefault));
    *sl.h_err = 0;
    return HM_OK;
}

// Size every slot for the resident matrices (workspaces of max_N / max_R rows
// at kServeMaxCols columns, counters for the largest plan) and upload its
// descriptor table.  Runs before any sweep (hm_server_add refuses otherwise).
hm_status provision_slots(hm_server S, int64_t n_counters) {
    const size_t rows[BUF_COUNT] = {(size_t)S->max_N, (size_t)S->max_N, (size_t)S->max_R, (size_t)S->max_R};
    for (Slot &sl : S->slots) {
        for (int b = 0; b < BUF_COUNT; b++) {  // grow only
            const size_t need = std::max<size_t>(rows[b] * kServeMaxCols * S->es, 256);
            if (sl.ws_bytes[b] >= need) continue;
            if (sl.ws[b]) HM_HIP(hipFree(sl.ws[b]));
            sl.ws[b] = nullptr;
            sl.ws_bytes[b] = 0;
            HM_HIP(hipMalloc(&sl.ws[b], need));
            sl.ws_bytes[b] = need;
        }
        if (n_counters > sl.n_counters) {
            if (sl.counters) HM_HIP(hipFree(sl.counters));
            sl.counters = nullptr;
            HM_HIP(hipMalloc(&sl.counters, sizeof(int32_t) * (size_t)n_counters));
            sl.n_counters = n_counters;
        }
        std::vector<MatDesc> md;
        for (const Resident &R : S->mats)
            md.push_back(MatDesc{R.h->prec[S->prec].blocks, {sl.ws[0], sl.ws[1], sl.ws[2], sl.ws[3]},
                                 kServeMaxCols, R.h->d_segs});
        if (sl.mats) HM_HIP(hipFree(sl.mats));
        sl.mats = nullptr;
        HM_HIP(hipMalloc(&sl.mats, sizeof(MatDesc) * std::max<size_t>(md.size(), 1)));
        if (!md.empty()) HM_HIP(hipMemcpy(sl.mats, md.data(), sizeof(MatDesc) * md.size(), hipMemcpyHostToDevice));
        sl.n_mats = (int)md.size();
    }
    return HM_OK;
}

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" {

hm_status hm_server_create(int device, size_t hbm_budget, int max_slots, hm_dtype dtype,
                           hm_prec prec, hm_server *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_server_create: out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 16) return fail(HM_ERR_INVALID, "hm_server_create: max_slots must be 1..16");
    if (hbm_budget == 0) return fail(HM_ERR_INVALID, "hm_server_create: hbm_budget is 0");
    if (!((dtype == HM_F64 && prec == HM_PREC_FP64) || (dtype == HM_F32 && prec == HM_PREC_FP32)))
        return fail(HM_ERR_INVALID, "hm_server_create: dtype and precision do not match");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(HM_ERR_INVALID, "hm_server_create: no such HIP device");
    hm_server S = new (std::nothrow) hm_server_s();
    if (!S) return fail(HM_ERR_NOMEM, "hm_server_create: allocation failed");
    S->device = device;
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    S->dtype = dtype;
    S->prec = prec;
    S->es = dtype == HM_F64 ? 8 : 4;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    S->slots.resize(max_slots);
    for (Slot &sl : S->slots) {
        hm_status st = init_slot(sl);
        if (st != HM_OK) {
            (void)hipSetDevice(prev);
            destroy_server(S);
            return st;
        }
    }
    (void)hipSetDevice(prev);
    S->th = std::thread(server_loop, S);
    *out = S;
    return HM_OK;
}

hm_status hm_server_add(hm_server S, hm_matrix h, int *mat_id) {
    if (!S || !h || !mat_id) return fail(HM_ERR_INVALID, "hm_server_add: NULL argument");
    if (h->device != S->device) return fail(HM_ERR_INVALID, "hm_server_add: matrix on another device");
    if (!h->prec[S->prec].blocks) return fail(HM_ERR_INVALID, "hm_server_add: precision not loaded");
    if (!h->near_stored || !h->far_stored)
        return fail(HM_ERR_INVALID, "hm_server_add: matrix loaded without its near or far blocks");
    std::lock_guard<std::mutex> g(S->mu);
    if (S->inflight > 0) return fail(HM_ERR_BUSY, "hm_server_add: sweeps are running; add matrices before submitting work");
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    struct Restore {
        int d;
        ~Restore() { (void)hipSetDevice(d); }
    } restore{prev};
    // a plan for every (column tile, padded columns) shape of a 1..kServeMaxCols
    // column sweep, so that sweeps never plan, allocate or upload
    Resident R;
    R.h = h;
    hm_status st = HM_OK;
    int64_t n_counters = 0;
    for (const Slot &sl : S->slots) n_counters = std::max(n_counters, sl.n_counters);
    for (int64_t q = 1; q <= kServeMaxCols && st == HM_OK; q++) {
        const std::pair<int, int> shape = sweep_shape(S, h, q);
        if (R.plans.count(shape)) continue;
        GraphPlan p;
        std::vector<PlanPart> parts{{h, 0, shape.second, 0, false}};
        const bool narrow = shape.second % shape.first != 0;
        st = build_plan(parts, shape.first, S->es,
                        persistent_occupancy(S->es, shape.first, false, h->symmetric, narrow) * h->n_cu, p);
        if (st == HM_OK) {
            n_counters = std::max<int64_t>(n_counters, p.n_tasks);
            R.plans[shape] = p;
        }
    }
    if (st != HM_OK) {
        for (auto &kv : R.plans) free_plan(kv.second);
        return st;
    }
    S->mats.push_back(std::move(R));
    S->max_N = std::max(S->max_N, h->N);
    S->max_R = std::max(S->max_R, h->skel_rows);
    st = provision_slots(S, std::max<int64_t>(n_counters, 1));
    if (st != HM_OK) {
        for (auto &kv : S->mats.back().plans) free_plan(kv.second);
        S->mats.pop_back();
        return st;
    }
    *mat_id = (int)S->mats.size() - 1;
    return HM_OK;
}

hm_status hm_submit(hm_server S, int mat_id, const void *W, int64_t ldw, void *Y, int64_t ldy,
                    int64_t Q, void *stream, hm_ticket *out) {
    if (!S || !out || !W || !Y) return fail(HM_ERR_INVALID, "hm_submit: NULL argument");
    *out = 0;
    if (Q < 1 || Q > kServeMaxCols) return fail(HM_ERR_INVALID, "hm_submit: Q must be in [1, 1024]");
    if (ldw < Q || ldy < Q) return fail(HM_ERR_INVALID, "hm_submit: leading dimension < Q");
    int64_t N = 0;
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (mat_id < 0 || mat_id >= (int)S->mats.size()) return fail(HM_ERR_INVALID, "hm_submit: unknown matrix");
        N = S->mats[mat_id].h->N;
        if (S->reqs.size() >= kMaxPending) return fail(HM_ERR_BUSY, "hm_submit: too many requests in flight");
    }
    const size_t need = 2 * (size_t)N * Q * S->es;
    if (need > S->budget) return fail(HM_ERR_BUSY, "hm_submit: request larger than the HBM budget");
    Req *r = new (std::nothrow) Req();
    if (!r) return fail(HM_ERR_NOMEM, "hm_submit: allocation failed");
    // order the request after the work the caller has enqueued on `stream`
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    hipError_t e = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->ready, (hipStream_t)stream);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        if (r->ready) (void)hipEventDestroy(r->ready);
        delete r;
        return fail(HM_ERR_DEVICE, std::string("hm_submit: recording the ready event: ") + hipGetErrorString(e));
    }
    r->mat = mat_id;
    r->W = W;
    r->ldw = ldw;
    r->Y = Y;
    r->ldy = ldy;
    r->Q = Q;
    r->t_submit = now_us();
    std::lock_guard<std::mutex> g(S->mu);
    r->ticket = S->next_ticket++;
    S->reqs[r->ticket] = r;
    S->incoming.push_back(r);
    S->cv.notify_one();
    *out = r->ticket;
    return HM_OK;
}

hm_status hm_poll(hm_server S, hm_ticket t, int *done, double *latency_us) {
    if (!S || !done) return fail(HM_ERR_INVALID, "hm_poll: NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) return fail(HM_ERR_INVALID, "hm_poll: unknown or retired ticket");
    Req *r = it->second;
    *done = r->done;
    if (!r->done) return HM_OK;
    if (latency_us) *latency_us = r->latency_us;
    const hm_status st = r->status;
    S->reqs.erase(it);  // a completed ticket is retired by the poll that reports it
    delete r;
    if (st == HM_OK) return HM_OK;
    return fail(st, st == HM_ERR_INTERNAL ? "hm_poll: a dependency wait of the request's sweep timed out; Y is invalid"
                                          : "hm_poll: the request's sweep failed");
}

hm_status hm_server_stats(hm_server S, hm_server_stats_t *o) {
    if (!S || !o) return fail(HM_ERR_INVALID, "hm_server_stats: NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    o->completed = S->completed;
    o->failed = S->failed;
    o->sweeps = S->sweeps;
    o->columns = S->columns;
    o->pending = 0;
    for (const Resident &R : S->mats) o->pending += (int64_t)R.pending.size();
    o->pending += (int64_t)S->incoming.size();
    o->inflight = (int32_t)S->inflight;
    o->peak_inflight = S->peak_inflight;
    o->peak_bytes = (double)S->peak_bytes;
    return HM_OK;
}

hm_status hm_server_destroy(hm_server S) {
    destroy_server(S);
    return HM_OK;
}

}  // extern "C"
