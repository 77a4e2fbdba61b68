// hm_serve.hip -- serving loop: several compressed matrices resident in HBM,
// requests Y = K~_m W of any width submitted without blocking, continuous
// batching on the device.
//
// A server thread keeps, per resident matrix, a FIFO of pending requests.
// Whenever the matrix has no sweep in flight, a slot (stream) is free and the
// HBM budget allows it, the pending requests are coalesced column-wise into
// one packed W (up to kMaxCols columns), evaluated by one sweep (the
// persistent task-graph launch of hm_eval), and their columns scattered back
// into each request's Y.  Requests that arrive while a sweep of their matrix
// is on the device join the next sweep; sweeps of different matrices run on
// different streams and overlap on the device.  Column j of Y depends only on
// column j of W and the arithmetic of a column does not depend on which
// columns share its sweep, so a result is bitwise the same alone and in the
// mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>

#include "hm_internal.h"

namespace {

constexpr int64_t kMaxCols = 1024;     // widest coalesced sweep
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
    double t_submit = 0, latency_us = 0;
    int done = 0;
    hm_status status = HM_OK;
};

struct Resident {
    hm_matrix h = nullptr;
    bool busy = false;
    std::deque<Req *> pending;
};

struct Sweep {
    int mat = -1, slot = -1;
    std::vector<Req *> reqs;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
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
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> incoming;
    std::unordered_map<hm_ticket, Req *> reqs;
    hm_ticket next_ticket = 1;
    std::thread th;
    std::atomic<bool> stop{false};
    std::vector<hipStream_t> streams;
    std::vector<void *> pack;          // per slot: packed W then packed Y
    std::vector<size_t> pack_bytes;
    std::vector<int> slot_busy;
    std::vector<Sweep> inflight;
    size_t inflight_bytes = 0;
    int rr = 0;                        // round-robin start over matrices
    // statistics
    int64_t completed = 0, sweeps = 0, columns = 0, failed = 0;
    size_t peak_bytes = 0;
    int peak_inflight = 0;
    std::string thread_error;
};

namespace hm {
namespace {

// Launch one sweep for matrix m (mutex held by the caller).
bool try_launch(hm_server S, int m) {
    Resident &R = S->mats[m];
    if (R.busy || R.pending.empty()) return false;
    int slot = -1;
    for (int i = 0; i < S->max_slots; i++)
        if (!S->slot_busy[i]) {
            slot = i;
            break;
        }
    if (slot < 0) return false;
    // coalesce pending requests, oldest first
    std::vector<Req *> take;
    int64_t cols = 0;
    for (Req *r : R.pending) {
        if (!take.empty() && cols + r->Q > kMaxCols) break;
        take.push_back(r);
        cols += r->Q;
    }
    const int64_t ld = cols;  // packed leading dimension
    const size_t need = 2 * (size_t)R.h->N * (size_t)ld * S->es;
    if (S->inflight_bytes + need > S->budget && !S->inflight.empty()) return false;  // wait for memory
    if (need > S->pack_bytes[slot]) return false;  // cannot happen: sized at add time
    for (size_t i = 0; i < take.size(); i++) R.pending.pop_front();
    char *Wp = (char *)S->pack[slot], *Yp = Wp + (size_t)R.h->N * ld * S->es;
    hipStream_t st = S->streams[slot];
    hm_status status = HM_OK;
    int64_t off = 0;
    for (Req *r : take) {
        if (hipMemcpy2DAsync(Wp + off * S->es, ld * S->es, r->W, r->ldw * S->es, r->Q * S->es,
                             R.h->N, hipMemcpyDeviceToDevice, st) != hipSuccess)
            status = HM_ERR_DEVICE;
        off += r->Q;
    }
    if (status == HM_OK)
        status = hm_eval(R.h, Wp, ld, Yp, ld, cols, S->dtype, S->prec, 0, st);
    off = 0;
    for (Req *r : take) {
        if (status == HM_OK &&
            hipMemcpy2DAsync(r->Y, r->ldy * S->es, Yp + off * S->es, ld * S->es, r->Q * S->es,
                             R.h->N, hipMemcpyDeviceToDevice, st) != hipSuccess)
            status = HM_ERR_DEVICE;
        off += r->Q;
    }
    Sweep sw;
    sw.mat = m;
    sw.slot = slot;
    sw.reqs = take;
    sw.bytes = need;
    if (hipEventCreateWithFlags(&sw.done, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(sw.done, st) != hipSuccess)
        status = HM_ERR_DEVICE;
    if (status != HM_OK) {
        // fail these requests, keep serving the others
        for (Req *r : take) {
            r->status = status;
            r->done = 1;
            r->latency_us = now_us() - r->t_submit;
            S->failed++;
        }
        if (sw.done) {
            (void)hipStreamSynchronize(st);
            (void)hipEventDestroy(sw.done);
        }
        return false;
    }
    R.busy = true;
    S->slot_busy[slot] = 1;
    S->inflight_bytes += need;
    S->peak_bytes = std::max(S->peak_bytes, S->inflight_bytes);
    S->inflight.push_back(sw);
    S->peak_inflight = std::max(S->peak_inflight, (int)S->inflight.size());
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
        for (size_t i = 0; i < S->inflight.size();) {
            Sweep &sw = S->inflight[i];
            hipError_t q = hipEventQuery(sw.done);
            if (q == hipErrorNotReady) {
                i++;
                continue;
            }
            const double t = now_us();
            for (Req *r : sw.reqs) {
                r->status = q == hipSuccess ? HM_OK : HM_ERR_DEVICE;
                r->latency_us = t - r->t_submit;
                r->done = 1;
                if (q == hipSuccess) S->completed++;
                else S->failed++;
            }
            (void)hipEventDestroy(sw.done);
            S->mats[sw.mat].busy = false;
            S->slot_busy[sw.slot] = 0;
            S->inflight_bytes -= sw.bytes;
            S->inflight[i] = S->inflight.back();
            S->inflight.pop_back();
        }
        // start sweeps, round robin over the matrices
        const int nm = (int)S->mats.size();
        for (int k = 0; k < nm; k++) {
            const int m = (S->rr + k) % std::max(nm, 1);
            if (try_launch(S, m)) S->rr = (m + 1) % nm;
        }
        const bool work = !S->inflight.empty();
        S->cv.wait_for(lk, std::chrono::microseconds(work ? 20 : 500));
    }
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
    for (hipStream_t st : S->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (Sweep &sw : S->inflight)
        if (sw.done) (void)hipEventDestroy(sw.done);
    for (void *p : S->pack)
        if (p) (void)hipFree(p);
    for (auto &kv : S->reqs) delete kv.second;
    for (Req *r : S->incoming) delete r;
    delete S;
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
    S->streams.assign(max_slots, nullptr);
    S->pack.assign(max_slots, nullptr);
    S->pack_bytes.assign(max_slots, 0);
    S->slot_busy.assign(max_slots, 0);
    for (int i = 0; i < max_slots; i++)
        if (hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking) != hipSuccess) {
            (void)hipSetDevice(prev);
            destroy_server(S);
            return fail(HM_ERR_DEVICE, "hm_server_create: stream creation failed");
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
    if (!S->inflight.empty()) return fail(HM_ERR_BUSY, "hm_server_add: add matrices before submitting work");
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    // workspaces and plans for every sweep width, so that sweeps never
    // allocate or synchronize
    const int slot = S->dtype == HM_F64 ? 0 : 1;
    hm_status st = reserve_ws(h, slot, kMaxCols);
    // every (column tile, tile count) that hm_eval can choose for a sweep of
    // 1..kMaxCols columns
    std::vector<std::pair<int, int64_t>> shapes;
    for (int64_t q = 1; q <= kMaxCols && st == HM_OK; q++) {
        const int bn = graph_bn(q, S->es, false, h->task_k);
        const std::pair<int, int64_t> key{bn, (q + bn - 1) / bn * bn};
        if (std::find(shapes.begin(), shapes.end(), key) != shapes.end()) continue;
        shapes.push_back(key);
        GraphPlan *p = nullptr;
        st = get_plan(h, slot, bn, key.second, persistent_occupancy(S->es, bn) * h->n_cu, &p);
    }
    const size_t need = 2 * (size_t)h->N * kMaxCols * S->es;
    for (int i = 0; i < S->max_slots && st == HM_OK; i++)
        if (S->pack_bytes[i] < need) {
            if (S->pack[i]) (void)hipFree(S->pack[i]);
            S->pack[i] = nullptr;
            S->pack_bytes[i] = 0;
            if (hipMalloc(&S->pack[i], need) != hipSuccess) st = fail(HM_ERR_NOMEM, "hm_server_add: packing buffers");
            else S->pack_bytes[i] = need;
        }
    (void)hipSetDevice(prev);
    if (st != HM_OK) return st;
    Resident R;
    R.h = h;
    S->mats.push_back(R);
    *mat_id = (int)S->mats.size() - 1;
    return HM_OK;
}

hm_status hm_submit(hm_server S, int mat_id, const void *W, int64_t ldw, void *Y, int64_t ldy,
                    int64_t Q, hm_ticket *out) {
    if (!S || !out || !W || !Y) return fail(HM_ERR_INVALID, "hm_submit: NULL argument");
    *out = 0;
    std::lock_guard<std::mutex> g(S->mu);
    if (mat_id < 0 || mat_id >= (int)S->mats.size()) return fail(HM_ERR_INVALID, "hm_submit: unknown matrix");
    if (Q < 1 || Q > kMaxCols) return fail(HM_ERR_INVALID, "hm_submit: Q must be in [1, 1024]");
    if (ldw < Q || ldy < Q) return fail(HM_ERR_INVALID, "hm_submit: leading dimension < Q");
    const size_t need = 2 * (size_t)S->mats[mat_id].h->N * Q * S->es;
    if (need > S->budget) return fail(HM_ERR_BUSY, "hm_submit: request larger than the HBM budget");
    if (S->reqs.size() >= kMaxPending) return fail(HM_ERR_BUSY, "hm_submit: too many requests in flight");
    Req *r = new (std::nothrow) Req();
    if (!r) return fail(HM_ERR_NOMEM, "hm_submit: allocation failed");
    r->ticket = S->next_ticket++;
    r->mat = mat_id;
    r->W = W;
    r->ldw = ldw;
    r->Y = Y;
    r->ldy = ldy;
    r->Q = Q;
    r->t_submit = now_us();
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
    return st == HM_OK ? HM_OK : fail(st, "hm_poll: the request's sweep failed");
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
    o->inflight = (int32_t)S->inflight.size();
    o->peak_inflight = S->peak_inflight;
    o->peak_bytes = (double)S->peak_bytes;
    return HM_OK;
}

hm_status hm_server_destroy(hm_server S) {
    destroy_server(S);
    return HM_OK;
}

}  // extern "C"
