// hm_batch.hip -- many compressed matrices of uneven size, rank and width
// evaluated by ONE persistent task-graph launch (their queues merged and list
// scheduled together), with batched permutes, captured once in a HIP graph
// and replayed, and a column tile chosen by timing the candidates.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "hm_internal.h"

namespace hm {
namespace {

#define HM_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? HM_ERR_NOMEM : HM_ERR_DEVICE,     \
                        std::string(#call ": ") + hipGetErrorString(e_));            \
    } while (0)

}  // namespace
}  // namespace hm

struct hm_batch_s {
    int device = 0, n = 0;
    std::vector<hm_matrix> hs;
    std::vector<int64_t> Q, ldq;
    hm_dtype dtype = HM_F64;
    hm_prec prec = HM_PREC_FP64;
    int es = 8, bn = 0, grid = 0;
    hm::GraphPlan plan;
    void *ws = nullptr;              // all workspaces of the batch
    size_t ws_bytes = 0;
    hm::MatDesc *d_mats = nullptr;
    hm::PermDesc *d_perm = nullptr;
    std::vector<hm::PermDesc> h_perm;
    int32_t *d_head = nullptr;       // queue head + error flag
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t exec = nullptr;
    double flops = 0;
    double tuned_ms[5] = {0, 0, 0, 0, 0};  // per candidate tile 16..256 (0 = not tried)
    bool use_graph = true;
};

namespace hm {
namespace {

void release_batch(hm_batch b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    free_plan(b->plan);
    if (b->ws) (void)hipFree(b->ws);
    if (b->d_mats) (void)hipFree(b->d_mats);
    if (b->d_perm) (void)hipFree(b->d_perm);
    if (b->d_head) (void)hipFree(b->d_head);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int bn_index(int bn) { return bn == 16 ? 0 : bn == 32 ? 1 : bn == 64 ? 2 : bn == 128 ? 3 : 4; }

// (Re)build workspaces, descriptors and the merged plan for column tile bn.
hm_status configure(hm_batch b, int bn) {
    if (b->exec) {
        HM_HIP(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
    }
    b->bn = bn;
    b->ldq.resize(b->n);
    bool sym = false;
    for (int i = 0; i < b->n; i++) sym = sym || b->hs[i]->symmetric;
    // with 256-column tiles, each matrix's last columns in a tile no wider
    // than they need (not with symmetric stores, whose launch has no
    // narrow-tile instantiation)
    const bool narrow_tail = !sym && bn == 256;
    bool narrow = false;
    size_t total = 0;
    std::vector<size_t> off(b->n);
    for (int i = 0; i < b->n; i++) {
        b->ldq[i] = padded_columns(b->Q[i], bn, narrow_tail);
        narrow = narrow || b->ldq[i] % bn != 0;
        off[i] = total;
        const size_t rows = 2 * (size_t)b->hs[i]->N + 2 * (size_t)b->hs[i]->skel_rows;
        total += (rows * (size_t)b->ldq[i] * b->es + 255) / 256 * 256;
    }
    total = std::max<size_t>(total, 256);
    if (total > b->ws_bytes) {
        if (b->ws) HM_HIP(hipFree(b->ws));
        b->ws = nullptr;
        b->ws_bytes = 0;
        HM_HIP(hipMalloc(&b->ws, total));
        b->ws_bytes = total;
    }
    HM_HIP(hipMemset(b->ws, 0, total));
    std::vector<MatDesc> mats(b->n);
    b->h_perm.assign(b->n, PermDesc{});
    std::vector<PlanPart> parts;
    for (int i = 0; i < b->n; i++) {
        hm_matrix h = b->hs[i];
        char *base = (char *)b->ws + off[i];
        const size_t nb = (size_t)h->N * b->ldq[i] * b->es, rb = (size_t)h->skel_rows * b->ldq[i] * b->es;
        void *buf[4] = {base, base + nb, base + 2 * nb, base + 2 * nb + rb};
        mats[i] = MatDesc{h->prec[b->prec].blocks, {buf[0], buf[1], buf[2], buf[3]}, b->ldq[i], h->d_segs};
        PermDesc &pd = b->h_perm[i];
        pd.Wt = buf[BUF_WT];
        pd.Yt = buf[BUF_YT];
        pd.ldq = b->ldq[i];
        pd.perm = h->d_perm;
        pd.N = h->N;
        pd.Q = b->Q[i];
        parts.push_back({h, i, b->ldq[i], 0, false});
    }
    HM_HIP(hipMemcpy(b->d_mats, mats.data(), sizeof(MatDesc) * b->n, hipMemcpyHostToDevice));
    const int occ = persistent_occupancy(b->es, bn, false, sym, narrow);
    const int workers = std::max(1, occ * b->hs[0]->n_cu);
    hm_status st = build_plan(parts, bn, b->es, workers, b->plan);
    if (st != HM_OK) return st;
    b->grid = std::min(b->plan.n_tasks, workers);
    return HM_OK;
}

// The device work of one batched evaluation (captured into the graph).
hm_status enqueue(hm_batch b, hipStream_t s) {
    int64_t maxq = 0;
    for (int64_t q : b->ldq) maxq = std::max(maxq, q);
    int64_t maxn = 0;
    for (hm_matrix h : b->hs) maxn = std::max(maxn, h->N);
    HM_HIP(launch_permute_batched(b->d_perm, b->n, maxn * maxq, b->es, true, s));
    HM_HIP(launch_persistent(b->plan, b->es, b->d_mats, b->d_head, b->grid, s));
    HM_HIP(launch_permute_batched(b->d_perm, b->n, maxn * maxq, b->es, false, s));
    return HM_OK;
}

hm_status run(hm_batch b, hipStream_t user) {
    HM_HIP(hipMemcpyAsync(b->d_perm, b->h_perm.data(), sizeof(PermDesc) * b->n,
                          hipMemcpyHostToDevice, b->stream));
    HM_HIP(hipEventRecord(b->ev_in, user));
    HM_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    if (b->use_graph) {
        if (!b->exec) {
            hipGraph_t g = nullptr;
            HM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            hm_status st = enqueue(b, b->stream);
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            if (st != HM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return fail(HM_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(HM_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        HM_HIP(hipGraphLaunch(b->exec, b->stream));
    } else {
        hm_status st = enqueue(b, b->stream);
        if (st != HM_OK) return st;
    }
    HM_HIP(hipEventRecord(b->ev_out, b->stream));
    HM_HIP(hipStreamWaitEvent(user, b->ev_out, 0));
    return HM_OK;
}

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" {

hm_status hm_batch_create(int n, const hm_matrix *hs, const int64_t *Q, hm_dtype dtype,
                          hm_prec prec, unsigned flags, hm_batch *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_batch_create: out is NULL");
    *out = nullptr;
    if (n < 1 || !hs || !Q) return fail(HM_ERR_INVALID, "hm_batch_create: need n >= 1 matrices and widths");
    if (flags & ~(HM_BATCH_AUTOTUNE | HM_BATCH_NO_GRAPH | HM_BATCH_TILE(0x1ff)))
        return fail(HM_ERR_INVALID, "hm_batch_create: unknown flags");
    const int fixed_bn = (int)((flags >> 8) & 0x1ff);
    if (fixed_bn && fixed_bn != 16 && fixed_bn != 32 && fixed_bn != 64 && fixed_bn != 128 && fixed_bn != 256)
        return fail(HM_ERR_INVALID, "hm_batch_create: HM_BATCH_TILE takes 16, 32, 64, 128 or 256");
    if (fixed_bn && (flags & HM_BATCH_AUTOTUNE))
        return fail(HM_ERR_INVALID, "hm_batch_create: HM_BATCH_TILE and HM_BATCH_AUTOTUNE exclude each other");
    if (!((dtype == HM_F64 && prec == HM_PREC_FP64) || (dtype == HM_F32 && prec == HM_PREC_FP32)))
        return fail(HM_ERR_INVALID, "hm_batch_create: dtype and precision do not match");
    int64_t maxq = 0;
    for (int i = 0; i < n; i++) {
        if (!hs[i]) return fail(HM_ERR_INVALID, "hm_batch_create: NULL matrix");
        if (hs[i]->device != hs[0]->device) return fail(HM_ERR_INVALID, "hm_batch_create: matrices on different devices");
        if (!hs[i]->prec[prec].blocks) return fail(HM_ERR_INVALID, "hm_batch_create: precision not loaded for a matrix");
        if (!hs[i]->near_stored || !hs[i]->far_stored)
            return fail(HM_ERR_INVALID, "hm_batch_create: a matrix was loaded without its near or far blocks");
        if (Q[i] < 1 || Q[i] > ((int64_t)1 << 24)) return fail(HM_ERR_INVALID, "hm_batch_create: each Q must be in [1, 2^24]");
        maxq = std::max(maxq, Q[i]);
    }
    hm_batch b = new (std::nothrow) hm_batch_s();
    if (!b) return fail(HM_ERR_NOMEM, "hm_batch_create: allocation failed");
    struct Guard {
        hm_batch b;
        bool keep = false;
        ~Guard() {
            if (!keep) release_batch(b);
        }
    } guard{b};
    b->device = hs[0]->device;
    b->n = n;
    b->hs.assign(hs, hs + n);
    b->Q.assign(Q, Q + n);
    b->dtype = dtype;
    b->prec = prec;
    b->es = dtype == HM_F64 ? 8 : 4;
    b->use_graph = !(flags & HM_BATCH_NO_GRAPH);
    for (int i = 0; i < n; i++) b->flops += hs[i]->E_V * 4.0 * Q[i] + hs[i]->E_T * 4.0 * Q[i] +
                                           (double)hs[i]->E_B * 2.0 * Q[i] + (double)hs[i]->E_D * 2.0 * Q[i];
    HM_HIP(hipSetDevice(b->device));
    HM_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HM_HIP(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    HM_HIP(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    HM_HIP(hipMalloc(&b->d_mats, sizeof(MatDesc) * n));
    HM_HIP(hipMalloc(&b->d_perm, sizeof(PermDesc) * n));
    HM_HIP(hipMalloc(&b->d_head, 2 * sizeof(int32_t)));
    HM_HIP(hipMemset(b->d_head, 0, 2 * sizeof(int32_t)));
    double tk = 0;
    for (int i = 0; i < n; i++) tk = std::max(tk, hs[i]->task_k);
    const int default_bn = fixed_bn ? fixed_bn : graph_bn(maxq, b->es, false, tk);
    if (flags & HM_BATCH_AUTOTUNE) {
        // time every candidate tile on the batch's own (zeroed) workspaces
        hipEvent_t t0, t1;
        HM_HIP(hipEventCreate(&t0));
        HM_HIP(hipEventCreate(&t1));
        double best = 1e30;
        int best_bn = default_bn;
        for (int bn : {32, 64, 128, 256}) {
            if (bn > std::max<int64_t>(32, (maxq + 15) / 16 * 16 * 2)) continue;
            hm_status st = configure(b, bn);
            if (st != HM_OK) return st;
            for (int i = 0; i < n; i++) {  // tuning input: the batch's own zeroed buffers
                b->h_perm[i].W = b->h_perm[i].Yt;
                b->h_perm[i].ldw = b->ldq[i];
                b->h_perm[i].Y = b->h_perm[i].Wt;
                b->h_perm[i].ldy = b->ldq[i];
            }
            st = run(b, b->stream);  // warm-up (and graph capture)
            if (st != HM_OK) return st;
            HM_HIP(hipEventRecord(t0, b->stream));
            for (int rep = 0; rep < 3; rep++)
                if ((st = run(b, b->stream)) != HM_OK) return st;
            HM_HIP(hipEventRecord(t1, b->stream));
            HM_HIP(hipEventSynchronize(t1));
            float ms = 0;
            HM_HIP(hipEventElapsedTime(&ms, t0, t1));
            b->tuned_ms[bn_index(bn)] = ms / 3;
            if (ms / 3 < best) {
                best = ms / 3;
                best_bn = bn;
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        hm_status st = configure(b, best_bn);
        if (st != HM_OK) return st;
    } else {
        hm_status st = configure(b, default_bn);
        if (st != HM_OK) return st;
    }
    HM_HIP(hipStreamSynchronize(b->stream));
    guard.keep = true;
    *out = b;
    return HM_OK;
}

hm_status hm_batch_eval(hm_batch b, const void *const *W, const int64_t *ldw, void *const *Y,
                        const int64_t *ldy, void *stream) {
    if (!b || !W || !ldw || !Y || !ldy) return fail(HM_ERR_INVALID, "hm_batch_eval: NULL argument");
    for (int i = 0; i < b->n; i++) {
        if (!W[i] || !Y[i]) return fail(HM_ERR_INVALID, "hm_batch_eval: NULL W or Y");
        if (ldw[i] < b->Q[i] || ldy[i] < b->Q[i]) return fail(HM_ERR_INVALID, "hm_batch_eval: leading dimension < Q");
        b->h_perm[i].W = W[i];
        b->h_perm[i].ldw = ldw[i];
        b->h_perm[i].Y = Y[i];
        b->h_perm[i].ldy = ldy[i];
    }
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(HM_ERR_DEVICE, "hm_batch_eval: hipGetDevice failed");
    if (prev != b->device && hipSetDevice(b->device) != hipSuccess)
        return fail(HM_ERR_DEVICE, "hm_batch_eval: cannot select the device");
    hm_status st = run(b, (hipStream_t)stream);
    if (prev != b->device) (void)hipSetDevice(prev);
    return st;
}

hm_status hm_batch_info(hm_batch b, hm_batch_info_t *o) {
    if (!b || !o) return fail(HM_ERR_INVALID, "hm_batch_info: NULL argument");
    o->n = b->n;
    o->column_tile = b->bn;
    o->n_tasks = b->plan.n_tasks;
    o->workgroups = b->grid;
    o->flops = b->flops;
    for (int i = 0; i < 5; i++) o->tuned_ms[i] = b->tuned_ms[i];
    o->workspace_bytes = (double)b->ws_bytes;
    return HM_OK;
}

hm_status hm_batch_check(hm_batch b) {
    if (!b) return fail(HM_ERR_INVALID, "hm_batch_check: NULL argument");
    HM_HIP(hipSetDevice(b->device));
    HM_HIP(hipStreamSynchronize(b->stream));
    int32_t err = 0;
    HM_HIP(hipMemcpy(&err, b->d_head + 1, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (err) {
        const int32_t zero = 0;
        HM_HIP(hipMemcpy(b->d_head + 1, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
        return fail(HM_ERR_INTERNAL, "a dependency wait of the batched launch timed out");
    }
    return HM_OK;
}

hm_status hm_batch_free(hm_batch b) {
    release_batch(b);
    return HM_OK;
}

hm_status hm_eval_batched(int n, const hm_matrix *hs, const void *const *W, const int64_t *ldw,
                          void *const *Y, const int64_t *ldy, const int64_t *Q, hm_dtype dtype,
                          hm_prec prec, void *stream) {
    hm_batch b = nullptr;
    hm_status st = hm_batch_create(n, hs, Q, dtype, prec, 0, &b);
    if (st != HM_OK) return st;
    st = hm_batch_eval(b, W, ldw, Y, ldy, stream);
    if (st == HM_OK) st = hm_batch_check(b);  // also waits before the batch is released
    release_batch(b);
    return st;
}

}  // extern "C"
