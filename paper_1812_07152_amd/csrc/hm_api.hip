// hm_api.hip -- the extern "C" entry points declared in include/hm.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "hm_internal.h"

namespace hm {

namespace {
thread_local std::string g_last_error;
}

hm_status fail(hm_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

namespace {

#define HM_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? HM_ERR_NOMEM : HM_ERR_DEVICE,     \
                        std::string(#call ": ") + hipGetErrorString(e_));            \
    } while (0)

struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Grow workspace `b` of element size `es` (slot 0: 8 bytes, 1: 4 bytes) to `bytes`.
hm_status ensure_ws(hm_matrix h, int slot, int b, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (h->ws_bytes[slot][b] >= bytes) return HM_OK;
    if (h->ws[slot][b]) {
        HM_HIP(hipDeviceSynchronize());
        HM_HIP(hipFree(h->ws[slot][b]));
        h->ws[slot][b] = nullptr;
        h->ws_bytes[slot][b] = 0;
    }
    HM_HIP(hipMalloc(&h->ws[slot][b], bytes));
    h->ws_bytes[slot][b] = bytes;
    return HM_OK;
}

// Grow split workspace `b` (see Split16) to `bytes`, zero-filled: rows past a
// node's last row are read as zeros by the split-BF16 products.
hm_status ensure_ws16(hm_matrix h, int b, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (h->ws16_bytes[b] >= bytes) return HM_OK;
    if (h->ws16[b]) {
        HM_HIP(hipDeviceSynchronize());
        HM_HIP(hipFree(h->ws16[b]));
        h->ws16[b] = nullptr;
        h->ws16_bytes[b] = 0;
    }
    HM_HIP(hipMalloc(&h->ws16[b], bytes));
    HM_HIP(hipMemset(h->ws16[b], 0, bytes));
    HM_HIP(hipDeviceSynchronize());  // the fill is done before work on any stream reads the buffer
    h->ws16_bytes[b] = bytes;
    return HM_OK;
}

}  // namespace

hm_status reserve_ws(hm_matrix h, int slot, int64_t ldq) {
    const int es = slot == 0 ? 8 : 4;
    const size_t rows[BUF_COUNT] = {(size_t)h->N, (size_t)h->N, (size_t)h->skel_rows,
                                    (size_t)h->skel_rows};
    for (int b = 0; b < BUF_COUNT; b++) {
        hm_status st = ensure_ws(h, slot, b, rows[b] * (size_t)ldq * es);
        if (st != HM_OK) return st;
    }
    return HM_OK;
}

namespace {

// Phase group of a Phase.kind for profiling: 1 up, 2 down, 3 leaf.
int group_of(int kind) { return kind; }

hm_status record(hm_matrix h, int group, hipStream_t s, hipEvent_t *ev) {
    HM_HIP(hipEventCreate(ev));
    HM_HIP(hipEventRecord(*ev, s));
    (void)h;
    (void)group;
    return HM_OK;
}

}  // namespace

hm_status eval_setup(const char *who, hm_matrix h, const void *W, int64_t ldw, void *Y, int64_t ldy, int64_t Q,
                     hm_dtype dtype, hm_prec prec, unsigned flags, EvalSetup &o) {
    const std::string w = std::string(who) + ": ";
    if (!h) return fail(HM_ERR_INVALID, w + "matrix handle is NULL");
    if (Q < 0) return fail(HM_ERR_INVALID, w + "Q < 0");
    if (Q == 0) return HM_OK;
    if (!W || !Y) return fail(HM_ERR_INVALID, w + "W or Y is NULL");
    if (ldw < Q || ldy < Q) return fail(HM_ERR_INVALID, w + "leading dimension < Q");
    if (flags & ~(HM_TREE_ORDER | HM_PROFILE | HM_NEAR_FROM_POINTS | HM_FAR_FROM_POINTS | HM_LEVEL_LAUNCHES))
        return fail(HM_ERR_INVALID, w + "unknown flags");
    if (!((dtype == HM_F64 && prec == HM_PREC_FP64) || (dtype == HM_F32 && prec == HM_PREC_FP32) ||
          (dtype == HM_F64 && prec == HM_PREC_BF16X3)))
        return fail(HM_ERR_INVALID, w + "dtype and precision do not match");
    o.mixed = prec == HM_PREC_BF16X3;
    if (o.mixed ? !(h->store16 && h->prec[HM_PREC_FP64].blocks) : !h->prec[prec].blocks)
        return fail(HM_ERR_INVALID, w + "precision was not loaded");
    if (Q > (int64_t)1 << 24) return fail(HM_ERR_INVALID, w + "Q too large");
    o.es = dtype == HM_F64 ? 8 : 4;
    o.slot = dtype == HM_F64 ? 0 : 1;
    if (o.mixed && (flags & HM_LEVEL_LAUNCHES))
        return fail(HM_ERR_INVALID, w + "HM_PREC_BF16X3 runs on the task-graph launch only");
    o.level_sched = (flags & HM_LEVEL_LAUNCHES) != 0;
    o.near_pts = (flags & HM_NEAR_FROM_POINTS) != 0;
    o.far_pts = (flags & HM_FAR_FROM_POINTS) != 0;
    o.from_points = o.near_pts || o.far_pts;
    if (!o.near_pts && !h->near_stored)
        return fail(HM_ERR_INVALID, w + "the near blocks were not loaded (use HM_NEAR_FROM_POINTS)");
    if (!o.far_pts && !h->far_stored)
        return fail(HM_ERR_INVALID, w + "the far blocks were not loaded (use HM_FAR_FROM_POINTS)");
    if (o.from_points && (prec != HM_PREC_FP64 || !h->d_pts || o.level_sched))
        return fail(HM_ERR_INVALID, w + "HM_NEAR_FROM_POINTS and HM_FAR_FROM_POINTS need HM_PREC_FP64, "
                                        "points set with hm_set_points and the task-graph launch");
    if (o.far_pts && !h->d_skel_pts)
        return fail(HM_ERR_INVALID, w + "HM_FAR_FROM_POINTS needs a representation loaded with its skeletons");
    int *bk = o.bn_kind;
    bk[0] = 0;
    bk[1] = pick_bn(Q, 1);
    bk[2] = pick_bn(Q, 2);
    bk[3] = pick_bn(Q, 3);
    if (!o.level_sched) bk[1] = bk[2] = bk[3] = graph_bn(Q, o.es, o.mixed, h->task_k);  // one tile for the graph
    if (o.from_points && bk[3] == 64) bk[1] = bk[2] = bk[3] = 128;  // see k_persistent
    const int bn_max = std::max({bk[1], bk[2], bk[3]});
    // a 256-column stored-block task graph in the launch's type (not the
    // split-BF16, points or symmetric-store launches, nor per-level launches)
    // ends a matrix's columns with a tile no wider than they need
    o.narrow = !o.level_sched && !o.mixed && !o.from_points && !h->symmetric && bk[3] == 256;
    o.Qp = padded_columns(Q, bn_max, o.narrow);
    o.perm = (flags & HM_TREE_ORDER) ? nullptr : h->d_perm;
    o.valid = true;
    return HM_OK;
}

}  // namespace hm

using namespace hm;

extern "C" {

const char *hm_last_error(void) { return g_last_error.c_str(); }

hm_status hm_load_compressed(const char *path, int device, unsigned prec_mask, hm_matrix *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_load_compressed: out is NULL");
    *out = nullptr;
    if (!(prec_mask & (HM_PRECBIT(HM_PREC_FP64) | HM_PRECBIT(HM_PREC_FP32) | HM_PRECBIT(HM_PREC_BF16X3))))
        return fail(HM_ERR_INVALID, "hm_load_compressed: prec_mask selects no precision");
    if ((prec_mask & (HM_LOAD_NO_NEAR_BLOCKS | HM_LOAD_NO_FAR_BLOCKS)) &&
        (!(prec_mask & HM_PRECBIT(HM_PREC_FP64)) ||
         (prec_mask & (HM_PRECBIT(HM_PREC_FP32) | HM_PRECBIT(HM_PREC_BF16X3)))))
        return fail(HM_ERR_INVALID, "hm_load_compressed: HM_LOAD_NO_NEAR_BLOCKS and HM_LOAD_NO_FAR_BLOCKS are for "
                                    "the FP64 store alone");
    HostRepr r;
    hm_status st = read_file(path, r);
    if (st != HM_OK) return st;
    if ((prec_mask & HM_LOAD_NO_FAR_BLOCKS) && r.skel_ptr.empty())
        return fail(HM_ERR_INVALID, "hm_load_compressed: HM_LOAD_NO_FAR_BLOCKS needs the skeletons");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(HM_ERR_INVALID, "hm_load_compressed: no such HIP device");
    return build_matrix(r, device, prec_mask, out);
}

hm_status hm_load_compressed_mem(const hm_host_repr *repr, int device, unsigned prec_mask,
                                 hm_matrix *out) {
    if (!out) return fail(HM_ERR_INVALID, "hm_load_compressed_mem: out is NULL");
    *out = nullptr;
    if (!repr) return fail(HM_ERR_INVALID, "hm_load_compressed_mem: repr is NULL");
    if (!(prec_mask & (HM_PRECBIT(HM_PREC_FP64) | HM_PRECBIT(HM_PREC_FP32) | HM_PRECBIT(HM_PREC_BF16X3))))
        return fail(HM_ERR_INVALID, "hm_load_compressed_mem: prec_mask selects no precision");
    if ((prec_mask & (HM_LOAD_NO_NEAR_BLOCKS | HM_LOAD_NO_FAR_BLOCKS)) &&
        (!(prec_mask & HM_PRECBIT(HM_PREC_FP64)) ||
         (prec_mask & (HM_PRECBIT(HM_PREC_FP32) | HM_PRECBIT(HM_PREC_BF16X3)))))
        return fail(HM_ERR_INVALID, "hm_load_compressed_mem: HM_LOAD_NO_NEAR_BLOCKS and HM_LOAD_NO_FAR_BLOCKS are for "
                                    "the FP64 store alone");
    HostRepr r;
    hm_status st = from_view(*repr, r);
    if (st != HM_OK) return st;
    if ((prec_mask & HM_LOAD_NO_FAR_BLOCKS) && r.skel_ptr.empty())
        return fail(HM_ERR_INVALID, "hm_load_compressed_mem: HM_LOAD_NO_FAR_BLOCKS needs the skeletons");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(HM_ERR_INVALID, "hm_load_compressed_mem: no such HIP device");
    return build_matrix(r, device, prec_mask, out);
}

hm_status hm_info(hm_matrix h, hm_info_t *o) {
    if (!h || !o) return fail(HM_ERR_INVALID, "hm_info: NULL argument");
    o->N = h->N;
    o->n_nodes = h->n_nodes;
    o->depth = h->depth;
    o->max_rank = h->max_rank;
    o->device = h->device;
    o->n_far = h->n_far;
    o->n_near = h->n_near;
    o->E_V = h->E_V;
    o->E_T = h->E_T;
    o->E_B = h->E_B;
    o->E_D = h->E_D;
    o->flops_per_col = 2.0 * (2.0 * h->E_V + 2.0 * h->E_T + (double)h->E_B + (double)h->E_D);
    o->bytes_fp64 = (double)h->prec[HM_PREC_FP64].bytes;
    o->bytes_fp32 = (double)h->prec[HM_PREC_FP32].bytes;
    o->bytes_bf16x3 = (double)h->store16_bytes;
    o->n_phases = (int32_t)h->phases.size();
    return HM_OK;
}

hm_status hm_free(hm_matrix h) {
    if (!h) return HM_OK;
    DeviceScope ds(h->device);
    for (int i = 0; i < 2; i++)
        if (h->prec[i].blocks) (void)hipFree(h->prec[i].blocks);
    if (h->store16) (void)hipFree(h->store16);
    for (int b = 0; b < BUF_COUNT; b++)
        if (h->ws16[b]) (void)hipFree(h->ws16[b]);
    if (h->d_wchunks) (void)hipFree(h->d_wchunks);
    for (int s = 0; s < 2; s++)
        for (int b = 0; b < BUF_COUNT; b++)
            if (h->ws[s][b]) (void)hipFree(h->ws[s][b]);
    if (h->d_perm) (void)hipFree(h->d_perm);
    for (int k = 0; k < 2; k++)
        for (GraphPlan &p : h->plans[k]) free_plan(p);
    if (h->d_mat) (void)hipFree(h->d_mat);
    if (h->d_head) (void)hipFree(h->d_head);
    if (h->d_tasks) (void)hipFree(h->d_tasks);
    if (h->d_segs) (void)hipFree(h->d_segs);
    if (h->d_pts) (void)hipFree(h->d_pts);
    if (h->d_skel_pts) (void)hipFree(h->d_skel_pts);
    for (int g = 0; g < 5; g++)
        for (auto &pr : h->prof.pending[g]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    delete h;
    return HM_OK;
}

hm_status hm_eval(hm_matrix h, const void *W, int64_t ldw, void *Y, int64_t ldy, int64_t Q,
                  hm_dtype dtype, hm_prec prec, unsigned flags, void *stream) {
    EvalSetup e;
    {
        hm_status vst = eval_setup("hm_eval", h, W, ldw, Y, ldy, Q, dtype, prec, flags, e);
        if (vst != HM_OK || !e.valid) return vst;  // Q = 0: nothing to do
    }
    DeviceScope ds(h->device);
    if (ds.err != hipSuccess) return fail(HM_ERR_DEVICE, "hm_eval: cannot select the device");
    hipStream_t s = (hipStream_t)stream;
    const int es = e.es, slot = e.slot;
    const bool mixed = e.mixed, level_sched = e.level_sched, near_pts = e.near_pts, far_pts = e.far_pts,
               from_points = e.from_points;
    const int *bn_kind = e.bn_kind;
    const int64_t Qp = e.Qp;
    {
        hm_status st = reserve_ws(h, slot, Qp);
        // split workspaces: W (leaf rows), Ŵ and Ŷ (skeleton rows), 4 bytes a value
        if (st == HM_OK && mixed) st = ensure_ws16(h, BUF_WT, (size_t)h->rows16_w * Qp * 4);
        if (st == HM_OK && mixed) st = ensure_ws16(h, BUF_WHAT, (size_t)h->rows16_h * Qp * 4);
        if (st == HM_OK && mixed) st = ensure_ws16(h, BUF_YHAT, (size_t)h->rows16_h * Qp * 4);
        if (st != HM_OK) return st;
    }
    void *bufs[BUF_COUNT];
    for (int b = 0; b < BUF_COUNT; b++) bufs[b] = h->ws[slot][b];
    const bool prof = (flags & HM_PROFILE) != 0;
    const int64_t *perm = e.perm;

    int grid = 0;
    GraphPlan *plan = nullptr;
    if (!level_sched) {
        const int workers =
            std::max(1, persistent_occupancy(es, bn_kind[3], mixed, h->symmetric, e.narrow && Qp % bn_kind[3] != 0) *
                            h->n_cu);
        hm_status pst = get_plan(h, slot, bn_kind[3], Qp, workers, &plan, mixed ? 1 : 0);
        if (pst != HM_OK) return pst;
        MatDesc md{h->prec[mixed ? HM_PREC_FP64 : prec].blocks, {bufs[0], bufs[1], bufs[2], bufs[3]},
                   Qp, h->d_segs, mixed ? h->store16 : nullptr,
                   {mixed ? h->ws16[BUF_WT] : nullptr, nullptr, mixed ? h->ws16[BUF_WHAT] : nullptr,
                    mixed ? h->ws16[BUF_YHAT] : nullptr},
                   near_pts ? h->d_pts : nullptr, far_pts ? h->d_skel_pts : nullptr, h->pts_d, h->pts_kern,
                   h->pts_scale};
        MatDesc &cache = h->mat_cache[slot];
        if (std::memcmp(&md, &cache, sizeof(MatDesc)) != 0 || h->mat_slot != slot) {
            HM_HIP(hipStreamSynchronize(s));
            HM_HIP(hipMemcpy(h->d_mat, &md, sizeof(MatDesc), hipMemcpyHostToDevice));
            cache = md;
            h->mat_slot = slot;
        }
        grid = std::min(plan->n_tasks, workers);
    }

    auto mark = [&](int group, bool begin) -> hm_status {
        if (!prof) return HM_OK;
        hipEvent_t ev;
        hm_status st = record(h, group, s, &ev);
        if (st != HM_OK) return st;
        if (begin)
            h->prof.pending[group].push_back({ev, nullptr});
        else
            h->prof.pending[group].back().second = ev;
        return HM_OK;
    };
    hm_status st;
    if ((st = mark(0, true)) != HM_OK) return st;
    if (mixed)  // only split-BF16 products read W in the mixed-precision graph
        HM_HIP(launch_permute_in_split((const double *)W, ldw, h->ws16[BUF_WT], Qp, perm, h->d_wchunks,
                                       h->n_wchunks, Q, s));
    else
        HM_HIP(launch_permute_in(W, ldw, bufs[BUF_WT], Qp, perm, h->N, Q, es, s));
    if ((st = mark(0, false)) != HM_OK) return st;
    if (!level_sched) {
        // the whole graph (up, down, near, leaf far part) in one launch,
        // reported as the leaf-pass group; the leaf rows are written straight
        // into Y in the caller's order, so no permute-out follows
        if ((st = mark(3, true)) != HM_OK) return st;
        HM_HIP(launch_persistent(*plan, es, h->d_mat, h->d_head, grid, s, OutScatter{Y, ldy, Q, perm, from_points}));
        if ((st = mark(3, false)) != HM_OK) return st;
        return HM_OK;
    } else {
        int open_group = -1;
        for (const Phase &ph : h->phases) {
            int g = group_of(ph.kind);
            if (g != open_group) {
                if (open_group >= 0 && (st = mark(open_group, false)) != HM_OK) return st;
                if ((st = mark(g, true)) != HM_OK) return st;
                open_group = g;
            }
            HM_HIP(launch_phase(h, ph, es, bn_kind[ph.kind], Qp, bufs, s));
        }
        if (open_group >= 0 && (st = mark(open_group, false)) != HM_OK) return st;
    }
    if ((st = mark(4, true)) != HM_OK) return st;
    HM_HIP(launch_permute_out(bufs[BUF_YT], Qp, Y, ldy, perm, h->N, Q, es, s));
    if ((st = mark(4, false)) != HM_OK) return st;
    return HM_OK;
}

hm_status hm_set_points(hm_matrix h, const double *X, int64_t ldx, int64_t d, int kernel, double h_param) {
    if (!h || !X) return fail(HM_ERR_INVALID, "hm_set_points: NULL argument");
    if (d < 1 || d > kMaxPointDimAny) return fail(HM_ERR_INVALID, "hm_set_points: d must be in [1, 64]");
    if (ldx < d) return fail(HM_ERR_INVALID, "hm_set_points: ldx < d");
    if (kernel != 0 && kernel != 1) return fail(HM_ERR_INVALID, "hm_set_points: unknown kernel");
    if (!(h_param > 0.0) || !std::isfinite(h_param)) return fail(HM_ERR_INVALID, "hm_set_points: h must be > 0");
    // the points must be those the representation was compressed from: its
    // metadata names d, the kernel and h (a representation that states none
    // cannot be checked)
    if (h->repr_d > 0 && d != h->repr_d)
        return fail(HM_ERR_INVALID, "hm_set_points: d differs from the representation's");
    if (h->repr_h > 0 && (kernel != h->repr_kernel || std::fabs(h_param - h->repr_h) > 1e-12 * h->repr_h))
        return fail(HM_ERR_INVALID, "hm_set_points: kernel or h differs from the representation's");
    DeviceScope ds(h->device);
    if (ds.err != hipSuccess) return fail(HM_ERR_DEVICE, "hm_set_points: cannot select the device");
    // tree order: row t holds the point perm[t]
    std::vector<int64_t> perm((size_t)h->N);
    HM_HIP(hipMemcpy(perm.data(), h->d_perm, sizeof(int64_t) * (size_t)h->N, hipMemcpyDeviceToHost));
    std::vector<double> xt((size_t)h->N * (size_t)d);
    for (int64_t t = 0; t < h->N; t++)
        for (int64_t c = 0; c < d; c++) xt[(size_t)(t * d + c)] = X[perm[(size_t)t] * ldx + c];
    std::vector<double> xs;  // skeleton points in Ŵ row order (for HM_FAR_FROM_POINTS)
    if (!h->skel_row_pt.empty()) {
        xs.resize(h->skel_row_pt.size() * (size_t)d);
        for (size_t t = 0; t < h->skel_row_pt.size(); t++)
            for (int64_t c = 0; c < d; c++) xs[t * (size_t)d + (size_t)c] = X[h->skel_row_pt[t] * ldx + c];
    }
    // build the new buffers first; the matrix keeps its old points (and
    // their d, kernel and scale) unless every step succeeds
    struct Owned {
        double *p = nullptr;
        ~Owned() {
            if (p) (void)hipFree(p);
        }
    } np_, ns_;
    HM_HIP(hipMalloc(&np_.p, sizeof(double) * xt.size()));
    HM_HIP(hipMemcpy(np_.p, xt.data(), sizeof(double) * xt.size(), hipMemcpyHostToDevice));
    if (!xs.empty()) {
        HM_HIP(hipMalloc(&ns_.p, sizeof(double) * xs.size()));
        HM_HIP(hipMemcpy(ns_.p, xs.data(), sizeof(double) * xs.size(), hipMemcpyHostToDevice));
    }
    HM_HIP(hipDeviceSynchronize());  // no evaluation may still read the old points
    std::swap(h->d_pts, np_.p);       // the old buffers are freed by the guards
    std::swap(h->d_skel_pts, ns_.p);
    h->pts_d = (int32_t)d;
    h->pts_kern = kernel;
    h->pts_scale = kernel == 0 ? 1.0 / (2.0 * h_param * h_param) : 1.0 / h_param;
    return HM_OK;
}

hm_status hm_check(hm_matrix h) {
    if (!h) return fail(HM_ERR_INVALID, "hm_check: NULL argument");
    DeviceScope ds(h->device);
    HM_HIP(hipDeviceSynchronize());
    int32_t err = 0;
    HM_HIP(hipMemcpy(&err, h->d_head + 1, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (err) {
        const int32_t zero = 0;
        HM_HIP(hipMemcpy(h->d_head + 1, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
        return fail(HM_ERR_INTERNAL, "a dependency wait of the persistent launch timed out; "
                                     "the results of the affected evaluations are invalid");
    }
    return HM_OK;
}

hm_status hm_profile_read(hm_matrix h, double ms[5], int64_t launches[5]) {
    if (!h || !ms || !launches) return fail(HM_ERR_INVALID, "hm_profile_read: NULL argument");
    DeviceScope ds(h->device);
    for (int g = 0; g < 5; g++) {
        for (auto &pr : h->prof.pending[g]) {
            HM_HIP(hipEventSynchronize(pr.second));
            float t = 0.f;
            HM_HIP(hipEventElapsedTime(&t, pr.first, pr.second));
            h->prof.ms[g] += t;
            h->prof.launches[g] += 1;
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        h->prof.pending[g].clear();
        ms[g] = h->prof.ms[g];
        launches[g] = h->prof.launches[g];
    }
    return HM_OK;
}

hm_status hm_profile_reset(hm_matrix h) {
    if (!h) return fail(HM_ERR_INVALID, "hm_profile_reset: NULL argument");
    double ms[5];
    int64_t l[5];
    hm_status st = hm_profile_read(h, ms, l);
    if (st != HM_OK) return st;
    for (int g = 0; g < 5; g++) {
        h->prof.ms[g] = 0;
        h->prof.launches[g] = 0;
    }
    return HM_OK;
}

}  // extern "C"
