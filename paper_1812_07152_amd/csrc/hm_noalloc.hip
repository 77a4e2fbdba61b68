// hm_noalloc.hip -- hm_eval_noalloc: the task-graph evaluation of hm_eval
// with its per-call device memory (the workspaces Wt, Ŵ, Ŷ, their split-BF16
// copies, the dependency counters and the matrix descriptor) carved out of
// one fixed array in device memory instead of the matrix's own, grown-on-
// demand workspaces.  The kernels are hm_eval's; only the addresses differ.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "hm_internal.h"

namespace hm {
namespace {

// The fixed device array.  Each device the library runs on holds its own
// copy, at its own address, until the process ends.
constexpr size_t kScratchBytes = (size_t)HM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device (which must be `dev`),
// looked up once per device.  In host code the array's name is only a
// host-side stand-in: every kernel argument and fill below uses this address.
hm_status scratch_address(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HM_ERR_INVALID, "hm_eval_noalloc: device index too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HM_ERR_DEVICE, std::string("hm_eval_noalloc: hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return HM_OK;
}

// Writes the launch's matrix descriptor into device memory from a kernel
// argument: no host copy, and the write is ordered on the stream.
__global__ void k_write_desc(MatDesc *dst, MatDesc v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}

// Zero n 16-byte words (the split workspaces' padding rows and columns are
// read as zeros by the split-BF16 products; a fill kernel rather than a
// memset, so that the sequence may be captured in a graph).
__global__ void k_zero16(uint4 *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = uint4{0u, 0u, 0u, 0u};
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

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

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" {

hm_status hm_eval_noalloc(hm_matrix h, const void *W, int64_t ldw, void *Y, int64_t ldy, int64_t Q,
                          hm_dtype dtype, hm_prec prec, unsigned flags, void *stream) {
    EvalSetup e;
    {
        hm_status vst = eval_setup("hm_eval_noalloc", h, W, ldw, Y, ldy, Q, dtype, prec, flags, e);
        if (vst != HM_OK || !e.valid) return vst;  // Q = 0: nothing to do
    }
    if (flags & (HM_LEVEL_LAUNCHES | HM_PROFILE))
        return fail(HM_ERR_INVALID, "hm_eval_noalloc: HM_LEVEL_LAUNCHES and HM_PROFILE are not available here");
    const int64_t Qp = e.Qp;
    // scratch layout: descriptor, counters, then the workspaces the task
    // graph touches (the leaf outputs go straight to Y: no Yt)
    const size_t es = (size_t)e.es;
    const size_t desc_b = align256(sizeof(MatDesc));
    const size_t wt_b = e.mixed ? 0 : align256((size_t)h->N * Qp * es);
    const size_t hat_b = align256(std::max<size_t>((size_t)h->skel_rows * Qp * es, 1));
    const size_t w16_b = e.mixed ? align256((size_t)h->rows16_w * Qp * 4) : 0;
    const size_t h16_b = e.mixed ? align256((size_t)h->rows16_h * Qp * 4) : 0;
    auto too_big = [&](size_t total) {
        return fail(HM_ERR_INVALID, "hm_eval_noalloc: this evaluation needs " + std::to_string(total) +
                                        " bytes of workspace, more than the fixed " +
                                        std::to_string(kScratchBytes) + " (use hm_eval)");
    };
    const size_t ws_total = desc_b + wt_b + 2 * hat_b + w16_b + 2 * h16_b;
    if (ws_total > kScratchBytes) return too_big(ws_total);
    DeviceScope ds(h->device);
    if (ds.err != hipSuccess) return fail(HM_ERR_DEVICE, "hm_eval_noalloc: cannot select the device");
    const int workers = std::max(
        1, persistent_occupancy(e.es, e.bn_kind[3], e.mixed, h->symmetric, e.narrow && Qp % e.bn_kind[3] != 0) *
               h->n_cu);
    GraphPlan *plan = nullptr;
    {
        hm_status pst = get_plan(h, e.slot, e.bn_kind[3], Qp, workers, &plan, e.mixed ? 1 : 0, false);
        if (pst != HM_OK) return pst;
    }
    const size_t cnt_b = align256((size_t)std::max(plan->n_tasks, 1) * sizeof(int32_t));
    if (ws_total + cnt_b > kScratchBytes) return too_big(ws_total + cnt_b);
    unsigned char *base = nullptr;
    {
        hm_status st = scratch_address(h->device, &base);
        if (st != HM_OK) return st;
    }
    size_t off = 0;
    auto carve = [&](size_t b) -> unsigned char * {
        unsigned char *p = b ? base + off : nullptr;
        off += b;
        return p;
    };
    MatDesc *d_desc = (MatDesc *)carve(desc_b);
    int32_t *d_counters = (int32_t *)carve(cnt_b);
    void *wt = carve(wt_b);
    void *what = carve(hat_b), *yhat = carve(hat_b);
    void *w16 = carve(w16_b), *what16 = carve(h16_b), *yhat16 = carve(h16_b);
    // buf[BUF_YT] is never dereferenced in the task-graph launch (its tiles
    // write the caller's Y); it gets a valid address all the same
    void *yt = e.mixed ? what : wt;
    MatDesc md{h->prec[e.mixed ? HM_PREC_FP64 : prec].blocks, {e.mixed ? nullptr : wt, yt, what, yhat}, Qp,
               h->d_segs, e.mixed ? h->store16 : nullptr, {w16, nullptr, what16, yhat16},
               e.near_pts ? h->d_pts : nullptr, e.far_pts ? h->d_skel_pts : nullptr, h->pts_d, h->pts_kern,
               h->pts_scale};
    hipStream_t s = (hipStream_t)stream;
#define NA_HIP(call)                                                                                    \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return fail(HM_ERR_DEVICE, std::string("hm_eval_noalloc: " #call ": ") + hipGetErrorString(e_)); \
    } while (0)
    hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, s, d_desc, md);
    NA_HIP(hipGetLastError());
    if (e.mixed) {
        // the split workspaces follow each other: one fill for the three
        const int64_t n16 = (int64_t)((w16_b + 2 * h16_b) / 16);
        const int g = (int)std::min<int64_t>((n16 + 255) / 256, 4096);
        hipLaunchKernelGGL(k_zero16, dim3(std::max(g, 1)), dim3(256), 0, s, (uint4 *)w16, n16);
        NA_HIP(hipGetLastError());
        NA_HIP(launch_permute_in_split((const double *)W, ldw, w16, Qp, e.perm, h->d_wchunks, h->n_wchunks, Q, s));
    } else {
        NA_HIP(launch_permute_in(W, ldw, wt, Qp, e.perm, h->N, Q, e.es, s));
    }
    NA_HIP(launch_persistent(*plan, e.es, d_desc, h->d_head, std::min(plan->n_tasks, workers), s,
                             OutScatter{Y, ldy, Q, e.perm, e.from_points}, d_counters));
#undef NA_HIP
    return HM_OK;
}

}  // extern "C"
